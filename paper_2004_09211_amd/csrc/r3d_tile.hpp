// Geometry and launchers of the tile kernels (fp16 histograms, one wavefront
// per 4x4 pixel block).
#pragma once

#include "r3d_internal.hpp"

namespace r3d {

enum { kEngValu = 0, kEngMfma16 = 1, kEngMfma16x2 = 2 };
constexpr int kTileMaxNBP = 5;  // 32-bin blocks spanned by a 32-bin pair of depth tiles
constexpr int kMaxChunks = 16;  // chunks of pairs of a block shared by a workgroup's wavefronts
#ifndef R3D_TILE_WAVES
#define R3D_TILE_WAVES 4
#endif
constexpr int kTileWaves = R3D_TILE_WAVES;  // wavefronts (4x4 pixel blocks) per workgroup of the
                                            // matrix-core step (4 for the vector-FMA engine)

struct TileGeom {
  int o;           // (d_lo - c) mod 32
  int kbA0;        // first 32-bin block of pair 0, floor((d_lo - c) / 32)
  int nbp;         // blocks spanned by the band of one pair
  int npairs;      // ceil(D / 32)
  int ntiles;      // ceil(D / 16)
  int mask_words;  // ceil(ntiles / 32): candidate tiles
  int pair_words;  // ceil(npairs / 32): candidate pairs
  int nkb;         // ceil(T / 32)
  int kb_last;     // last block touched by the pairs
  int nbc;         // 4x4 pixel blocks per block-row
  int nblk;        // 4x4 pixel blocks in the frame
  int lds_a;       // byte offset of the matrix-core A operands
  int lds_fixed;   // bytes before the four wavefront regions
  int lds_per_wave, off_trange, off_halo, off_comp, off_ring;  // per-wavefront bytes, offsets
  int off_share;   // byte offset of the workgroup's shared chunk region
  int lds_total;   // bytes of LDS of one workgroup
  int chunk;       // pairs per chunk of a shared block
  int nchunks;     // ceil(npairs / chunk) <= kMaxChunks
  int waves;       // wavefronts per workgroup of the step
  int lda_band;    // minimum-divergence kernels: offset of a band's A operands in its region
};

// Minimum-divergence estimates: up to kMaxBands bands sharing the frame, T,
// the depth grid and beta, each with its own IRF (its own model).
constexpr int kMaxBands = 4;
struct MindivArgs {
  DevModel M[kMaxBands];
  TileGeom G[kMaxBands];
  const uint16_t* hist[kMaxBands];
  int nb;        // bands
  int lds_band;  // LDS bytes per band (IRF staging and A operands)
  int32_t* argmax;
  float* value;
};
hipError_t launch_mindiv(const DevModel* M, const uint16_t* const* hist, int nb, int engine,
                         bool msl, int32_t* argmax, float* value, hipStream_t s);

bool tile_geometry(const DevModel& M, int engine, TileGeom& G);
bool tile_supported(const DevModel& M, int engine);
hipError_t launch_step_tile(const DevModel& M, int engine, const StepIO& io, hipStream_t s);
hipError_t launch_cost_tile(const DevModel& M, int engine, const uint16_t* hist, int npix,
                            float* ell, hipStream_t s);

}  // namespace r3d
