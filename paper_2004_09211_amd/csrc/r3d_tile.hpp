// Geometry and launchers of the tile kernels (fp16 histograms, one wavefront
// per 4x4 pixel block).
#pragma once

#include "r3d_internal.hpp"

namespace r3d {

enum { kEngValu = 0, kEngMfma16 = 1, kEngMfma16x2 = 2 };
constexpr int kTileMaxNBP = 5;  // 32-bin blocks spanned by a 32-bin pair of depth tiles

struct TileGeom {
  int o;           // (d_lo - c) mod 32
  int kbA0;        // first 32-bin block of pair 0, floor((d_lo - c) / 32)
  int nbp;         // blocks spanned by the band of one pair
  int npairs;      // ceil(D / 32)
  int ntiles;      // ceil(D / 16)
  int mask_words;  // ceil(ntiles / 32): candidate tiles
  int pair_words;  // ceil(npairs / 32): candidate pairs
  int need_words;  // ceil((npairs + nbp - 1) / 32): blocks read by candidate pairs
  int nkb;         // ceil(T / 32)
  int kb_last;     // last block touched by the pairs
  int nbc;         // 4x4 pixel blocks per block-row
  int nblk;        // 4x4 pixel blocks in the frame
  int lds_a;       // byte offset of the matrix-core A operands
  int lds_share;   // byte offset of the resolve role's shared counts and partial moments
  int lds_fixed;   // bytes shared by the workgroup
  int lds_per_wave, off_trange, off_halo, off_comp, off_ring;  // per-wavefront bytes, offsets
};

// Per-pixel output of the bound pass: the largest cost over the depth grid
// (matrix engines: of the fp16-hi contraction, in its raw units) and the
// photon count K.
typedef float2 TileBound;

// One launch of the tile kernel: resolve one frame (whose bounds are ready)
// and/or compute the bounds of another frame. nr / nb are the workgroups of
// each role (0 = none).
struct TileJob {
  StepIO io;                 // resolved frame: histograms, states, outputs
  const TileBound* rbound;   // its bounds
  int nr;
  const uint16_t* bhist;     // frame whose bounds are computed
  const uint8_t* bfaulty;
  TileBound* bbound;
  int nb;
};

bool tile_geometry(const DevModel& M, int engine, TileGeom& G);
bool tile_supported(const DevModel& M, int engine);
hipError_t launch_tile(const DevModel& M, int engine, const TileJob& job, hipStream_t s);
// workgroups for a bound-only or resolve-only launch of the frame
int tile_workgroups(const DevModel& M);
hipError_t launch_cost_tile(const DevModel& M, int engine, const uint16_t* hist, int npix,
                            float* ell, hipStream_t s);

}  // namespace r3d
