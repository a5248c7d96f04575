// Geometry of the tile kernels (one wavefront per 4x4 pixel block).
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
  int mask_words;  // ceil(ntiles / 32)
  int nkb;         // ceil(T / 32)
  int kb_last;     // last block touched by the pairs
  int nbc;         // 4x4 pixel blocks per block-row
  int nblk;        // 4x4 pixel blocks in the frame
  int lds_fixed, mask_bytes, halo_bytes, ring_bytes, lds_per_wave;
};

bool tile_geometry(const DevModel& M, int engine, TileGeom& G);
bool tile_supported(const DevModel& M, int engine);
hipError_t launch_step_tile(const DevModel& M, int engine, const StepIO& io, hipStream_t s);
hipError_t launch_cost_tile(const DevModel& M, int engine, const uint16_t* hist, int npix,
                            float* ell, hipStream_t s);

}  // namespace r3d
