// Declarations of the reverse-mode (adjoint) kernels of the filter.
#pragma once

#include "r3d_internal.hpp"

namespace r3d {

// Parameter gradient layout (also the per-block partial layout):
// [0] beta, [1] sigma_rw2, [2..10] nu[0..8], [11..11+W) irf taps.
constexpr int kThetaFixed = 11;

// Per-frame inputs and outputs of the adjoint kernel (device memory).
struct AdjIO {
  const int32_t* row_ptr;  // photon lists of the frame
  const int16_t* toa;
  const uint8_t* faulty;   // [P] or null
  const float *pm, *pv, *ppi;  // state before the frame
  const float *mean, *var;     // [P] the frame's posterior mean and variance (the state after it)
  const float* lognorm;        // [P] log2 of the frame's posterior normaliser (forward step)
  const float* gm;         // [P] adjoint of the frame's posterior mean
  const float* gv;         // [P] adjoint of the frame's posterior variance, or null
  float* cm;               // [9][P] adjoint of the previous mean of neighbour k of p
  float* cv;               // [9][P] adjoint of the previous variance of neighbour k of p
  float* part;             // [blocks][kThetaFixed + W] per-block parameter partials
};

struct AdjGeom {
  int waves;   // wavefronts per block
  int blocks;  // grid size (fixed for a model: deterministic partial order)
  size_t lds;  // dynamic LDS bytes
};

// Launch shape of the adjoint kernel; waves == 0 when the model does not fit.
AdjGeom adjoint_geometry(const DevModel& M);
hipError_t launch_adjoint(const DevModel& M, const AdjIO& io, const AdjGeom& g, hipStream_t s);
// am[q] = gm_prev[q] + sum over the pixels p that have q as neighbour k of cm[k][p] (same for v)
hipError_t launch_adjoint_gather(const DevModel& M, const float* cm, const float* cv,
                                 const float* gm_prev, const float* gv_prev, float* am, float* av,
                                 hipStream_t s);
// grad[i] += sum over blocks of part[b][i] (irf entries scaled by the
// derivative of irf^beta), in double, in block order
hipError_t launch_theta_reduce(const DevModel& M, const float* part, int blocks, double* grad,
                               hipStream_t s);
hipError_t launch_fill_f32(float* x, size_t n, float v, hipStream_t s);
hipError_t launch_fill_f64(double* x, size_t n, double v, hipStream_t s);

}  // namespace r3d
