// Internal declarations shared by the kernels and the C ABI of libr3d.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "r3d.h"

namespace r3d {

constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kLn2 = 0.69314718055994530942f;
constexpr float kLog2TwoPi = 2.65149612947231879804f;  // log2(2*pi)
constexpr int kMaxW = 256;
constexpr float kMaxFp16Count = 2048.0f;  // largest count fp16 holds exactly with all below

// error bits of the device error word
enum : unsigned { kErrRange = 1u, kErrOverflow = 2u, kErrTimeout = 4u, kErrIrf = 8u };

// Model in the form the kernels use; passed by value as a kernel argument.
// Log-quantities are in base 2 (the hardware exp/log are base 2).
struct DevModel {
  int rows, cols, P, T, d_lo, D, W, c;
  float beta;        // beta-divergence parameter
  double beta_d;     // the same in double (IRF powers are taken in double)
  float scale2;      // (beta+1)/beta * log2(e): cost in log2 units
  float hmax;        // an upper bound of max_j irf^beta[j] (for the culling bound)
  float m_flat;      // (d_min+d_max)/2
  float v_flat;      // (d_max-d_min)^2/12
  float sigma_rw2;   // random-walk variance
  float nu[9];       // stencil weights
  float lognu2[9];   // log2(nu), -inf where nu == 0
  const float* h;    // irf^beta, fp32 [W]
  const float* irf;  // irf, fp32 [W]
  const _Float16* h16hi;  // fp16(irf^beta) [W]
  const _Float16* h16lo;  // fp16((irf^beta - hi) * 2048) [W]
  unsigned* err;     // device error word
  int lds_max;       // bytes of LDS a workgroup may use on this device
};

// Per-step pointers (device memory, caller-owned).
struct StepIO {
  const int32_t* row_ptr;
  const int16_t* toa;
  const uint16_t* hist;
  const float* pi_in;
  const uint8_t* faulty;
  const float *pm, *pv, *ppi, *pb;  // previous state
  float *nm, *nv, *npi, *nb;        // next state
  float *depth, *var, *intensity, *background, *pi0_next;
  int32_t* argmax;
  float* lognorm;  // photon-list step only: log2 of the posterior's normaliser on the grid, or null
};

// launchers (one translation unit each)
hipError_t launch_prepare_irf(const double* irf_dev, int W, double beta, float* h, float* irf,
                              _Float16* hi, _Float16* lo, double* hmax, hipStream_t s);
hipError_t launch_state_init(const DevModel& m, float* sm, float* sv, float* spi, float* sb,
                             hipStream_t s);
hipError_t launch_histogram(const DevModel& m, const int32_t* row_ptr, const int16_t* toa,
                            uint16_t* hist, hipStream_t s);
hipError_t launch_cost_plain(const DevModel& m, const uint16_t* hist, int npix, float* ell,
                             hipStream_t s);
hipError_t launch_step_plain(const DevModel& m, const StepIO& io, bool from_hist, hipStream_t s);
// the per-pixel step with every pixel's own IRF: irf_pix double [P][W],
// c_pix int32 [P] or null (the model's c)
hipError_t launch_step_pirf(const DevModel& m, const StepIO& io, bool from_hist,
                            const double* irf_pix, const int32_t* c_pix, hipStream_t s);
bool plain_supported(const DevModel& m);
// continuous minimum-divergence depth for a Gaussian IRF of standard
// deviation sigma, from photon lists; value and grid_argmax may be null
hipError_t launch_gauss_mindiv(const DevModel& m, const int32_t* row_ptr, const int16_t* toa,
                               double sigma, float* depth, float* value, int32_t* grid_argmax,
                               hipStream_t s);

}  // namespace r3d
