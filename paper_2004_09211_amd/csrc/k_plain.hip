// Plain fp32 kernels: IRF preparation, state initialisation, photon
// histogramming (a1), the cost alone (a3) and the fused per-frame step
// (a1..a7) with one wavefront per pixel.
//
// The fused step (pixel_step, r3d_pixel.hpp) keeps the pixel's histogram in
// LDS, evaluates the cost and the prior only on candidate depths, and
// reduces argmax and moments over the wavefront.
#include <cmath>

#include "r3d_device.hpp"
#include "r3d_pixel.hpp"

namespace r3d {

// a2: h = irf^beta (Sec. II-B), also split into fp16 high and scaled low
// parts for the matrix-core contraction: h ~ hi + lo / 2048.
// irf^beta of one tap (the shared IRF and the per-pixel ones alike)
__device__ __forceinline__ double irf_pow(double x, double beta) { return x > 0.0 ? pow(x, beta) : 0.0; }

__global__ void k_prepare_irf(const double* __restrict__ irf, int W, double beta,
                              float* __restrict__ h, float* __restrict__ irf32,
                              _Float16* __restrict__ hi, _Float16* __restrict__ lo,
                              double* __restrict__ hmax) {
  __shared__ double mx[256];
  double m = 0.0;
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    const double x = irf[j];
    const double hv = irf_pow(x, beta);
    h[j] = (float)hv;
    irf32[j] = (float)x;
    const _Float16 a = (_Float16)hv;
    hi[j] = a;
    lo[j] = (_Float16)((hv - (double)a) * 2048.0);
    m = fmax(m, hv);
  }
  mx[threadIdx.x] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)blockDim.x; ++i) m = fmax(m, mx[i]);
    *hmax = m;
  }
}

hipError_t launch_prepare_irf(const double* irf_dev, int W, double beta, float* h, float* irf,
                              _Float16* hi, _Float16* lo, double* hmax, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare_irf, dim3(1), dim3(256), 0, s, irf_dev, W, beta, h, irf, hi, lo, hmax);
  return hipGetLastError();
}

__global__ void k_state_init(int P, float m, float v, float* __restrict__ sm,
                             float* __restrict__ sv, float* __restrict__ spi,
                             float* __restrict__ sb) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
    sm[p] = m;
    sv[p] = v;
    spi[p] = 0.5f;
    sb[p] = 0.f;
  }
}

hipError_t launch_state_init(const DevModel& M, float* sm, float* sv, float* spi, float* sb,
                             hipStream_t s) {
  const int blocks = (M.P + 255) / 256 < 4096 ? (M.P + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_state_init, dim3(blocks), dim3(256), 0, s, M.P, M.m_flat, M.v_flat, sm,
                     sv, spi, sb);
  return hipGetLastError();
}

// waves per block so that nw * per_wave_bytes + fixed_bytes fits in 64 KiB
static int waves_for(size_t per_wave_bytes, size_t fixed_bytes) {
  const size_t cap = 65536;
  if (per_wave_bytes + fixed_bytes > cap) return 0;
  size_t nw = (cap - fixed_bytes) / per_wave_bytes;
  return nw >= 4 ? 4 : (int)nw;
}

// ---------------------------------------------------------------- a1
// One wavefront per pixel: integer LDS atomics (order-independent, hence
// bit-exact), then the counts are written as fp16.
__global__ void __launch_bounds__(256) k_histogram(DevModel M, const int32_t* __restrict__ row_ptr,
                                                   const int16_t* __restrict__ toa,
                                                   uint16_t* __restrict__ out) {
  extern __shared__ unsigned smem_u[];
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned* hist = smem_u + wave * M.T;
  const int p = blockIdx.x * nw + wave;
  const bool active = p < M.P;
  for (int t = lane; t < M.T; t += 64) hist[t] = 0u;
  __syncthreads();
  unsigned bad = 0;
  if (active) {
    const int b = row_ptr[p], e = row_ptr[p + 1];
    if (e < b) bad |= kErrRange;
    for (int k = b + lane; k < e; k += 64) {
      const int t = toa[k];
      if ((unsigned)t < (unsigned)M.T)
        atomicAdd(&hist[t], 1u);
      else
        bad |= kErrRange;
    }
  }
  __syncthreads();
  if (active) {
    uint16_t* row = out + (size_t)p * M.T;
    for (int t = lane; t < M.T; t += 64) {
      const unsigned n = hist[t];
      if (n > 2048u) bad |= kErrOverflow;
      const _Float16 h = (_Float16)(float)n;
      uint16_t bits;
      __builtin_memcpy(&bits, &h, 2);
      row[t] = bits;
    }
  }
  if (bad) atomicOr(M.err, bad);
}

hipError_t launch_histogram(const DevModel& M, const int32_t* row_ptr, const int16_t* toa,
                            uint16_t* hist, hipStream_t s) {
  const int nw = waves_for((size_t)M.T * 4, 0);
  if (nw == 0) return hipErrorInvalidValue;
  const dim3 grid((M.P + nw - 1) / nw);
  hipLaunchKernelGGL(k_histogram, grid, dim3(64 * nw), (size_t)nw * M.T * 4, s, M, row_ptr, toa,
                     hist);
  return hipGetLastError();
}

// Load an fp16 histogram row into LDS as integers; returns the photon count
// K (sum over the wavefront) and flags counts that are negative, above 2048
// or fractional.
__device__ __forceinline__ float load_hist_row(const DevModel& M, const uint16_t* __restrict__ row,
                                               unsigned* hist, int lane, unsigned& bad) {
  float ks = 0.f;
  for (int t = lane; t < M.T; t += 64) {
    const float x = half_bits_to_float(row[t]);
    const bool ok = fp16_count_ok(row[t]);
    if (!ok) bad |= kErrOverflow;
    const float xc = ok ? x : 0.f;
    hist[t] = (unsigned)xc;
    ks += xc;
  }
  return group_sum<1, 32>(ks);
}

// cost at grid point d from the LDS histogram: sum_j h[j] z[d - c + j]
__device__ __forceinline__ float cost_at(const DevModel& M, const float* sh_h,
                                         const unsigned* hist, int d) {
  const int t0 = d - M.c;
  const int jlo = t0 < 0 ? -t0 : 0;
  const int jhi = (M.T - t0) < M.W ? (M.T - t0) : M.W;
  float ell = 0.f;
  for (int j = jlo; j < jhi; ++j) ell = fmaf(sh_h[j], (float)hist[t0 + j], ell);
  return ell;
}

// ---------------------------------------------------------------- a3 alone
__global__ void __launch_bounds__(256) k_cost_plain(DevModel M, const uint16_t* __restrict__ hist_in,
                                                    int npix, float* __restrict__ ell_out) {
  extern __shared__ float smem_f[];
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* sh_h = smem_f;
  unsigned* hist = reinterpret_cast<unsigned*>(smem_f + M.W) + wave * M.T;
  const int p = blockIdx.x * nw + wave;
  for (int i = threadIdx.x; i < M.W; i += blockDim.x) sh_h[i] = M.h[i];
  unsigned bad = 0;
  if (p < npix) load_hist_row(M, hist_in + (size_t)p * M.T, hist, lane, bad);
  __syncthreads();
  if (bad) atomicOr(M.err, bad);
  if (p >= npix) return;
  const float scale = M.scale2 * kLn2;
  for (int i = lane; i < M.D; i += 64)
    ell_out[(size_t)p * M.D + i] = scale * cost_at(M, sh_h, hist, M.d_lo + i);
}

hipError_t launch_cost_plain(const DevModel& M, const uint16_t* hist, int npix, float* ell,
                             hipStream_t s) {
  const int nw = waves_for((size_t)M.T * 4, (size_t)M.W * 4);
  if (nw == 0) return hipErrorInvalidValue;
  const dim3 grid((npix + nw - 1) / nw);
  hipLaunchKernelGGL(k_cost_plain, grid, dim3(64 * nw), (size_t)M.W * 4 + (size_t)nw * M.T * 4, s,
                     M, hist, npix, ell);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a1..a7
// One wavefront per pixel (pixel_step): photon lists, or histograms whose
// length the tile kernels do not take.
template <bool kHist>
__global__ void __launch_bounds__(256) k_step_plain(DevModel M, StepIO io) {
  extern __shared__ __align__(16) float smem_f[];
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* sh_h = smem_f;
  float* sh_irf = smem_f + M.W;
  unsigned* hist = reinterpret_cast<unsigned*>(smem_f + ((2 * M.W + 3) & ~3)) +
                   (size_t)wave * pixel_lds_words(M.T);
  for (int i = threadIdx.x; i < M.W; i += blockDim.x) {
    sh_h[i] = M.h[i];
    sh_irf[i] = M.irf[i];
  }
  __syncthreads();
  const int p = blockIdx.x * nw + wave;
  if (p >= M.P) return;
  pixel_step<kHist>(M, io, p, lane, hist, sh_h, sh_irf);
}

// One wavefront per pixel with the pixel's own IRF (Sec. II-A: the method
// applies when the IRF shape depends on the pixel): the wavefront raises the
// pixel's taps to beta exactly as the shared IRF is prepared (double pow,
// rounded to fp32), bounds its largest power for the candidate range, and
// runs the per-pixel step with the pixel's peak tap. A negative, non-finite
// or all-zero row, or a peak tap outside [0, W), sets kErrIrf.
template <bool kHist>
__global__ void __launch_bounds__(256) k_step_pirf(DevModel M, StepIO io, const double* __restrict__ irf_pix,
                                                   const int32_t* __restrict__ c_pix) {
  extern __shared__ __align__(16) float smem_f[];
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tw = (2 * M.W + 3) & ~3;
  float* sh_h = smem_f + wave * tw;
  float* sh_irf = sh_h + M.W;
  unsigned* hist = reinterpret_cast<unsigned*>(smem_f + nw * tw) + (size_t)wave * pixel_lds_words(M.T);
  const int p = blockIdx.x * nw + wave;
  if (p >= M.P) return;
  const double* row = irf_pix + (size_t)p * M.W;
  double hm = 0.0, tot = 0.0;
  bool bad = false;
  for (int j = lane; j < M.W; j += 64) {
    const double x = row[j];
    bad |= !(x >= 0.0) || !(x < 1e300);
    const double hv = irf_pow(x, (double)M.beta_d);
    sh_h[j] = (float)hv;
    sh_irf[j] = (float)x;
    hm = fmax(hm, hv);
    tot += x;
  }
#pragma unroll
  for (int m = 1; m <= 32; m <<= 1) {
    hm = fmax(hm, __shfl_xor(hm, m));
    tot += __shfl_xor(tot, m);
  }
  const int c = c_pix ? c_pix[p] : M.c;
  bad |= !(tot > 0.0) || c < 0 || c >= M.W;
  if (__any(bad)) {
    if (lane == 0) atomicOr(M.err, kErrIrf);
    return;
  }
  DevModel Mp = M;
  Mp.c = c;
  Mp.hmax = (float)(hm * (1.0 + 1e-6));
  wave_fence();
  pixel_step<kHist>(Mp, io, p, lane, hist, sh_h, sh_irf);
}

hipError_t launch_step_pirf(const DevModel& M, const StepIO& io, bool from_hist,
                            const double* irf_pix, const int32_t* c_pix, hipStream_t s) {
  const size_t tw = (size_t)((2 * M.W + 3) & ~3) * 4;
  const int nw = waves_for(tw + (size_t)pixel_lds_words(M.T) * 4, 0);
  if (nw == 0) return hipErrorInvalidValue;
  const dim3 grid((M.P + nw - 1) / nw);
  const size_t lds = nw * (tw + (size_t)pixel_lds_words(M.T) * 4);
  if (from_hist)
    hipLaunchKernelGGL(k_step_pirf<true>, grid, dim3(64 * nw), lds, s, M, io, irf_pix, c_pix);
  else
    hipLaunchKernelGGL(k_step_pirf<false>, grid, dim3(64 * nw), lds, s, M, io, irf_pix, c_pix);
  return hipGetLastError();
}

// ---------------------------------------------- continuous depth, Gaussian IRF
// Minimum-divergence depth off the grid for a Gaussian IRF of standard
// deviation sigma (Sec. II-B, eq. beta_div2 in its photon form; Sec. V: the
// correlation may be continuous, and a Gaussian IRF simplifies the updates).
// With f0(y|d) = N(y; d, sigma^2) the photon sum is, up to the factor
// (beta+1)/beta (2 pi sigma^2)^(-beta/2),
//   J(d) = sum_t z_t exp2(-a (t - d)^2),  a = beta log2(e) / (2 sigma^2),
// over the pixel's histogram (ToAs are bin indices). One wavefront per
// pixel: the LDS histogram of its photon list, J on every grid depth (each
// lane walks the non-empty bins within the truncation radius of its depths;
// terms beyond it are below 2^-40 of one photon's peak) and the first grid
// maximiser, then the stationarity fixed point d <- d + sum w (t - d) /
// sum w (w = z_t exp2(-a (t - d)^2)) from it, lanes taking the window's
// bins, until the step is below 1e-5 bins (at most 200 steps); the result is
// held to the grid's span.
constexpr float kGaussTail2 = 40.f;  // log2 units: truncation of the Gaussian terms

// Sum over all 64 lanes (every lane active), the same value in every lane
// and bit for bit the result of the xor butterfly over lane masks 1..32:
// within each 16-lane row the pair, quad, half-row and row steps are DPP
// moves (after the quad step every lane of a quad holds the same value, so
// the mirrored partner adds the same operand as the xor partner), then the
// four row sums are added as (r0 + r1) + (r2 + r3), the butterfly's order.
// No LDS round trip: the fixed point below is bound by this latency.
template <int kCtrl>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, 0xf, 0xf, false));
}

__device__ __forceinline__ float wave_sum64(float x) {
  x += dpp_move<0xb1>(x);   // quad_perm [1,0,3,2]: lane ^ 1
  x += dpp_move<0x4e>(x);   // quad_perm [2,3,0,1]: lane ^ 2
  x += dpp_move<0x141>(x);  // row_half_mirror: the other quad of the 8
  x += dpp_move<0x140>(x);  // row_mirror: the other 8 of the row
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 48));
  return (r0 + r1) + (r2 + r3);
}

__global__ void __launch_bounds__(256) k_gauss_mindiv(DevModel M, const int32_t* __restrict__ row_ptr,
                                                      const int16_t* __restrict__ toa, float a, float amp,
                                                      float* __restrict__ depth, float* __restrict__ value,
                                                      int32_t* __restrict__ grid_argmax) {
  extern __shared__ __align__(16) float smem_f[];
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned* hist = reinterpret_cast<unsigned*>(smem_f) + (size_t)wave * pixel_lds_words(M.T);
  unsigned* nzmask = hist + ((M.T + 1) >> 1);
  const int p = blockIdx.x * nw + wave;
  if (p >= M.P) return;
  {
    uint4* z4 = reinterpret_cast<uint4*>(hist);
    const int n4 = pixel_lds_words(M.T) >> 2;
    for (int w = lane; w < n4; w += 64) z4[w] = make_uint4(0u, 0u, 0u, 0u);
  }
  wave_fence();
  unsigned bad = 0u;
  const float K = csr_histogram(M, row_ptr, toa, p, lane, hist, nzmask, bad);
  if (bad) atomicOr(M.err, bad);
  wave_fence();
  const int R = (int)ceilf(sqrtf(kGaussTail2 / a));  // truncation radius, bins
  const int dhi = M.d_lo + M.D - 1;

  // J on the grid: each lane its depths, in increasing bin order
  float best = -INFINITY;
  int bidx = 0x7fffffff;
  if (K > 0.f) {
    for (int i = lane; i < M.D; i += 64) {
      const int d = M.d_lo + i;
      const int lo = max(d - R, 0), hi = min(d + R, M.T - 1);
      float J = 0.f;
      for (int t = lo; t <= hi;) {
        const int base = t & ~31;
        unsigned bits = nzmask[base >> 5] & (~0u << (t - base));
        if (hi - base < 31) bits &= (2u << (hi - base)) - 1u;
        while (bits) {
          const int tb = base + __builtin_ctz(bits);
          bits &= bits - 1u;
          const float e = (float)(tb - d);
          J = fmaf(packed_count(hist, tb), fast_exp2(-a * e * e), J);
        }
        t = base + 32;
      }
      if (J > best) {
        best = J;
        bidx = i;
      }
    }
  }
  group_argmax<1, 32>(best, bidx);
  if (bidx == 0x7fffffff) bidx = 0;

  // the stationarity fixed point from the grid maximiser
  float d = (float)(M.d_lo + bidx);
  float S0 = 0.f;
  auto sums = [&](float x, float& s0, float& s1) {
    const int lo = max((int)floorf(x) - R, 0), hi = min((int)ceilf(x) + R, M.T - 1);
    float a0 = 0.f, a1 = 0.f;
    for (int t = lo + lane; t <= hi; t += 64) {
      const float z = packed_count(hist, t);
      if (z > 0.f) {
        const float e = (float)t - x;
        const float w = z * fast_exp2(-a * e * e);
        a0 += w;
        a1 = fmaf(w, e, a1);
      }
    }
    s0 = wave_sum64(a0);
    s1 = wave_sum64(a1);
  };
  if (K > 0.f) {
    for (int it = 0; it < 200; ++it) {
      float s1;
      sums(d, S0, s1);
      if (!(S0 > 0.f)) break;
      const float step = s1 / S0;
      // a step that leaves d unchanged in fp32 (below half its spacing,
      // which exceeds 1e-5 from 256 bins on) would repeat itself to the last
      // iteration: stopping here gives the same d
      const float dn = d + step;
      if (dn == d) break;
      d = dn;
      if (fabsf(step) <= 1e-5f) break;
    }
    d = fminf(fmaxf(d, (float)M.d_lo), (float)dhi);
    float s1;
    sums(d, S0, s1);
  }
  if (lane == 0) {
    depth[p] = d;
    if (value) value[p] = M.scale2 * kLn2 * amp * S0;
    if (grid_argmax) grid_argmax[p] = M.d_lo + bidx;
  }
}

hipError_t launch_gauss_mindiv(const DevModel& M, const int32_t* row_ptr, const int16_t* toa,
                               double sigma, float* depth, float* value, int32_t* grid_argmax,
                               hipStream_t s) {
  const int nw = waves_for((size_t)pixel_lds_words(M.T) * 4, 0);
  if (nw == 0) return hipErrorInvalidValue;
  const float a = (float)(M.beta_d * 1.4426950408889634 / (2.0 * sigma * sigma));
  const float amp = (float)std::pow(2.0 * 3.14159265358979323846 * sigma * sigma, -0.5 * M.beta_d);
  const dim3 grid((M.P + nw - 1) / nw);
  hipLaunchKernelGGL(k_gauss_mindiv, grid, dim3(64 * nw), (size_t)nw * pixel_lds_words(M.T) * 4, s,
                     M, row_ptr, toa, a, amp, depth, value, grid_argmax);
  return hipGetLastError();
}

static size_t step_plain_fixed(const DevModel& M) { return (size_t)((2 * M.W + 3) & ~3) * 4; }
static size_t step_plain_per_wave(const DevModel& M) { return (size_t)pixel_lds_words(M.T) * 4; }

bool plain_supported(const DevModel& M) {
  return waves_for(step_plain_per_wave(M), step_plain_fixed(M)) > 0;
}

hipError_t launch_step_plain(const DevModel& M, const StepIO& io, bool from_hist, hipStream_t s) {
  const int nw = waves_for(step_plain_per_wave(M), step_plain_fixed(M));
  if (nw == 0) return hipErrorInvalidValue;
  const dim3 grid((M.P + nw - 1) / nw);
  const size_t lds = step_plain_fixed(M) + nw * step_plain_per_wave(M);
  if (from_hist)
    hipLaunchKernelGGL(k_step_plain<true>, grid, dim3(64 * nw), lds, s, M, io);
  else
    hipLaunchKernelGGL(k_step_plain<false>, grid, dim3(64 * nw), lds, s, M, io);
  return hipGetLastError();
}

}  // namespace r3d
