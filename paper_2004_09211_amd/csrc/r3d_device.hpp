// Device-side building blocks shared by the step kernels.
//
// Reductions over a lane group use an xor butterfly: every lane of the group
// combines the same two operands at every level (a + b == b + a bitwise), so
// all lanes end with bit-identical results and data-dependent branches on
// them stay uniform across the group.
#pragma once

#include "r3d_internal.hpp"

namespace r3d {

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

__device__ __forceinline__ float half_bits_to_float(uint16_t b) {
  _Float16 h;
  __builtin_memcpy(&h, &b, 2);
  return (float)h;
}

template <int kLo, int kHi>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
  for (int m = kLo; m <= kHi; m <<= 1) x += __shfl_xor(x, m);
  return x;
}

template <int kLo, int kHi>
__device__ __forceinline__ float group_max(float x) {
#pragma unroll
  for (int m = kLo; m <= kHi; m <<= 1) x = fmaxf(x, __shfl_xor(x, m));
  return x;
}

template <int kLo, int kHi>
__device__ __forceinline__ float group_min(float x) {
#pragma unroll
  for (int m = kLo; m <= kHi; m <<= 1) x = fminf(x, __shfl_xor(x, m));
  return x;
}

// (value, index) maximum; on equal values the lower index wins.
template <int kLo, int kHi>
__device__ __forceinline__ void group_argmax(float& v, int& i) {
#pragma unroll
  for (int m = kLo; m <= kHi; m <<= 1) {
    const float ov = __shfl_xor(v, m);
    const int oi = __shfl_xor(i, m);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

// Prior mixture of one pixel (Sec. III-A, eq. predict): component k of the
// 3x3 stencil is the previous Gaussian of neighbour k if that neighbour is in
// the frame and detected (pi > 0.5), the flat Gaussian otherwise; the random
// walk adds sigma_rw2 to its variance. Stored as the log2-density
//   q_k(d) = w2[k] - (d - m[k])^2 * k2[k],
//   w2 = log2(nu_k) - log2(2 pi V)/2,  k2 = log2(e) / (2 V).
struct Comps {
  float m[9], k2[9], w2[9];
};

__device__ __forceinline__ void build_components(const DevModel& M, const float* __restrict__ pm,
                                                 const float* __restrict__ pv,
                                                 const float* __restrict__ ppi, int p, Comps& C) {
  const int r = p / M.cols;
  const int col = p - r * M.cols;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int rr = r + k / 3 - 1, cc = col + k % 3 - 1;
    float m = M.m_flat, v = M.v_flat;
    if (rr >= 0 && rr < M.rows && cc >= 0 && cc < M.cols) {
      const int q = rr * M.cols + cc;
      if (ppi[q] > 0.5f) {
        m = pm[q];
        v = pv[q];
      }
    }
    const float V = v + M.sigma_rw2;
    C.m[k] = m;
    C.k2[k] = 0.5f * kLog2e / V;
    C.w2[k] = M.lognu2[k] - 0.5f * (kLog2TwoPi + log2f(V));
  }
}

// log2 f(d) by a max-shifted log-sum-exp over the 9 components.
__device__ __forceinline__ float log_prior2(const Comps& C, float d) {
  float q[9];
  float mx = -INFINITY;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float e = d - C.m[k];
    q[k] = C.w2[k] - e * e * C.k2[k];
    mx = fmaxf(mx, q[k]);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) s += fast_exp2(q[k] - mx);
  return mx + fast_log2(s);
}

// Presence probability of pixel q in the current frame: 0.5 when faulty,
// otherwise the caller's value (1 when none is given).
__device__ __forceinline__ float pi_now_at(const float* __restrict__ pi_in,
                                           const uint8_t* __restrict__ faulty, int q) {
  if (faulty && faulty[q]) return 0.5f;
  return pi_in ? pi_in[q] : 1.0f;
}

// Prior presence probability of the next frame (Sec. III-B, eq. prior_detect):
// sigmoid of the nu-weighted sum of logits over the stencil, pi clamped to
// [1e-6, 1-1e-6], out-of-frame neighbours counted as 0.5.
__device__ __forceinline__ float pi0_next_at(const DevModel& M, const float* __restrict__ pi_in,
                                             const uint8_t* __restrict__ faulty, int p) {
  const int r = p / M.cols;
  const int col = p - r * M.cols;
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (M.nu[k] == 0.f) continue;
    const int rr = r + k / 3 - 1, cc = col + k % 3 - 1;
    if (rr < 0 || rr >= M.rows || cc < 0 || cc >= M.cols) continue;
    float pk = pi_now_at(pi_in, faulty, rr * M.cols + cc);
    pk = fminf(fmaxf(pk, 1e-6f), 1.0f - 1e-6f);
    acc += M.nu[k] * logf(pk / (1.0f - pk));
  }
  return 1.0f / (1.0f + expf(-acc));
}

// Maximum-likelihood reflectivity r and background b of a detected pixel
// (Sec. II-E, eq. lik_bg_poisson) at depth d*: z_t ~ Poisson(r s_t + b) with
// s_t the IRF placed at d*. The optimum satisfies K = r S + b T, so it lies on
// b(r) = (K - r S)/T with r in [0, K/S]; the likelihood restricted to that
// segment is concave and its derivative
//   phi'(r) = sum_{t in window} z_t (s_t - S/T) / (r s_t + b) - K_out (S/T) / b
// (K_out = photons outside the IRF window, where s_t = 0) is bisected.
// Each lane of the group holds U window taps (s = 0, z = 0 for unused slots).
template <int kLo, int kHi, int U>
__device__ __forceinline__ void mle_reflectivity(const float (&s)[U], const float (&z)[U], float K,
                                                 float T, float& r_hat, float& b_hat) {
  float S = 0.f, Kw = 0.f;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    S += s[u];
    Kw += z[u];
  }
  S = group_sum<kLo, kHi>(S);
  Kw = group_sum<kLo, kHi>(Kw);
  const float invT = 1.0f / T;
  r_hat = 0.f;
  b_hat = K * invT;
  if (!(K > 0.f) || !(S > 0.f)) return;
  const float SoT = S * invT;
  const float Kout = K - Kw;
  auto dphi = [&](float r) {
    const float b = fmaxf((K - r * S) * invT, 0.f);
    float acc = 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (z[u] > 0.f) acc += z[u] * (s[u] - SoT) / (r * s[u] + b);
    acc = group_sum<kLo, kHi>(acc);
    if (Kout > 0.f) acc -= Kout * SoT / b;
    return acc;
  };
  if (!(dphi(0.f) > 0.f)) return;
  float hi = K / S;
  if (dphi(hi) >= 0.f) {
    r_hat = hi;
    b_hat = 0.f;
    return;
  }
  float lo = 0.f;
  for (int it = 0; it < 64; ++it) {
    const float mid = 0.5f * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (dphi(mid) > 0.f)
      lo = mid;
    else
      hi = mid;
  }
  r_hat = 0.5f * (lo + hi);
  b_hat = fmaxf((K - r_hat * S) * invT, 0.f);
}

}  // namespace r3d
