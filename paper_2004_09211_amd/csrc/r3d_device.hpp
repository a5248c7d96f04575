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
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float half_bits_to_float(uint16_t b) {
  _Float16 h;
  __builtin_memcpy(&h, &b, 2);
  return (float)h;
}

// A histogram count as the paths take it: an fp16 integer in [0, 2048] with
// a clear sign bit (so -0 is rejected like a negative count).
__device__ __forceinline__ bool fp16_count_ok(uint16_t b) {
  const float x = half_bits_to_float(b);
  return !(b & 0x8000u) && x <= kMaxFp16Count && x == truncf(x);
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
// Components with identical (m, V) (all flat ones, for instance) are merged
// into the first of them by adding their weights; a merged or zero-weight
// slot has w2 = -inf and its bit cleared in ``live``.
struct Comps {
  float m[9], k2[9], w2[9];
  unsigned live;
};

// log2(2^a + 2^b) with the hardware exp2 / log2 (about 1 ulp each)
__device__ __forceinline__ float log2_add(float a, float b) {
  const float mx = fmaxf(a, b), mn = fminf(a, b);
  return mx + fast_log2(1.0f + fast_exp2(mn - mx));
}

// merge components with identical (m, V) into the first of them
__device__ __forceinline__ void merge_components(Comps& C) {
#pragma unroll
  for (int k = 1; k < 9; ++k)
#pragma unroll
    for (int j = 0; j < k; ++j)
      if (C.w2[j] > -INFINITY && C.w2[k] > -INFINITY && C.m[j] == C.m[k] && C.k2[j] == C.k2[k]) {
        C.w2[j] = log2_add(C.w2[j], C.w2[k]);
        C.w2[k] = -INFINITY;
      }
  C.live = 0u;
#pragma unroll
  for (int k = 0; k < 9; ++k) C.live |= (C.w2[k] > -INFINITY ? 1u : 0u) << k;
}

// The 9 prior components of pixel p before merging (Sec. III-A, eq.
// predict): a detected in-frame neighbour contributes its state N(m, v), any
// other position the flat Gaussian; the random walk adds sigma_rw2. Also
// returns each variance V[k] and the mask of positions that read a
// neighbour's state (detected and in frame).
__device__ __forceinline__ void build_components_raw(const DevModel& M,
                                                     const float* __restrict__ pm,
                                                     const float* __restrict__ pv,
                                                     const float* __restrict__ ppi, int p,
                                                     Comps& C, float (&Vk)[9], unsigned& nb) {
  const int r = p / M.cols;
  const int col = p - r * M.cols;
  nb = 0u;
  C.live = 0u;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int rr = r + k / 3 - 1, cc = col + k % 3 - 1;
    float m = M.m_flat, v = M.v_flat;
    if (rr >= 0 && rr < M.rows && cc >= 0 && cc < M.cols) {
      const int q = rr * M.cols + cc;
      if (ppi[q] > 0.5f) {
        m = pm[q];
        v = pv[q];
        nb |= 1u << k;
      }
    }
    const float V = v + M.sigma_rw2;
    Vk[k] = V;
    C.m[k] = m;
    C.k2[k] = 0.5f * kLog2e / V;
    C.w2[k] = M.lognu2[k] - 0.5f * (kLog2TwoPi + fast_log2(V));
    C.live |= (C.w2[k] > -INFINITY ? 1u : 0u) << k;
  }
}

__device__ __forceinline__ void build_components(const DevModel& M, const float* __restrict__ pm,
                                                 const float* __restrict__ pv,
                                                 const float* __restrict__ ppi, int p, Comps& C) {
  float Vk[9];
  unsigned nb;
  build_components_raw(M, pm, pv, ppi, p, C, Vk, nb);
  merge_components(C);
}

// log2 f(d) by a max-shifted log-sum-exp over the components whose bit is set
// in ``mask`` (wave-uniform, so skipped components cost nothing). Returns
// -inf when none of this lane's components is in the mask.
__device__ __forceinline__ float log_prior2(const Comps& C, float d, unsigned mask) {
  float q[9];
  float mx = -INFINITY;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (mask & (1u << k)) {
      const float e = d - C.m[k];
      q[k] = C.w2[k] - e * e * C.k2[k];
      mx = fmaxf(mx, q[k]);
    }
  }
  if (mx == -INFINITY) return -INFINITY;
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k)
    if (mask & (1u << k)) s += fast_exp2(q[k] - mx);
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
  // without presence probabilities or faulty pixels every in-frame
  // neighbour has pi = 1: one logit serves them all
  const bool all_one = !pi_in && !faulty;
  float logit1 = 0.f;
  if (all_one) {
    const float pk = fminf(fmaxf(1.0f, 1e-6f), 1.0f - 1e-6f);
    logit1 = fast_log2(pk) - fast_log2(1.0f - pk);
  }
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (M.nu[k] == 0.f) continue;
    const int rr = r + k / 3 - 1, cc = col + k % 3 - 1;
    if (rr < 0 || rr >= M.rows || cc < 0 || cc >= M.cols) continue;
    float lg = logit1;  // logit in log2 units
    if (!all_one) {
      float pk = pi_now_at(pi_in, faulty, rr * M.cols + cc);
      pk = fminf(fmaxf(pk, 1e-6f), 1.0f - 1e-6f);
      lg = fast_log2(pk) - fast_log2(1.0f - pk);
    }
    acc += M.nu[k] * lg;
  }
  return fast_rcp(1.0f + fast_exp2(-acc));
}

// Maximum-likelihood reflectivity r and background b of a detected pixel
// (Sec. II-E, eq. lik_bg_poisson) at depth d*: z_t ~ Poisson(r s_t + b) with
// s_t the IRF placed at d*. The optimum satisfies K = r S + b T, so it lies on
// b(r) = (K - r S)/T with r in [0, K/S]; the likelihood restricted to that
// segment is concave and its derivative
//   phi'(r) = sum_{t in window} z_t (s_t - S/T) / (r s_t + b) - K_out (S/T) / b
// (K_out = photons outside the IRF window, where s_t = 0) is decreasing.
// Its root is found by Newton steps on phi' kept inside a shrinking bracket
// (bisection when a step leaves it). ``terms(r, b, SoT, g1, g2)`` adds this
// lane's window taps to phi' (g1) and phi'' (g2); the group sums them.
template <int kLo, int kHi, class Terms>
__device__ __forceinline__ void mle_reflectivity(Terms terms, float K, float S, float Kw, float nwin,
                                                 float T, float& r_hat, float& b_hat) {
  const float invT = 1.0f / T;
  r_hat = 0.f;
  b_hat = K * invT;
  if (!(K > 0.f) || !(S > 0.f)) return;
  const float SoT = S * invT;
  const float Kout = K - Kw;
  auto eval = [&](float r, float& g1, float& g2) {
    const float b = fmaxf((K - r * S) * invT, 0.f);
    float a1 = 0.f, a2 = 0.f;
    terms(r, b, SoT, a1, a2);
    g1 = group_sum<kLo, kHi>(a1);
    g2 = group_sum<kLo, kHi>(a2);
    if (Kout > 0.f) {
      const float q = SoT / b;
      g1 -= Kout * q;
      g2 -= Kout * q * q;
    }
  };
  float g1, g2;
  eval(0.f, g1, g2);
  if (!(g1 > 0.f)) return;
  float lo = 0.f, hi = K / S;
  eval(hi, g1, g2);
  if (g1 >= 0.f) {
    r_hat = hi;
    b_hat = 0.f;
    return;
  }
  // start from the window excess over the background it would hold
  float r = (Kw - K * nwin * invT) / fmaxf(S - nwin * SoT, 1e-30f);
  if (!(r > lo && r < hi)) r = 0.5f * (lo + hi);
  // fp32 sums of the score carry rounding noise near the root, so the
  // iteration stops at a step (or bracket width) of 1e-5 * max(r, 1)
  for (int it = 0; it < 16; ++it) {
    eval(r, g1, g2);
    if (g1 > 0.f)
      lo = r;
    else
      hi = r;
    if (g1 == 0.f) break;
    const float step = g1 * fast_rcp(g2);
    const float tol = 1e-5f * fmaxf(r, 1.0f);
    if (fabsf(step) <= tol) {  // converged: the Newton step is below the noise floor
      r = fminf(fmaxf(r - step, lo), hi);
      break;
    }
    float rn = r - step;
    if (!(rn > lo && rn < hi)) rn = 0.5f * (lo + hi);  // outside the bracket: bisect
    r = rn;
    if (!(hi - lo > tol)) break;
  }
  r_hat = r;
  b_hat = fmaxf((K - r * S) * invT, 0.f);
}

}  // namespace r3d
