// One pixel of one frame (a1..a7) on one wavefront, for photon lists or
// histograms of any length: the per-pixel step shared by the single-frame
// photon-list kernel and the persistent batched kernel.
//
// The histogram is built in LDS as 16-bit counts packed two per word, and
// for photon lists also as one bit per bin marking the non-empty bins. The
// cost is only evaluated on candidate depths: since the cost is non-negative
// and at most scale * max(irf^beta) * K, and the log prior at the mean of one
// of its components is a lower bound of the best log pseudo-posterior, every
// depth where no component's log2-density reaches
//   theta = L_lb - 160 - scale2 * hmax * K - log2(9)
// has exp2(L - L*) below the smallest fp32 denormal: it contributes exactly
// zero weight and cannot be the argmax. Lanes walk the candidate range 64
// depths at a time (chunks that meet no component interval are skipped),
// keep online centred moments, and the wavefront merges them at the end.
//
// Cost gather: ell(d) sums irf^beta[j] * z[d - c + j] over the taps in
// increasing j. With few photons per bin range (3K <= T) the sum walks only
// the set bits of the non-empty-bin mask inside the window, in increasing
// bin order; the skipped terms are exact zeros (fma(h, 0, ell) == ell), so
// both gathers give the same bits.
#pragma once

#include "r3d_device.hpp"

namespace r3d {

constexpr float kPixCullMargin2 = 160.f;  // log2 units
constexpr float kPixLiveGap = 40.f;       // log2 units
constexpr float kPixLog2Nine = 3.16992500144231236f;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS words one wavefront needs for a pixel of T bins: packed 16-bit counts
// then the non-empty-bin mask, rounded up to whole 16-byte vectors.
__host__ __device__ constexpr int pixel_lds_words(int T) {
  return ((((T + 1) >> 1) + ((T + 31) >> 5)) + 3) & ~3;
}

// count of bin t in the packed LDS histogram
__device__ __forceinline__ float packed_count(const unsigned* hist, int t) {
  return (float)((hist[t >> 1] >> ((t & 1) << 4)) & 0xffffu);
}

// Candidate depth range [dlo_c, dhi_c] of a pixel (empty when dlo_c > dhi_c)
// from the bound above, and per component the radius R around its mean
// inside which its log2-density reaches theta, and the wider radius Rl
// (theta - kPixLiveGap) of the components kept in a chunk's mixture.
__device__ __forceinline__ void candidate_range(const DevModel& M, const Comps& C, unsigned live,
                                                float K, bool faulty, int lane, float (&R)[9],
                                                float (&Rl)[9], int& dlo_c, int& dhi_c) {
  const int dhi = M.d_lo + M.D - 1;
  const float l2max_ub = faulty ? 0.f : M.scale2 * M.hmax * K;
  float Llb = -INFINITY;
  if (lane < 9 && ((live >> lane) & 1u)) {
    float mk = C.m[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) mk = lane == k ? C.m[k] : mk;
    const float dk = fminf(fmaxf(rintf(mk), (float)M.d_lo), (float)dhi);
    Llb = log_prior2(C, dk, live);
  }
  Llb = group_max<1, 32>(Llb);
  const float theta = Llb - kPixCullMargin2 - l2max_ub - kPixLog2Nine;
  float lo = INFINITY, hi = -INFINITY;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    R[k] = C.w2[k] >= theta ? sqrtf((C.w2[k] - theta) / C.k2[k]) + 2.0f : -1e30f;
    Rl[k] = C.w2[k] >= theta - kPixLiveGap ? sqrtf((C.w2[k] - theta + kPixLiveGap) / C.k2[k]) + 2.0f
                                           : -1e30f;
    if (R[k] > 0.f) {
      lo = fminf(lo, C.m[k] - R[k]);
      hi = fmaxf(hi, C.m[k] + R[k]);
    }
  }
  dlo_c = M.d_lo;
  dhi_c = M.d_lo - 1;  // empty unless some component reaches theta
  if (lo <= hi) {
    dlo_c = (int)fmaxf(floorf(lo), (float)M.d_lo);
    dhi_c = (int)fminf(ceilf(hi), (float)dhi);
  }
}

// Wave-uniform masks of the 64-depth chunk starting at d0: ``cand`` the
// components that reach theta somewhere in it (zero: the chunk has no
// weight), ``cmask`` the components kept in its mixture.
__device__ __forceinline__ void chunk_masks(const Comps& C, const float (&R)[9],
                                            const float (&Rl)[9], int d0, unsigned& cand,
                                            unsigned& cmask) {
  const float dc = (float)d0 + 31.5f;
  cand = 0u;
  cmask = 0u;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    cand |= (fabsf(dc - C.m[k]) <= R[k] + 32.0f ? 1u : 0u) << k;
    cmask |= (fabsf(dc - C.m[k]) <= Rl[k] + 32.0f ? 1u : 0u) << k;
  }
  cand = __builtin_amdgcn_readfirstlane(cand);
  cmask = __builtin_amdgcn_readfirstlane(cmask);
}

// Cost gather at depth d: sum over taps j of tap[j] * z[d - c + j] in
// increasing j (bins outside [0, T) count zero). ``sparse`` walks only the
// non-empty bins of the window; both forms give the same bits.
__device__ __forceinline__ float cost_gather(const DevModel& M, const unsigned* hist,
                                             const unsigned* nzmask, const float* tap, int d,
                                             bool sparse) {
  float ell = 0.f;
  const int t0 = d - M.c;
  if (sparse) {
    const int lo = t0 > 0 ? t0 : 0;
    const int hi = (t0 + M.W) < M.T ? (t0 + M.W) : M.T;
    for (int t = lo; t < hi;) {
      const int base = t & ~31;
      unsigned bits = nzmask[base >> 5] & (~0u << (t - base));
      if (hi - base < 32) bits &= (1u << (hi - base)) - 1u;
      while (bits) {
        const int tb = base + __builtin_ctz(bits);
        bits &= bits - 1u;
        ell = fmaf(tap[tb - t0], packed_count(hist, tb), ell);
      }
      t = base + 32;
    }
  } else {
    const int jlo = t0 < 0 ? -t0 : 0;
    const int jhi = (M.T - t0) < M.W ? (M.T - t0) : M.W;
    for (int j = jlo; j < jhi; ++j) ell = fmaf(tap[j], packed_count(hist, t0 + j), ell);
  }
  return ell;
}

// Online centred moments of the weights exp2(L2 - Rm) at depths d: a new
// maximum rescales the sums and re-centres them on its depth.
__device__ __forceinline__ void moment_push(float L2, float d, float& Rm, float& ref, float& S0,
                                            float& S1, float& S2) {
  if (L2 > Rm) {
    const float sc = fast_exp2(Rm - L2);
    const float delta = ref - d;
    S0 *= sc;
    S1 *= sc;
    S2 *= sc;
    S2 = fmaf(delta, fmaf(2.f, S1, delta * S0), S2);
    S1 = fmaf(delta, S0, S1);
    Rm = L2;
    ref = d;
  }
  if (L2 > -INFINITY) {
    const float w = fast_exp2(L2 - Rm);
    const float e = d - ref;
    S0 += w;
    S1 = fmaf(e, w, S1);
    S2 = fmaf(e * e, w, S2);
  }
}

// Merge the lanes' moments: larger maximum wins (lower depth on ties); the
// other's sums are rescaled and re-centred on the winner (symmetric, so every
// lane ends with the same bits).
__device__ __forceinline__ void moment_merge_lanes(float& Rm, float& ref, float& S0, float& S1,
                                                   float& S2) {
#pragma unroll
  for (int xm = 1; xm <= 32; xm <<= 1) {
    const float oR = __shfl_xor(Rm, xm), oref = __shfl_xor(ref, xm);
    const float o0 = __shfl_xor(S0, xm), o1 = __shfl_xor(S1, xm), o2 = __shfl_xor(S2, xm);
    const bool other = (oR > Rm) || (oR == Rm && oref < ref);
    const float wR = other ? oR : Rm, wref = other ? oref : ref;
    auto bring = [&](float r, float rf, float& s0, float& s1, float& s2)
        __attribute__((always_inline)) {
      const float sc = (r == -INFINITY) ? 0.f : fast_exp2(r - wR);
      s0 *= sc;
      s1 *= sc;
      s2 *= sc;
      const float delta = rf - wref;
      s2 = fmaf(delta, fmaf(2.f, s1, delta * s0), s2);
      s1 = fmaf(delta, s0, s1);
    };
    float a0 = S0, a1 = S1, a2 = S2, b0 = o0, b1 = o1, b2 = o2;
    bring(Rm, ref, a0, a1, a2);
    bring(oR, oref, b0, b1, b2);
    S0 = a0 + b0;
    S1 = a1 + b1;
    S2 = a2 + b2;
    Rm = wR;
    ref = wref;
  }
}

// Photon-list histogram of pixel p into the zeroed LDS region (packed
// counts and non-empty-bin mask); returns the photon count and ORs error
// bits into ``bad``.
__device__ __forceinline__ float csr_histogram(const DevModel& M, const int32_t* row_ptr,
                                               const int16_t* toa, int p, int lane,
                                               unsigned* hist, unsigned* nzmask, unsigned& bad) {
  const int b = row_ptr[p], e = row_ptr[p + 1];
  if (e < b) bad |= kErrRange;
  if (e - b > 65535) bad |= kErrOverflow;  // 16-bit bins could overflow
  for (int k = b + lane; k < e; k += 64) {
    const int t = toa[k];
    if ((unsigned)t < (unsigned)M.T) {
      atomicAdd(&hist[t >> 1], 1u << ((t & 1) << 4));
      atomicOr(&nzmask[t >> 5], 1u << (t & 31));
    } else {
      bad |= kErrRange;
    }
  }
  return (float)(e > b ? e - b : 0);
}

// Per-pixel step. ``hist`` is this wavefront's 16-byte aligned LDS region of
// pixel_lds_words(T) words; ``sh_h`` and ``sh_irf`` hold irf^beta and irf
// (W floats each).
template <bool kHist>
__device__ __forceinline__ void pixel_step(const DevModel& M, const StepIO& io, int p, int lane,
                                           unsigned* hist, const float* sh_h,
                                           const float* sh_irf) {
  const int nwords = (M.T + 1) >> 1;
  unsigned* nzmask = hist + nwords;
  if constexpr (!kHist) {
    uint4* z4 = reinterpret_cast<uint4*>(hist);
    const int n4 = pixel_lds_words(M.T) >> 2;
    for (int w = lane; w < n4; w += 64) z4[w] = make_uint4(0u, 0u, 0u, 0u);
    wave_fence();
  }

  // ---- a1: histogram of the pixel ----
  const bool faulty = io.faulty && io.faulty[p];
  float K = 0.f;
  unsigned bad = 0;
  if (!faulty) {
    if constexpr (kHist) {
      const uint16_t* row = io.hist + (size_t)p * M.T;
      float ks = 0.f;
      for (int w = lane; w < nwords; w += 64) {
        unsigned packed = 0u;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int t = 2 * w + h;
          if (t < M.T) {
            const float x = half_bits_to_float(row[t]);
            const bool ok = fp16_count_ok(row[t]);
            if (!ok) bad |= kErrOverflow;
            const unsigned n = ok ? (unsigned)x : 0u;
            packed |= n << (16 * h);
            ks += (float)n;
          }
        }
        hist[w] = packed;
      }
      K = group_sum<1, 32>(ks);
    } else {
      K = csr_histogram(M, io.row_ptr, io.toa, p, lane, hist, nzmask, bad);
    }
  }
  if (bad) atomicOr(M.err, bad);
  wave_fence();

  // ---- a4: prior components (one pixel per wavefront: all uniform) ----
  Comps C;
  build_components(M, io.pm, io.pv, io.ppi, p, C);
  const unsigned live = __builtin_amdgcn_readfirstlane(C.live);

  // ---- candidate depth range from the bound ----
  float R[9], Rl[9];
  int dlo_c, dhi_c;
  candidate_range(M, C, live, K, faulty, lane, R, Rl, dlo_c, dhi_c);

  // ---- a3 + a5 on the candidates: online centred moments per lane ----
  const bool sparse = !kHist && 3.f * K <= (float)M.T;  // wave-uniform
  float Rm = -INFINITY, S0 = 0.f, S1 = 0.f, S2 = 0.f, ref = 0.f;
  for (int d0 = dlo_c; d0 <= dhi_c; d0 += 64) {
    unsigned cand, cmask;
    chunk_masks(C, R, Rl, d0, cand, cmask);
    if (cand == 0u) continue;
    const int d = d0 + lane;
    if (d > dhi_c) continue;
    const float ell = faulty ? 0.f : cost_gather(M, hist, nzmask, sh_h, d, sparse);
    const float L2 = fmaf(ell, M.scale2, log_prior2(C, (float)d, cmask));
    moment_push(L2, (float)d, Rm, ref, S0, S1, S2);
  }
  moment_merge_lanes(Rm, ref, S0, S1, S2);
  const float mu = S1 / S0;
  const int dstar = (int)ref;
  const float mean = ref + mu;
  // the MLE's depth: the posterior mean's nearest bin (Sec. II-E)
  const int dmle = (int)fminf(fmaxf(rintf(mean), (float)M.d_lo), (float)(M.d_lo + M.D - 1));
  const float var = fmaxf(S2 / S0 - mu * mu, 0.f);

  // ---- a6 + a7 ----
  const float pi_now = faulty ? 0.5f : (io.pi_in ? io.pi_in[p] : 1.0f);
  const bool detected = pi_now > 0.5f;
  float r_hat = 0.f, b_hat = K / (float)M.T;
  if (faulty) {
    b_hat = io.pb[p];
  } else if (detected) {
    constexpr int U = kMaxW / 64;
    float s[U], z[U];
    float S = 0.f, Kw = 0.f, nw = 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = lane + 64 * u;
      const int t = dmle - M.c + j;
      const bool in = j < M.W && t >= 0 && t < M.T;
      s[u] = in ? sh_irf[j] : 0.f;
      z[u] = in ? packed_count(hist, t) : 0.f;
      S += s[u];
      Kw += z[u];
      nw += in ? 1.f : 0.f;
    }
    S = group_sum<1, 32>(S);
    Kw = group_sum<1, 32>(Kw);
    nw = group_sum<1, 32>(nw);
    auto terms = [&](float r, float b, float SoT, float& g1, float& g2)
        __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (z[u] > 0.f) {
          const float q = (s[u] - SoT) * fast_rcp(fmaf(r, s[u], b));
          g1 = fmaf(z[u], q, g1);
          g2 = fmaf(-z[u] * q, q, g2);
        }
      }
    };
    mle_reflectivity<1, 32>(terms, K, S, Kw, nw, (float)M.T, r_hat, b_hat);
  }

  if (lane == 0) {
    io.nm[p] = mean;
    io.nv[p] = var;
    io.npi[p] = pi_now;
    io.nb[p] = b_hat;
    if (io.depth) io.depth[p] = detected ? mean : __builtin_nanf("");
    if (io.var) io.var[p] = var;
    if (io.argmax) io.argmax[p] = dstar;
    if (io.intensity) io.intensity[p] = r_hat;
    if (io.background) io.background[p] = b_hat;
    if (io.pi0_next) io.pi0_next[p] = pi0_next_at(M, io.pi_in, io.faulty, p);
    if (io.lognorm) io.lognorm[p] = Rm + fast_log2(S0);  // log2 sum_d exp2(L(d))
  }
}

}  // namespace r3d
