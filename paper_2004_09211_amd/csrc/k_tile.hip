// Fused per-frame step on fp16 histograms, one wavefront per 4x4 pixel block.
//
// Cost (a3). For a 16-bin depth tile [d0, d0+16) the cost of the 16 pixels is
// a banded Toeplitz product C[d][p] = sum_t H[d][t] Z[t][p] with
// H[d][t] = irf^beta[t - d + c]. Bins are taken in 32-bin blocks aligned to
// multiples of 32, so H only depends on (d0 - c) mod 32, which takes two
// values for the two tiles of each 32-bin pair: the A operands of every
// (tile-of-pair, block) combination are built once and stay in registers,
// and each histogram block (the B operand: 8 fp16 counts of one pixel per
// lane, the matrix core's 16x16x32 layout) is loaded once, kept in a register
// ring with a prefetch distance, and used by every tile whose band touches it.
// Engines: fp16 matrix cores with irf^beta in fp16 (kEngMfma16), the same with
// irf^beta split into hi*2^11 and lo = (irf^beta - hi)*2^11 contracted into
// one fp32 accumulator (kEngMfma16x2), or fp32 vector FMAs from an LDS copy of
// the same blocks (kEngValu, the plain form).
//
// Posterior (a4, a5) in two passes. Pass 1 streams every tile and keeps the
// maximum cost per pixel and the cost at a reference depth (the rounded mean
// of the pixel's own prior component). With lmax the cost maximum and L* the
// maximum of the log2 pseudo-posterior L = ell + log f, a lower bound
//   L* >= max(lmax + min_grid log f, ell(d_ref) + log f(d_ref))
// and the upper bound L(d) <= lmax + max_k q_k(d) + log2(9) give, per prior
// component, the interval of depths where L(d) can reach L* - 160 (log2
// units): outside every interval exp2(L - L*) is below the smallest fp32
// denormal, so those depths contribute exactly zero weight and cannot be the
// argmax. Pass 2 recomputes the cost on the 16-bin tiles that meet an
// interval of any pixel of the block and accumulates the argmax and the
// moments online (running maximum, rescaled and re-centred sums).
#include "r3d_device.hpp"
#include "r3d_tile.hpp"

#include <type_traits>

namespace r3d {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kRingT = 256;            // LDS ring per pixel (fp16 bins), VALU engine
constexpr float kCullMargin2 = 160.f;  // log2 units: exp2(-150) rounds to zero in fp32
constexpr float kLog2Nine = 3.16992500144231236f;
constexpr float kLiveGap = 40.f;     // log2 units
constexpr unsigned kOob = 0x80000000u;  // buffer offset past every record: loads return zeros
constexpr int kBufWord3 = 0x00020000;   // raw buffer descriptor, 32-bit data format

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ floatx4 mfma16(half8 a, half8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Block order: the blocks on the frame's border first (their out-of-frame
// neighbours bring flat prior components, which make every depth tile a
// candidate and these blocks the slowest), then the interior row by row.
__device__ __forceinline__ void block_of(int idx, int nbr, int nbc, int& br, int& bc) {
  if (nbr <= 2 || nbc <= 2) {
    br = idx / nbc;
    bc = idx - br * nbc;
    return;
  }
  const int nb = 2 * nbc + 2 * (nbr - 2);
  if (idx < nbc) {
    br = 0;
    bc = idx;
  } else if (idx < 2 * nbc) {
    br = nbr - 1;
    bc = idx - nbc;
  } else if (idx < 2 * nbc + (nbr - 2)) {
    br = 1 + idx - 2 * nbc;
    bc = 0;
  } else if (idx < nb) {
    br = 1 + idx - 2 * nbc - (nbr - 2);
    bc = nbc - 1;
  } else {
    const int i = idx - nb;
    br = 1 + i / (nbc - 2);
    bc = 1 + i - (i / (nbc - 2)) * (nbc - 2);
  }
}

// Prior components of the lane's pixel from the block's 6x6 halo of
// previous states in LDS (halo[0..35] = m, [36..71] = v, [72..107] = pi,
// pi = -1 outside the frame).
__device__ __forceinline__ void halo_components(const DevModel& M, const float* halo, int i16,
                                                Comps& C) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int idx = ((i16 >> 2) + k / 3) * 6 + (i16 & 3) + k % 3;
    const float hp = halo[72 + idx];
    const bool det = hp > 0.5f;
    const float m = det ? halo[idx] : M.m_flat;
    const float V = (det ? halo[36 + idx] : M.v_flat) + M.sigma_rw2;
    C.m[k] = m;
    C.k2[k] = 0.5f * kLog2e / V;
    C.w2[k] = M.lognu2[k] - 0.5f * (kLog2TwoPi + log2f(V));
  }
  merge_components(C);
}

template <int kEng, int NBP, bool kCostOnly>
__global__ void __launch_bounds__(256) k_step_tile(DevModel M, TileGeom G, StepIO io,
                                                   float* __restrict__ ell_out) {
  constexpr bool kMfma = kEng != kEngValu;
  constexpr bool kSplit = kEng == kEngMfma16x2;
  constexpr int PF = kMfma ? 6 : 3;  // pass-1 prefetch distance, in 32-bin pairs
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;

  float* sh_irf = reinterpret_cast<float*>(smem);
  unsigned char* wbase = smem + G.lds_fixed + wave * G.lds_per_wave;
  unsigned* mask = reinterpret_cast<unsigned*>(wbase);
  float* halo = reinterpret_cast<float*>(wbase + G.mask_bytes);
  _Float16* ring_lds = reinterpret_cast<_Float16*>(wbase + G.mask_bytes + G.halo_bytes);

  for (int j = threadIdx.x; j < M.W; j += blockDim.x) sh_irf[j] = M.irf[j];
  __syncthreads();
  const int gw = blockIdx.x * 4 + wave;
  if (gw >= G.nblk) return;

  // ---- pixel of this lane (column i16 of the tile) ----
  int br, bc;
  block_of(gw, G.nblk / G.nbc, G.nbc, br, bc);
  br = __builtin_amdgcn_readfirstlane(br);
  bc = __builtin_amdgcn_readfirstlane(bc);
  const int pr = 4 * br + (i16 >> 2), pc = 4 * bc + (i16 & 3);
  const bool valid = pr < M.rows && pc < M.cols && pr * M.cols + pc < M.P;
  const int p = valid ? pr * M.cols + pc : 0;
  const bool faulty = valid && io.faulty && io.faulty[p];
  const bool has_data = valid && !faulty;
  const uint16_t* row = io.hist + (size_t)p * M.T;
  const int dhi = M.d_lo + M.D - 1;

  // previous states of the block's 6x6 halo into LDS (read after pass 1)
  if constexpr (!kCostOnly) {
    if (lane < 36) {
      const int hr = 4 * br - 1 + lane / 6, hc = 4 * bc - 1 + lane % 6;
      float hm = 0.f, hv = 1.f, hp = -1.f;
      if (hr >= 0 && hr < M.rows && hc >= 0 && hc < M.cols) {
        const int q = hr * M.cols + hc;
        hm = io.pm[q];
        hv = io.pv[q];
        hp = io.ppi[q];
      }
      halo[lane] = hm;
      halo[36 + lane] = hv;
      halo[72 + lane] = hp;
    }
  }

  // ---- reference depth: the rounded mean of the pixel's own prior component ----
  int dref = M.d_lo, mref = -1;
  if constexpr (!kCostOnly) {
    const float mown = (valid && io.ppi[p] > 0.5f) ? io.pm[p] : M.m_flat;
    dref = (int)fminf(fmaxf(rintf(mown), (float)M.d_lo), (float)dhi);
    mref = (dref - M.d_lo) >> 5;
  }
  const int rrel = dref - M.d_lo;
  const int tref = (rrel >> 4) & 1, gref = (rrel >> 2) & 3, qref = rrel & 3;
  const int mref_lane = (valid && g == gref) ? mref : -1;  // only this lane sees d_ref

  // ---- histogram blocks through a buffer descriptor based at the block's
  // first pixel: an offset past the records (a pixel outside the frame, a
  // faulty pixel, a block outside [0, T)) reads zeros ----
  const int p0 = __builtin_amdgcn_readfirstlane((4 * br) * M.cols + 4 * bc);
  const long long rec = (long long)(M.P - p0) * M.T * 2;
  const __amdgpu_buffer_rsrc_t hbuf = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(io.hist + (size_t)p0 * M.T), (short)0, (int)(rec < 0x7fffffffLL ? rec : 0x7fffffffLL),
      kBufWord3);
  const unsigned lane_off = has_data ? (unsigned)(((p - p0) * M.T + 8 * g) * 2) : kOob;
  auto load_block = [&](int kb) __attribute__((always_inline)) -> half8 {
    const bool in = kb >= 0 && 32 * kb + 8 * g < M.T && lane_off != kOob;
    const unsigned off = in ? lane_off + 64u * (unsigned)kb : kOob;
    return __builtin_bit_cast(half8, __builtin_amdgcn_raw_buffer_load_b128(hbuf, off, 0, 0));
  };

  // ---- Toeplitz A operands: hi part (and lo part for the split engine) ----
  half8 Ahi[2][NBP], Alo[2][NBP];
  auto build_A = [&](half8 (&A)[2][NBP], const _Float16* src, bool scale) __attribute__((always_inline)) {
#pragma unroll
    for (int tau = 0; tau < 2; ++tau)
#pragma unroll
      for (int b = 0; b < NBP; ++b)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int j = 32 * b + 8 * g + s - 16 * tau - i16 - G.o;
          const _Float16 v = (j >= 0 && j < M.W) ? src[j] : (_Float16)0.f;
          A[tau][b][s] = scale ? v * (_Float16)2048.f : v;
        }
  };
  if constexpr (kMfma) build_A(Ahi, M.h16hi, kSplit);
  const float cs2 = M.scale2 * (kSplit ? (1.0f / 2048.0f) : 1.0f);

  // fp32 cost of tile tau of pair m from the LDS ring (VALU engine): lane
  // computes its 4 depths d = d_lo + 32 m + 16 tau + 4 g + q.
  auto valu_tile = [&](int m, int tau) __attribute__((always_inline)) -> floatx4 {
    const int t0 = M.d_lo + 32 * m + 16 * tau + 4 * g - M.c;
    const _Float16* rp = ring_lds + i16 * kRingT;
    float a0 = (float)rp[(t0 + 0) & (kRingT - 1)];
    float a1 = (float)rp[(t0 + 1) & (kRingT - 1)];
    float a2 = (float)rp[(t0 + 2) & (kRingT - 1)];
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < M.W; ++j) {
      const float a3 = (float)rp[(t0 + j + 3) & (kRingT - 1)];
      const float hj = M.h[j];
      acc[0] = fmaf(hj, a0, acc[0]);
      acc[1] = fmaf(hj, a1, acc[1]);
      acc[2] = fmaf(hj, a2, acc[2]);
      acc[3] = fmaf(hj, a3, acc[3]);
      a0 = a1;
      a1 = a2;
      a2 = a3;
    }
    return acc;
  };
  auto ring_store = [&](int kb, half8 v) __attribute__((always_inline)) {
    *reinterpret_cast<half8*>(ring_lds + i16 * kRingT + ((32 * kb + 8 * g) & (kRingT - 1))) = v;
  };

  // photon count K and the largest fp16 bit pattern (count validation)
  float Kv = 0.f;
  floatx4 Kacc = {0.f, 0.f, 0.f, 0.f};  // via a ones-row contraction
  ushort8 vmax = {0, 0, 0, 0, 0, 0, 0, 0};
  half8 ones;
#pragma unroll
  for (int s = 0; s < 8; ++s) ones[s] = (_Float16)1.f;
  auto account = [&](half8 v) __attribute__((always_inline)) {
    vmax = __builtin_elementwise_max(vmax, __builtin_bit_cast(ushort8, v));
    if constexpr (kMfma) {
      Kacc = mfma16(ones, v, Kacc);
    } else {
#pragma unroll
      for (int s = 0; s < 8; ++s) Kv += (float)v[s];
    }
  };

  // Exact cost of both tiles of pair m from its NBP blocks: fp16 hi (and lo)
  // contractions in independent chains, or fp32 from the LDS ring.
  auto pair_cost = [&](int m, const half8 (&blk)[NBP], floatx4& c0, floatx4& c1)
      __attribute__((always_inline)) {
    if constexpr (kMfma) {
      floatx4 h0 = {0.f, 0.f, 0.f, 0.f}, h1 = h0, l0 = h0, l1 = h0;
#pragma unroll
      for (int b = 0; b < NBP; ++b) {
        h0 = mfma16(Ahi[0][b], blk[b], h0);
        h1 = mfma16(Ahi[1][b], blk[b], h1);
        if constexpr (kSplit) {
          l0 = mfma16(Alo[0][b], blk[b], l0);
          l1 = mfma16(Alo[1][b], blk[b], l1);
        }
      }
      if constexpr (kSplit) {
        c0 = h0 + l0;
        c1 = h1 + l1;
      } else {
        c0 = h0;
        c1 = h1;
      }
    } else {
      c0 = valu_tile(m, 0);
      c1 = valu_tile(m, 1);
    }
  };
  // Stream every pair in order through the register ring (the blocks of the
  // current pair plus PF prefetched ones); the VALU engine mirrors the
  // current pair's blocks into its LDS ring.
  auto stream = [&](auto pf, auto&& on_pair) __attribute__((always_inline)) {
    constexpr int RING = NBP + decltype(pf)::value;
    half8 ring[RING];
#pragma unroll
    for (int x = 0; x < RING - 1; ++x) ring[x] = load_block(G.kbA0 + x);
    for (int m0 = 0; m0 < G.npairs; m0 += RING) {
#pragma unroll
      for (int u = 0; u < RING; ++u) {
        const int m = m0 + u;
        if (m < G.npairs) {
          ring[(u + RING - 1) % RING] = load_block(G.kbA0 + m + RING - 1);
          if constexpr (!kMfma) {
            wave_sync();
            if (m == 0) {
#pragma unroll
              for (int b = 0; b < NBP; ++b) ring_store(G.kbA0 + b, ring[(u + b) % RING]);
            } else {
              ring_store(G.kbA0 + m + NBP - 1, ring[(u + NBP - 1) % RING]);
            }
            wave_sync();
          }
          on_pair(m, ring, u, std::integral_constant<int, RING>{});
        }
      }
    }
  };

  // ============================ pass 1 ============================
  // Matrix engines evaluate the fp16-hi cost only: it bounds the exact cost
  // within a relative 2^-10 plus K 2^-24 (the rounding of irf^beta to fp16),
  // which the bound below absorbs. The cost is >= 0, so its fp32 maximum is
  // the integer maximum of the bit patterns.
  unsigned lmax_bits = 0u;
  float lref = -INFINITY;
  stream(std::integral_constant<int, PF>{}, [&](int m, auto& ring, int u, auto rt)
             __attribute__((always_inline)) {
    constexpr int RING = decltype(rt)::value;
    if (m == 0) {
#pragma unroll
      for (int b = 0; b < NBP - 1; ++b) account(ring[(u + b) % RING]);
    }
    account(ring[(u + NBP - 1) % RING]);
    floatx4 c0, c1;
    if constexpr (kCostOnly) {
      half8 blk[NBP];
#pragma unroll
      for (int b = 0; b < NBP; ++b) blk[b] = ring[(u + b) % RING];
      if constexpr (kSplit) {
        if (m == 0) build_A(Alo, M.h16lo, false);
      }
      pair_cost(m, blk, c0, c1);
      const float sc = cs2 * kLn2;
      if (valid) {
#pragma unroll
        for (int tau = 0; tau < 2; ++tau) {
          const int dbase = M.d_lo + 32 * m + 16 * tau + 4 * g;
          const floatx4 acc = tau ? c1 : c0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (dbase + q <= dhi) ell_out[(size_t)p * M.D + (dbase + q - M.d_lo)] = acc[q] * sc;
        }
      }
    } else {
      if constexpr (kMfma) {
        c0 = floatx4{0.f, 0.f, 0.f, 0.f};
        c1 = c0;
#pragma unroll
        for (int b = 0; b < NBP; ++b) {
          c0 = mfma16(Ahi[0][b], ring[(u + b) % RING], c0);
          c1 = mfma16(Ahi[1][b], ring[(u + b) % RING], c1);
        }
      } else {
        c0 = valu_tile(m, 0);
        c1 = valu_tile(m, 1);
      }
      const unsigned a = __builtin_elementwise_max(__float_as_uint(c0[0]), __float_as_uint(c0[1]));
      const unsigned b = __builtin_elementwise_max(__float_as_uint(c0[2]), __float_as_uint(c0[3]));
      const unsigned c = __builtin_elementwise_max(__float_as_uint(c1[0]), __float_as_uint(c1[1]));
      const unsigned d = __builtin_elementwise_max(__float_as_uint(c1[2]), __float_as_uint(c1[3]));
      lmax_bits = __builtin_elementwise_max(lmax_bits, __builtin_elementwise_max(
                      __builtin_elementwise_max(a, b), __builtin_elementwise_max(c, d)));
      const floatx4 cr = tref ? c1 : c0;
      const float v = qref == 0 ? cr[0] : qref == 1 ? cr[1] : qref == 2 ? cr[2] : cr[3];
      lref = m == mref_lane ? v : lref;
    }
  });
  // blocks of [0, T) that no depth window reaches still hold photons
  for (int kb = 0; kb < G.nkb; ++kb) {
    if (kb >= G.kbA0 && kb <= G.kb_last) continue;
    account(load_block(kb));
  }
  {
    unsigned bad = 0;
#pragma unroll
    for (int s = 0; s < 8; ++s) bad |= vmax[s] > 0x6800u ? kErrOverflow : 0u;  // > 2048 or negative
    if (bad) atomicOr(M.err, bad);
  }
  if constexpr (kCostOnly) return;

  const float K = kMfma ? Kacc[0] : group_sum<16, 32>(Kv);
  lmax_bits = max(lmax_bits, (unsigned)__shfl_xor((int)lmax_bits, 16));
  lmax_bits = max(lmax_bits, (unsigned)__shfl_xor((int)lmax_bits, 32));
  float lmax = __uint_as_float(lmax_bits);
  lref = group_max<16, 32>(lref);
  if constexpr (kMfma) {
    const float slack = K * (kSplit ? 2048.0f : 1.0f) * 0x1p-23f;
    lmax = lmax * (1.0f + 0x1p-9f) + slack;
    if (lref > -INFINITY) lref = lref * (1.0f - 0x1p-9f) - slack;
  }

  // ===================== candidate depth tiles =====================
  wave_sync();
  Comps C;
  halo_components(M, halo, i16, C);
  const float l2max = lmax * cs2;
  float lbf = -INFINITY;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float e = fmaxf(fabsf((float)M.d_lo - C.m[k]), fabsf((float)dhi - C.m[k]));
    lbf = fmaxf(lbf, C.w2[k] - e * e * C.k2[k]);
  }
  unsigned wave_live = 0u;
#pragma unroll
  for (int k = 0; k < 9; ++k) wave_live |= (__any(valid && (C.live >> k & 1u)) ? 1u : 0u) << k;
  float Llb = l2max + lbf;
  if (lref > -INFINITY) Llb = fmaxf(Llb, fmaf(lref, cs2, log_prior2(C, (float)dref, wave_live)));
  const float theta = Llb - kCullMargin2 - l2max - kLog2Nine;

  // Component k is "live" on depths where q_k >= theta - kLiveGap: at a
  // candidate depth some component reaches theta, so components below
  // theta - kLiveGap change f by less than 9 * 2^-kLiveGap relative and are
  // skipped; depths where no component is live are not candidates at all.
  // The wavefront keeps, per component, the tile range covering every lane's
  // live interval (wave-uniform, so the per-tile test is scalar).
  int TA[9], TB[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const bool lv = valid && C.w2[k] >= theta - kLiveGap;
    const float R = lv ? sqrtf((C.w2[k] - theta + kLiveGap) / C.k2[k]) + 2.0f : 0.f;
    float lo = lv ? C.m[k] - R : INFINITY;
    float hi = lv ? C.m[k] + R : -INFINITY;
#pragma unroll
    for (int xm = 1; xm <= 32; xm <<= 1) {
      lo = fminf(lo, __shfl_xor(lo, xm));
      hi = fmaxf(hi, __shfl_xor(hi, xm));
    }
    lo = fmaxf(lo, (float)M.d_lo);
    hi = fminf(hi, (float)dhi);
    const bool any = lo <= hi;
    TA[k] = __builtin_amdgcn_readfirstlane(any ? ((int)floorf(lo) - M.d_lo) >> 4 : 1);
    TB[k] = __builtin_amdgcn_readfirstlane(any ? ((int)ceilf(hi) - M.d_lo) >> 4 : 0);
  }

  for (int w = lane; w < G.mask_words; w += 64) mask[w] = 0u;
  wave_sync();
  if (valid) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if ((k & 3) != g || !(C.w2[k] >= theta)) continue;
      const float R = sqrtf((C.w2[k] - theta) / C.k2[k]) + 2.0f;
      const float lo = fmaxf(floorf(C.m[k] - R), (float)M.d_lo);
      const float hi = fminf(ceilf(C.m[k] + R), (float)dhi);
      if (!(lo <= hi)) continue;
      const int ta = ((int)lo - M.d_lo) >> 4, tb = ((int)hi - M.d_lo) >> 4;
      for (int w = ta >> 5; w <= (tb >> 5); ++w) {
        const int a = w == (ta >> 5) ? (ta & 31) : 0;
        const int z = w == (tb >> 5) ? (tb & 31) : 31;
        const unsigned bits = (z == 31 ? 0xffffffffu : ((1u << (z + 1)) - 1u)) & ~((1u << a) - 1u);
        atomicOr(&mask[w], bits);
      }
    }
  }
  wave_sync();
  if constexpr (kSplit) build_A(Alo, M.h16lo, false);

  // ============================ pass 2 ============================
  float R = -INFINITY, S0 = 0.f, S1 = 0.f, S2 = 0.f, ref = 0.f;
  auto is_cand = [&](int dt) __attribute__((always_inline)) -> bool {
    return (__builtin_amdgcn_readfirstlane(mask[dt >> 5]) >> (dt & 31)) & 1u;
  };
  // log2 pseudo-posterior of the lane's 4 depths of tile dt, online moments
  auto tile_epi = [&](const floatx4& acc, int dt) __attribute__((always_inline)) {
    const int dbase = M.d_lo + 16 * dt + 4 * g;
    unsigned tmask = 0u;  // components live in this tile for some lane
#pragma unroll
    for (int k = 0; k < 9; ++k) tmask |= (TA[k] <= dt && dt <= TB[k] ? 1u : 0u) << k;
    float lp[4];
    if (__builtin_popcount(tmask) == 1) {
      // one live component: log f is its log density
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (tmask == (1u << k)) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float e = (float)(dbase + q) - C.m[k];
            lp[q] = fmaf(-e * e, C.k2[k], C.w2[k]);
          }
        }
    } else {
      float mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
      float sm[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (tmask & (1u << k)) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float e = (float)(dbase + q) - C.m[k];
            mx[q] = fmaxf(mx[q], fmaf(-e * e, C.k2[k], C.w2[k]));
          }
        }
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (tmask & (1u << k)) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float e = (float)(dbase + q) - C.m[k];
            sm[q] += fast_exp2(fmaf(-e * e, C.k2[k], C.w2[k]) - mx[q]);
          }
        }
#pragma unroll
      for (int q = 0; q < 4; ++q) lp[q] = mx[q] == -INFINITY ? -INFINITY : mx[q] + fast_log2(sm[q]);
    }
    float L[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      L[q] = (valid && dbase + q <= dhi) ? fmaf(acc[q], cs2, lp[q]) : -INFINITY;
    float mt = L[0];
    int qt = 0;
#pragma unroll
    for (int q = 1; q < 4; ++q)
      if (L[q] > mt) {
        mt = L[q];
        qt = q;
      }
    if (mt > R) {
      const float sc = fast_exp2(R - mt);
      const float dnew = (float)(dbase + qt);
      const float delta = ref - dnew;
      S0 *= sc;
      S1 *= sc;
      S2 *= sc;
      S2 = fmaf(delta, fmaf(2.f, S1, delta * S0), S2);
      S1 = fmaf(delta, S0, S1);
      R = mt;
      ref = dnew;
    }
    if (mt > -INFINITY) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float wq = fast_exp2(L[q] - R);
        const float e = (float)(dbase + q) - ref;
        S0 += wq;
        S1 = fmaf(e, wq, S1);
        S2 = fmaf(e * e, wq, S2);
      }
    }
  };
  auto pair_epi = [&](int m, const half8 (&blk)[NBP]) __attribute__((always_inline)) {
    const bool c0 = is_cand(2 * m), c1 = is_cand(2 * m + 1);
    if (!c0 && !c1) return;
    floatx4 a0, a1;
    pair_cost(m, blk, a0, a1);
    if (c0) tile_epi(a0, 2 * m);
    if (c1) tile_epi(a1, 2 * m + 1);
  };
  // pairs holding a candidate tile: bit 2i of pbits(word w) is pair 16 w + i
  auto pbits = [&](int w) __attribute__((always_inline)) -> unsigned {
    const unsigned x = __builtin_amdgcn_readfirstlane(mask[w]);
    return (x | (x >> 1)) & 0x55555555u;
  };
  int ncand = 0;
  for (int w = 0; w < G.mask_words; ++w) ncand += __builtin_popcount(pbits(w));
  if (4 * ncand >= G.npairs) {
    // dense: stream every pair again, evaluate the candidate ones
    stream(std::integral_constant<int, 2>{}, [&](int m, auto& ring, int u, auto rt)
               __attribute__((always_inline)) {
      constexpr int RING = decltype(rt)::value;
      half8 blk[NBP];
#pragma unroll
      for (int b = 0; b < NBP; ++b) blk[b] = ring[(u + b) % RING];
      pair_epi(m, blk);
    });
  } else {
    // sparse: candidate pairs in order, the next one fetched while the
    // current one is evaluated
    int mw = 0;
    unsigned mb = G.mask_words > 0 ? pbits(0) : 0u;
    auto next_pair = [&]() __attribute__((always_inline)) -> int {
      while (mb == 0u) {
        if (++mw >= G.mask_words) return -1;
        mb = pbits(mw);
      }
      const int i = __builtin_ctz(mb);
      mb &= mb - 1u;
      return 16 * mw + (i >> 1);
    };
    half8 blc[NBP], bln[NBP];
    int cur = next_pair();
    int nxt = cur >= 0 ? next_pair() : -1;
    auto to_lds = [&](int m, const half8 (&blk)[NBP]) __attribute__((always_inline)) {
      if constexpr (!kMfma) {
        wave_sync();
#pragma unroll
        for (int b = 0; b < NBP; ++b) ring_store(G.kbA0 + m + b, blk[b]);
        wave_sync();
      }
    };
    if (cur >= 0) {
#pragma unroll
      for (int b = 0; b < NBP; ++b) blc[b] = load_block(G.kbA0 + cur + b);
      to_lds(cur, blc);
    }
    while (cur >= 0) {
      if (nxt >= 0) {
#pragma unroll
        for (int b = 0; b < NBP; ++b) bln[b] = load_block(G.kbA0 + nxt + b);
      }
      pair_epi(cur, blc);
      cur = nxt;
      nxt = cur >= 0 ? next_pair() : -1;
      if (cur >= 0) {
#pragma unroll
        for (int b = 0; b < NBP; ++b) blc[b] = bln[b];
        to_lds(cur, blc);
      }
    }
  }
  // merge the four lanes of each pixel: larger maximum wins (lower depth on
  // ties); the other's sums are rescaled and re-centred on the winner
#pragma unroll
  for (int xm = 16; xm <= 32; xm <<= 1) {
    const float oR = __shfl_xor(R, xm), oref = __shfl_xor(ref, xm);
    const float o0 = __shfl_xor(S0, xm), o1 = __shfl_xor(S1, xm), o2 = __shfl_xor(S2, xm);
    const bool other = (oR > R) || (oR == R && oref < ref);
    const float wR = other ? oR : R, wref = other ? oref : ref;
    auto bring = [&](float r, float rf, float& s0, float& s1, float& s2) __attribute__((always_inline)) {
      const float sc = (r == -INFINITY) ? 0.f : fast_exp2(r - wR);
      s0 *= sc;
      s1 *= sc;
      s2 *= sc;
      const float delta = rf - wref;
      s2 = fmaf(delta, fmaf(2.f, s1, delta * s0), s2);
      s1 = fmaf(delta, s0, s1);
    };
    float a0 = S0, a1 = S1, a2 = S2, b0 = o0, b1 = o1, b2 = o2;
    bring(R, ref, a0, a1, a2);
    bring(oR, oref, b0, b1, b2);
    S0 = a0 + b0;
    S1 = a1 + b1;
    S2 = a2 + b2;
    R = wR;
    ref = wref;
  }
  const float mu = S1 / S0;
  const int dstar = (int)ref;
  const float mean = ref + mu;
  const float var = fmaxf(S2 / S0 - mu * mu, 0.f);

  // ============================ a6 + a7 ============================
  const float pi_now = faulty ? 0.5f : (io.pi_in && valid ? io.pi_in[p] : 1.0f);
  const bool detected = pi_now > 0.5f;
  float r_hat = 0.f, b_hat = K / (float)M.T;
  if (faulty) b_hat = io.pb[p];
  // window taps j = g + 4 u of the pixel, kept in registers
  constexpr int U = 8 * NBP;  // W <= 32 NBP - 30 by construction of NBP
  float ws[U], wz[U];
  float S = 0.f, Kw = 0.f, nw = 0.f;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = g + 4 * u;
    const int t = dstar - M.c + j;
    const bool in = j < M.W && t >= 0 && t < M.T;
    wz[u] = (in && has_data) ? half_bits_to_float(row[t]) : 0.f;
    ws[u] = in ? sh_irf[j] : 0.f;
    S += ws[u];
    Kw += wz[u];
    nw += in ? 1.f : 0.f;
  }
  S = group_sum<16, 32>(S);
  Kw = group_sum<16, 32>(Kw);
  nw = group_sum<16, 32>(nw);
  if (has_data && detected) {
    auto terms = [&](float r, float b, float SoT, float& g1, float& g2) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (wz[u] > 0.f) {
          const float q = (ws[u] - SoT) * fast_rcp(fmaf(r, ws[u], b));
          g1 = fmaf(wz[u], q, g1);
          g2 = fmaf(-wz[u] * q, q, g2);
        }
      }
    };
    mle_reflectivity<16, 32>(terms, K, S, Kw, nw, (float)M.T, r_hat, b_hat);
  }

  if (valid && g == 0) {
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
  }
}

static int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

bool tile_geometry(const DevModel& M, int engine, TileGeom& G) {
  if (M.T % 8 != 0) return false;
  G = TileGeom{};
  G.o = ((M.d_lo - M.c) % 32 + 32) % 32;
  G.kbA0 = floor_div(M.d_lo - M.c, 32);
  G.nbp = (G.o + 30 + M.W) / 32 + 1;
  if (G.nbp > kTileMaxNBP) return false;
  if (G.nbp < 2) G.nbp = 2;
  G.npairs = (M.D + 31) / 32;
  G.ntiles = (M.D + 15) / 16;
  G.mask_words = (G.ntiles + 31) / 32;
  G.nkb = (M.T + 31) / 32;
  G.kb_last = G.kbA0 + G.npairs - 1 + G.nbp - 1;
  G.nbc = (M.cols + 3) / 4;
  G.nblk = ((M.rows + 3) / 4) * G.nbc;
  G.lds_fixed = ((M.W * 4 + 15) / 16) * 16;
  G.mask_bytes = ((G.mask_words * 4 + 15) / 16) * 16;
  G.halo_bytes = 448;
  G.ring_bytes = engine == kEngValu ? 16 * kRingT * 2 : 0;
  G.lds_per_wave = G.mask_bytes + G.halo_bytes + G.ring_bytes;
  if (engine == kEngValu && 32 * (G.nbp) > kRingT) return false;
  return (size_t)G.lds_fixed + 4 * (size_t)G.lds_per_wave <= 65536;
}

template <int kEng, bool kCost>
static hipError_t launch_nbp(const DevModel& M, const TileGeom& G, const StepIO& io, float* ell,
                             hipStream_t s) {
  const dim3 grid((G.nblk + 3) / 4), block(256);
  const size_t lds = G.lds_fixed + 4 * (size_t)G.lds_per_wave;
  switch (G.nbp) {
    case 2: hipLaunchKernelGGL((k_step_tile<kEng, 2, kCost>), grid, block, lds, s, M, G, io, ell); break;
    case 3: hipLaunchKernelGGL((k_step_tile<kEng, 3, kCost>), grid, block, lds, s, M, G, io, ell); break;
    case 4: hipLaunchKernelGGL((k_step_tile<kEng, 4, kCost>), grid, block, lds, s, M, G, io, ell); break;
    case 5: hipLaunchKernelGGL((k_step_tile<kEng, 5, kCost>), grid, block, lds, s, M, G, io, ell); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step_tile(const DevModel& M, int engine, const StepIO& io, hipStream_t s) {
  TileGeom G;
  if (!tile_geometry(M, engine, G)) return hipErrorInvalidValue;
  switch (engine) {
    case kEngValu: return launch_nbp<kEngValu, false>(M, G, io, nullptr, s);
    case kEngMfma16: return launch_nbp<kEngMfma16, false>(M, G, io, nullptr, s);
    case kEngMfma16x2: return launch_nbp<kEngMfma16x2, false>(M, G, io, nullptr, s);
  }
  return hipErrorInvalidValue;
}

// a3 alone through the tile engines: the pixels are taken as a column of
// 4x4 blocks of an npix x 1 frame, i.e. consecutive rows of 16 pixels.
hipError_t launch_cost_tile(const DevModel& M0, int engine, const uint16_t* hist, int npix,
                            float* ell, hipStream_t s) {
  // the npix histograms are viewed as a frame of 4 columns, so that 4x4 block
  // g holds pixels 16 g .. 16 g + 15 (rows past npix are masked)
  DevModel M = M0;
  M.cols = 4;
  M.rows = (npix + 3) / 4;
  M.P = npix;
  TileGeom G;
  if (!tile_geometry(M, engine, G)) return hipErrorInvalidValue;
  StepIO io{};
  io.hist = hist;
  switch (engine) {
    case kEngValu: return launch_nbp<kEngValu, true>(M, G, io, ell, s);
    case kEngMfma16: return launch_nbp<kEngMfma16, true>(M, G, io, ell, s);
    case kEngMfma16x2: return launch_nbp<kEngMfma16x2, true>(M, G, io, ell, s);
  }
  return hipErrorInvalidValue;
}

bool tile_supported(const DevModel& M, int engine) {
  TileGeom G;
  return tile_geometry(M, engine, G);
}

}  // namespace r3d
