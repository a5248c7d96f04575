// Per-frame step on fp16 histograms, one wavefront per 4x4 pixel block, in
// two passes that can run a frame apart.
//
// Cost (a3). For a 16-bin depth tile [d0, d0+16) the cost of the 16 pixels is
// a banded Toeplitz product C[d][p] = sum_t H[d][t] Z[t][p] with
// H[d][t] = irf^beta[t - d + c]. Bins are taken in 32-bin blocks aligned to
// multiples of 32, so H only depends on (d0 - c) mod 32, which takes two
// values for the two tiles of each 32-bin pair: the A operands of every
// (tile-of-pair, block) combination are built once per workgroup, and each
// histogram block (the B operand: 8 fp16 counts of one pixel per lane, the
// matrix core's 16x16x32 layout) is loaded once into a register ring and
// used by every tile whose band touches it. Engines: fp16 matrix cores with
// irf^beta in fp16 (kEngMfma16); the same with irf^beta split into hi*2^11
// and lo = (irf^beta - hi)*2^11 contracted into one fp32 accumulator
// (kEngMfma16x2); fp32 vector FMAs from an LDS copy of the blocks (kEngValu,
// the plain form).
//
// Bound pass. Streams every block of the frame and keeps, per pixel, the
// maximum of the cost over the grid (matrix engines: of the fp16-hi part,
// which bounds the exact cost within a relative 2^-10 plus K 2^-24) and the
// photon count K. It reads nothing of the filter state, so the bounds of
// frame n+1 can be computed while frame n is resolved.
//
// Resolve pass (a4..a7). The prior mixture of each pixel comes from the
// previous states of the block's 6x6 halo. With lmax the cost bound, the
// exact cost at a reference depth d_ref (the rounded mean of the pixel's own
// prior component, gathered directly in fp32) and L = ell + log f the log2
// pseudo-posterior, its maximum L* satisfies
//   L* >= max(lmax + min_grid log f, ell(d_ref) + log f(d_ref)),
// and L(d) <= lmax + max_k q_k(d) + log2(9). Per prior component this leaves
// the interval of depths where L can reach L* - 160 (log2 units): outside
// every interval exp2(L - L*) is below the smallest fp32 denormal, so those
// depths contribute exactly zero weight and cannot be the argmax. The 16-bin
// tiles meeting any pixel's interval are candidates; the blocks their pairs
// read are streamed once through a register ring, the exact cost is
// recomputed on the candidate tiles, and the argmax and the centred moments
// are accumulated online (running maximum with rescaled, re-centred sums;
// the four lanes of a pixel merge with a symmetric rule, so all of them hold
// bit-identical results). Then the state update (a6) and the reflectivity /
// background MLE (a7).
#include "r3d_device.hpp"
#include "r3d_tile.hpp"

namespace r3d {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kRingT = 256;            // LDS ring per pixel (fp16 bins), VALU engine
constexpr float kCullMargin2 = 160.f;  // log2 units: exp2(-150) rounds to zero in fp32
constexpr float kLog2Nine = 3.16992500144231236f;
constexpr float kLiveGap = 40.f;        // log2 units
constexpr unsigned kOob = 0x80000000u;  // buffer offset past every record: loads return zeros
constexpr int kBufWord3 = 0x00020000;   // raw buffer descriptor, 32-bit data format
constexpr int kHaloBytes = 448;         // 6x6 halo of (m, v, pi), 108 floats
constexpr int kCompBytes = 9 * 3 * 16 * 4;  // (m, k2, w2) of 9 components x 16 pixels

// blocks in flight per wavefront (beyond the blocks of the current pair)
template <int kEng> struct TilePF {
  static constexpr int bound = kEng == kEngValu ? 3 : 10;
  static constexpr int resolve = kEng == kEngValu ? 3 : 5;
};

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
// candidate and these blocks the slowest to resolve), then the interior row
// by row.
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

// The lane's pixel (column i16 of the 16-pixel tile) of block idx and its
// histogram row, read through a buffer descriptor based at the block's first
// pixel: an offset past the records (a pixel outside the frame, a faulty
// pixel, a block outside [0, T)) reads zeros.
struct LanePix {
  int br, bc, p;
  bool valid, faulty, has_data;
  __amdgpu_buffer_rsrc_t hbuf;
  unsigned off;
};

__device__ __forceinline__ LanePix lane_pixel(const DevModel& M, const TileGeom& G,
                                              const uint16_t* hist, const uint8_t* faulty,
                                              int idx, int i16, int g) {
  LanePix L;
  int br, bc;
  block_of(idx, G.nblk / G.nbc, G.nbc, br, bc);
  L.br = __builtin_amdgcn_readfirstlane(br);
  L.bc = __builtin_amdgcn_readfirstlane(bc);
  const int pr = 4 * L.br + (i16 >> 2), pc = 4 * L.bc + (i16 & 3);
  L.valid = pr < M.rows && pc < M.cols && pr * M.cols + pc < M.P;
  L.p = L.valid ? pr * M.cols + pc : 0;
  L.faulty = L.valid && faulty && faulty[L.p];
  L.has_data = L.valid && !L.faulty;
  const int p0 = __builtin_amdgcn_readfirstlane((4 * L.br) * M.cols + 4 * L.bc);
  const long long rec = (long long)(M.P - p0) * M.T * 2;
  L.hbuf = __builtin_amdgcn_make_buffer_rsrc((void*)(hist + (size_t)p0 * M.T), (short)0,
                                             (int)(rec < 0x7fffffffLL ? rec : 0x7fffffffLL),
                                             kBufWord3);
  L.off = L.has_data ? (unsigned)(((L.p - p0) * M.T + 8 * g) * 2) : kOob;
  return L;
}

// Block kb (bins 32 kb .. 32 kb + 31) of the lane's pixel, 8 bins per lane.
__device__ __forceinline__ half8 load_block(const DevModel& M, const LanePix& L, int g, int kb) {
  const bool in = kb >= 0 && 32 * kb + 8 * g < M.T && L.off != kOob;
  const unsigned off = in ? L.off + 64u * (unsigned)kb : kOob;
  return __builtin_bit_cast(half8, __builtin_amdgcn_raw_buffer_load_b128(L.hbuf, off, 0, 0));
}

// A load past every record: zeros, no memory traffic (keeps the count of
// loads in flight regular where a stream has run out of blocks).
__device__ __forceinline__ half8 load_nothing(const LanePix& L) {
  return __builtin_bit_cast(half8, __builtin_amdgcn_raw_buffer_load_b128(L.hbuf, kOob, 0, 0));
}

// A operand of (part, tile-of-pair tau, block b) for this lane, in LDS:
// part 0 = irf^beta in fp16 (times 2^11 for the split engine), part 1 = the
// split engine's low part.
__device__ __forceinline__ const half8& a_op(const half8* sA, int nbp, int part, int tau, int b,
                                             int lane) {
  return sA[((part * 2 + tau) * nbp + b) * 64 + lane];
}

// fp32 cost of tile tau of pair m from the LDS ring (VALU engine): the lane
// computes its 4 depths d = d_lo + 32 m + 16 tau + 4 g + q.
__device__ __forceinline__ floatx4 valu_tile(const DevModel& M, const _Float16* ring_lds, int i16,
                                             int g, int m, int tau) {
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
}

__device__ __forceinline__ void ring_store(_Float16* ring_lds, int i16, int g, int kb, half8 v) {
  *reinterpret_cast<half8*>(ring_lds + i16 * kRingT + ((32 * kb + 8 * g) & (kRingT - 1))) = v;
}

// Exact cost of both tiles of pair m from its NBP blocks: fp16 hi (and lo)
// contractions in independent chains, or fp32 from the LDS ring.
template <int kEng, int NBP>
__device__ __forceinline__ void pair_cost(const DevModel& M, const half8* sA, const _Float16* ring_lds,
                                          int lane, int m, const half8 (&blk)[NBP], floatx4& c0,
                                          floatx4& c1) {
  if constexpr (kEng != kEngValu) {
    floatx4 h0 = {0.f, 0.f, 0.f, 0.f}, h1 = h0, l0 = h0, l1 = h0;
#pragma unroll
    for (int b = 0; b < NBP; ++b) {
      h0 = mfma16(a_op(sA, NBP, 0, 0, b, lane), blk[b], h0);
      h1 = mfma16(a_op(sA, NBP, 0, 1, b, lane), blk[b], h1);
      if constexpr (kEng == kEngMfma16x2) {
        l0 = mfma16(a_op(sA, NBP, 1, 0, b, lane), blk[b], l0);
        l1 = mfma16(a_op(sA, NBP, 1, 1, b, lane), blk[b], l1);
      }
    }
    if constexpr (kEng == kEngMfma16x2) {
      c0 = h0 + l0;
      c1 = h1 + l1;
    } else {
      c0 = h0;
      c1 = h1;
    }
  } else {
    c0 = valu_tile(M, ring_lds, lane & 15, lane >> 4, m, 0);
    c1 = valu_tile(M, ring_lds, lane & 15, lane >> 4, m, 1);
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
    C.w2[k] = M.lognu2[k] - 0.5f * (kLog2TwoPi + fast_log2(V));
  }
  merge_components(C);
}

// ============================ bound pass ============================
// Streams every pair of the block through the ring (the blocks of the
// current pair plus PF prefetched ones), counts photons, validates counts,
// and writes (lmax, K) per pixel. The cost is >= 0, so its fp32 maximum is
// the integer maximum of the bit patterns.
template <int kEng, int NBP>
__device__ __forceinline__ void bound_block(const DevModel& M, const TileGeom& G,
                                            const uint16_t* hist, const uint8_t* faulty,
                                            TileBound* __restrict__ bound, int idx,
                                            const half8 (&Ahi)[2][NBP], _Float16* ring_lds,
                                            int lane) {
  constexpr bool kMfma = kEng != kEngValu;
  constexpr int RING = NBP + TilePF<kEng>::bound;
  const int i16 = lane & 15, g = lane >> 4;
  const LanePix L = lane_pixel(M, G, hist, faulty, idx, i16, g);

  float Kv = 0.f;
  floatx4 Kacc = {0.f, 0.f, 0.f, 0.f};  // photon count via a ones-row contraction
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
  auto fetch = [&](int kb) __attribute__((always_inline)) -> half8 {
    return load_block(M, L, g, kb <= G.kb_last ? kb : -1);
  };

  unsigned lmax_bits = 0u;
  half8 ring[RING];
#pragma unroll
  for (int x = 0; x < RING - 1; ++x) ring[x] = fetch(G.kbA0 + x);
  for (int m0 = 0; m0 < G.npairs; m0 += RING) {
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      const int m = m0 + u;
      ring[(u + RING - 1) % RING] = fetch(G.kbA0 + m + RING - 1);
      if (m < G.npairs) {
      if constexpr (!kMfma) {
        wave_sync();
        if (m == 0) {
#pragma unroll
          for (int b = 0; b < NBP; ++b) ring_store(ring_lds, i16, g, G.kbA0 + b, ring[(u + b) % RING]);
        } else {
          ring_store(ring_lds, i16, g, G.kbA0 + m + NBP - 1, ring[(u + NBP - 1) % RING]);
        }
        wave_sync();
      }
      if (m == 0) {
#pragma unroll
        for (int b = 0; b < NBP - 1; ++b) account(ring[(u + b) % RING]);
      }
      account(ring[(u + NBP - 1) % RING]);
      floatx4 c0, c1;
      if constexpr (kMfma) {
        c0 = floatx4{0.f, 0.f, 0.f, 0.f};
        c1 = c0;
#pragma unroll
        for (int b = 0; b < NBP; ++b) {
          c0 = mfma16(Ahi[0][b], ring[(u + b) % RING], c0);
          c1 = mfma16(Ahi[1][b], ring[(u + b) % RING], c1);
        }
      } else {
        c0 = valu_tile(M, ring_lds, i16, g, m, 0);
        c1 = valu_tile(M, ring_lds, i16, g, m, 1);
      }
      const unsigned a = __builtin_elementwise_max(__float_as_uint(c0[0]), __float_as_uint(c0[1]));
      const unsigned b = __builtin_elementwise_max(__float_as_uint(c0[2]), __float_as_uint(c0[3]));
      const unsigned c = __builtin_elementwise_max(__float_as_uint(c1[0]), __float_as_uint(c1[1]));
      const unsigned d = __builtin_elementwise_max(__float_as_uint(c1[2]), __float_as_uint(c1[3]));
      lmax_bits = __builtin_elementwise_max(lmax_bits, __builtin_elementwise_max(
                      __builtin_elementwise_max(a, b), __builtin_elementwise_max(c, d)));
      }
    }
  }
  // blocks of [0, T) that no depth window reaches still hold photons
  for (int kb = 0; kb < G.nkb; ++kb) {
    if (kb >= G.kbA0 && kb <= G.kb_last) continue;
    account(load_block(M, L, g, kb));
  }
  unsigned bad = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s) bad |= vmax[s] > 0x6800u ? kErrOverflow : 0u;  // > 2048 or negative
  if (bad) atomicOr(M.err, bad);

  const float K = kMfma ? Kacc[0] : group_sum<16, 32>(Kv);
  lmax_bits = max(lmax_bits, (unsigned)__shfl_xor((int)lmax_bits, 16));
  lmax_bits = max(lmax_bits, (unsigned)__shfl_xor((int)lmax_bits, 32));
  if (L.valid && g == 0) bound[L.p] = make_float2(__uint_as_float(lmax_bits), K);
}

// ============================ resolve pass ============================
// A resolve workgroup takes the four blocks w * nr + j (w = its wavefronts),
// so the border blocks, first in block order, land one per workgroup. Each
// wavefront prepares its own block (prior, bounds, candidate masks, all in
// its LDS region); the candidate pairs of a block are then evaluated by its
// own wavefront, except for blocks with many needed histogram blocks (the
// border blocks, whose flat prior components make every depth a candidate),
// whose stream is split into four consecutive ranges, one per wavefront of
// the workgroup. Partial moments are merged in wavefront order, so the
// result depends only on the inputs.
constexpr int kSplitMin = 24;  // needed blocks above which a block is shared

// Online argmax and centred moments of the log2 pseudo-posterior: running
// maximum R at depth ref and sums S0 = sum w, S1 = sum w (d - ref),
// S2 = sum w (d - ref)^2 with w = exp2(L - R).
struct Moments {
  float R, ref, S0, S1, S2;
};

// Merge b into a with a symmetric rule: the larger maximum wins (the lower
// depth on ties); the other's sums are rescaled and re-centred on it.
__device__ __forceinline__ void merge_moments(Moments& a, const Moments& b) {
  const float aR = a.R, aref = a.ref, bR = b.R, bref = b.ref;
  const bool other = (bR > aR) || (bR == aR && bref < aref);
  const float wR = other ? bR : aR, wref = other ? bref : aref;
  const float sa = aR == -INFINITY ? 0.f : fast_exp2(aR - wR);
  const float sb = bR == -INFINITY ? 0.f : fast_exp2(bR - wR);
  float a0 = a.S0 * sa, a1 = a.S1 * sa, a2 = a.S2 * sa;
  float b0 = b.S0 * sb, b1 = b.S1 * sb, b2 = b.S2 * sb;
  const float da = aref - wref, db = bref - wref;
  a2 = fmaf(da, fmaf(2.f, a1, da * a0), a2);
  a1 = fmaf(da, a0, a1);
  b2 = fmaf(db, fmaf(2.f, b1, db * b0), b2);
  b1 = fmaf(db, b0, b1);
  a.S0 = a0 + b0;
  a.S1 = a1 + b1;
  a.S2 = a2 + b2;
  a.R = wR;
  a.ref = wref;
}

// Per-wavefront LDS region of a resolved block.
struct BlockLds {
  unsigned *tmask, *pmask, *nmask;
  int* trange;  // [0..8] first and [9..17] last tile of each component's live range
  float* halo;
  float* comp;  // (m, k2, w2) of each component, comp[(3 k + f) * 16 + i16]
  _Float16* ring;
};

__device__ __forceinline__ BlockLds block_lds(const TileGeom& G, unsigned char* wbase) {
  BlockLds B;
  B.tmask = reinterpret_cast<unsigned*>(wbase);
  B.pmask = B.tmask + G.mask_words;
  B.nmask = B.pmask + G.pair_words;
  B.trange = reinterpret_cast<int*>(wbase + G.off_trange);
  B.halo = reinterpret_cast<float*>(wbase + G.off_halo);
  B.comp = reinterpret_cast<float*>(wbase + G.off_comp);
  B.ring = reinterpret_cast<_Float16*>(wbase + G.off_ring);
  return B;
}

// Prior, bounds and candidate masks of block idx into its LDS region;
// returns the number of needed histogram blocks (wave-uniform).
template <int kEng, int NBP>
__device__ __forceinline__ int resolve_prep(const DevModel& M, const TileGeom& G, const StepIO& io,
                                            const TileBound* __restrict__ bound, int idx,
                                            const float* sh_h, const BlockLds& B, int lane) {
  constexpr bool kMfma = kEng != kEngValu;
  constexpr bool kSplit = kEng == kEngMfma16x2;
  // taps per lane (j = g + 4 u): W <= 32 NBP - 30 by construction of NBP, so u < 8 NBP - 7
  constexpr int U = 8 * NBP - 7;
  const int i16 = lane & 15, g = lane >> 4;
  const LanePix L = lane_pixel(M, G, io.hist, io.faulty, idx, i16, g);
  const int dhi = M.d_lo + M.D - 1;
  const uint16_t* row = io.hist + (size_t)L.p * M.T;

  // previous states of the block's 6x6 halo
  if (lane < 36) {
    const int hr = 4 * L.br - 1 + lane / 6, hc = 4 * L.bc - 1 + lane % 6;
    float hm = 0.f, hv = 1.f, hp = -1.f;
    if (hr >= 0 && hr < M.rows && hc >= 0 && hc < M.cols) {
      const int q = hr * M.cols + hc;
      hm = io.pm[q];
      hv = io.pv[q];
      hp = io.ppi[q];
    }
    B.halo[lane] = hm;
    B.halo[36 + lane] = hv;
    B.halo[72 + lane] = hp;
  }
  float lmax = 0.f, K = 0.f;
  // reference depth: the rounded mean of the pixel's own prior component,
  // read directly so that the gather of its cost starts at once
  float mown = M.m_flat;
  if (L.valid) {
    const TileBound bv = bound[L.p];
    lmax = bv.x;
    K = bv.y;
    const float pm = io.pm[L.p];
    mown = io.ppi[L.p] > 0.5f ? pm : M.m_flat;
  }
  const int dref = (int)fminf(fmaxf(rintf(mown), (float)M.d_lo), (float)dhi);
  // exact cost at d_ref by an fp32 gather (the lane takes taps j = g + 4 u)
  float zr[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = g + 4 * u;
    const int t = dref - M.c + j;
    zr[u] = (L.has_data && j < M.W && t >= 0 && t < M.T) ? half_bits_to_float(row[t]) : 0.f;
  }
  if constexpr (kMfma) lmax = lmax * (1.0f + 0x1p-9f) + K * (kSplit ? 2048.0f : 1.0f) * 0x1p-23f;
  const float cs2 = M.scale2 * (kSplit ? (1.0f / 2048.0f) : 1.0f);  // raw cost -> log2 units
  wave_sync();

  Comps C;
  halo_components(M, B.halo, i16, C);
  float lref = 0.f;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = g + 4 * u;
    if (j < M.W) lref = fmaf(sh_h[j], zr[u], lref);
  }
  lref = group_sum<16, 32>(lref);

  const float l2max = lmax * cs2;
  float lbf = -INFINITY;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float e = fmaxf(fabsf((float)M.d_lo - C.m[k]), fabsf((float)dhi - C.m[k]));
    lbf = fmaxf(lbf, C.w2[k] - e * e * C.k2[k]);
  }
  unsigned wave_live = 0u;
#pragma unroll
  for (int k = 0; k < 9; ++k) wave_live |= (__any(L.valid && (C.live >> k & 1u)) ? 1u : 0u) << k;
  float Llb = l2max + lbf;
  if (L.valid) Llb = fmaxf(Llb, fmaf(lref, M.scale2, log_prior2(C, (float)dref, wave_live)));
  const float theta = Llb - kCullMargin2 - l2max - kLog2Nine;

  // Component k is "live" on depths where q_k >= theta - kLiveGap: at a
  // candidate depth some component reaches theta, so components below
  // theta - kLiveGap change f by less than 9 * 2^-kLiveGap relative and are
  // skipped; depths where no component is live are not candidates at all.
  // The block keeps, per component, the tile range covering every pixel's
  // live interval (LDS min / max over the pixels).
  if (lane < 9) {
    B.trange[lane] = 0x7fffffff;
    B.trange[9 + lane] = -1;
  }
  wave_sync();
  if (L.valid && g == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if (!(C.w2[k] >= theta - kLiveGap)) continue;
      const float R = sqrtf((C.w2[k] - theta + kLiveGap) / C.k2[k]) + 2.0f;
      const float lo = fmaxf(C.m[k] - R, (float)M.d_lo);
      const float hi = fminf(C.m[k] + R, (float)dhi);
      if (!(lo <= hi)) continue;
      atomicMin(&B.trange[k], ((int)floorf(lo) - M.d_lo) >> 4);
      atomicMax(&B.trange[9 + k], ((int)ceilf(hi) - M.d_lo) >> 4);
    }
  }

  // candidate tiles and pairs (LDS bit masks, or-ed by the lanes)
  const int nwords = G.mask_words + G.pair_words + G.need_words;
  for (int w = lane; w < nwords; w += 64) B.tmask[w] = 0u;
  wave_sync();
  auto set_bits = [&](unsigned* mk, int a0, int z0) __attribute__((always_inline)) {
    for (int w = a0 >> 5; w <= (z0 >> 5); ++w) {
      const int a = w == (a0 >> 5) ? (a0 & 31) : 0;
      const int z = w == (z0 >> 5) ? (z0 & 31) : 31;
      const unsigned bits = (z == 31 ? 0xffffffffu : ((1u << (z + 1)) - 1u)) & ~((1u << a) - 1u);
      atomicOr(&mk[w], bits);
    }
  };
  if (L.valid) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if ((k & 3) != g || !(C.w2[k] >= theta)) continue;
      const float R = sqrtf((C.w2[k] - theta) / C.k2[k]) + 2.0f;
      const float lo = fmaxf(floorf(C.m[k] - R), (float)M.d_lo);
      const float hi = fminf(ceilf(C.m[k] + R), (float)dhi);
      if (!(lo <= hi)) continue;
      const int ta = ((int)lo - M.d_lo) >> 4, tb = ((int)hi - M.d_lo) >> 4;
      set_bits(B.tmask, ta, tb);
      set_bits(B.pmask, ta >> 1, tb >> 1);
    }
  }
  // the pixels' components, component-major
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      B.comp[(3 * k + 0) * 16 + i16] = C.m[k];
      B.comp[(3 * k + 1) * 16 + i16] = C.k2[k];
      B.comp[(3 * k + 2) * 16 + i16] = C.w2[k];
    }
  }
  wave_sync();
  // blocks read by the candidate pairs: block kbA0 + r is needed when a
  // candidate pair starts at one of r - NBP + 1 .. r
  for (int w = lane; w < G.need_words; w += 64) {
    const unsigned cur = w < G.pair_words ? B.pmask[w] : 0u;
    const unsigned prev = (w > 0 && w - 1 < G.pair_words) ? B.pmask[w - 1] : 0u;
    unsigned acc = cur;
#pragma unroll
    for (int k = 1; k < NBP; ++k) acc |= (cur << k) | (prev >> (32 - k));
    B.nmask[w] = acc;
  }
  wave_sync();
  int nneed = 0;
  for (int w = 0; w < G.need_words; ++w)
    nneed += __builtin_popcount(__builtin_amdgcn_readfirstlane(B.nmask[w]));
  return nneed;
}

// Evaluate the candidate pairs of block idx whose first block is at
// positions [pos_lo, pos_hi) of its needed-block stream, accumulating into
// mo. The block's masks, tile ranges and components come from its LDS region
// B (prepared by its own wavefront); any wavefront may run this.
template <int kEng, int NBP>
__device__ __forceinline__ void resolve_range(const DevModel& M, const TileGeom& G,
                                              const StepIO& io, int idx, const half8* sA,
                                              const BlockLds& B, _Float16* ring_lds, int pos_lo,
                                              int pos_hi, Moments& mo, int lane) {
  constexpr bool kMfma = kEng != kEngValu;
  constexpr bool kSplit = kEng == kEngMfma16x2;
  constexpr int RING = NBP + TilePF<kEng>::resolve;
  const int i16 = lane & 15, g = lane >> 4;
  const LanePix L = lane_pixel(M, G, io.hist, io.faulty, idx, i16, g);
  const int dhi = M.d_lo + M.D - 1;
  const float cs2 = M.scale2 * (kSplit ? (1.0f / 2048.0f) : 1.0f);
  // lane k < 9 holds component k's tile range (empty elsewhere), so the set
  // of components live in a tile is one ballot
  const int TAv = lane < 9 ? B.trange[lane] : 1, TBv = lane < 9 ? B.trange[9 + lane] : 0;
  const float* comp = B.comp;

  auto is_cand = [&](const unsigned* mk, int i) __attribute__((always_inline)) -> bool {
    return (__builtin_amdgcn_readfirstlane(mk[i >> 5]) >> (i & 31)) & 1u;
  };
  // log2 pseudo-posterior of the lane's 4 depths of tile dt, online moments
  auto tile_epi = [&](const floatx4& acc, int dt) __attribute__((always_inline)) {
    const int dbase = M.d_lo + 16 * dt + 4 * g;
    const unsigned tmk = (unsigned)__ballot(TAv <= dt && dt <= TBv) & 0x1ffu;
    // log2 f by an online log-sum-exp over the live components
    float mx[4], sm[4];
    unsigned bits = tmk;
    const bool single = __builtin_popcount(tmk) == 1;
    {
      const int k = bits ? __builtin_ctz(bits) : 0;
      bits &= bits - 1u;
      const float mk = comp[(3 * k) * 16 + i16], kk = comp[(3 * k + 1) * 16 + i16];
      const float wk = tmk ? comp[(3 * k + 2) * 16 + i16] : -INFINITY;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float e = (float)(dbase + q) - mk;
        mx[q] = fmaf(-e * e, kk, wk);
        sm[q] = 1.f;
      }
    }
    while (bits) {
      const int k = __builtin_ctz(bits);
      bits &= bits - 1u;
      const float mk = comp[(3 * k) * 16 + i16], kk = comp[(3 * k + 1) * 16 + i16];
      const float wk = comp[(3 * k + 2) * 16 + i16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float e = (float)(dbase + q) - mk;
        const float qv = fmaf(-e * e, kk, wk);
        const float nm = fmaxf(mx[q], qv);
        const float sa = nm == -INFINITY ? 0.f : fast_exp2(mx[q] - nm);
        const float sb = nm == -INFINITY ? 0.f : fast_exp2(qv - nm);
        sm[q] = fmaf(sm[q], sa, sb);
        mx[q] = nm;
      }
    }
    float Lq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float lp = (single || mx[q] == -INFINITY) ? mx[q] : mx[q] + fast_log2(sm[q]);
      Lq[q] = (L.valid && dbase + q <= dhi) ? fmaf(acc[q], cs2, lp) : -INFINITY;
    }
    float mt = Lq[0];
    int qt = 0;
#pragma unroll
    for (int q = 1; q < 4; ++q)
      if (Lq[q] > mt) {
        mt = Lq[q];
        qt = q;
      }
    if (mt > mo.R) {
      const float sc = fast_exp2(mo.R - mt);
      const float dnew = (float)(dbase + qt);
      const float delta = mo.ref - dnew;
      mo.S0 *= sc;
      mo.S1 *= sc;
      mo.S2 *= sc;
      mo.S2 = fmaf(delta, fmaf(2.f, mo.S1, delta * mo.S0), mo.S2);
      mo.S1 = fmaf(delta, mo.S0, mo.S1);
      mo.R = mt;
      mo.ref = dnew;
    }
    if (mt > -INFINITY) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float wq = fast_exp2(Lq[q] - mo.R);
        const float e = (float)(dbase + q) - mo.ref;
        mo.S0 += wq;
        mo.S1 = fmaf(e, wq, mo.S1);
        mo.S2 = fmaf(e * e, wq, mo.S2);
      }
    }
  };

  // Cursors over the set bits of the needed mask (wave-uniform), both
  // starting at position pos_lo.
  int lw = 0, skipped = 0;
  unsigned lbits = G.need_words > 0 ? __builtin_amdgcn_readfirstlane(B.nmask[0]) : 0u;
  while (lw < G.need_words) {
    const int c = __builtin_popcount(lbits);
    if (skipped + c > pos_lo) break;
    skipped += c;
    if (++lw < G.need_words) lbits = __builtin_amdgcn_readfirstlane(B.nmask[lw]);
  }
  for (; skipped < pos_lo && lw < G.need_words; ++skipped) lbits &= lbits - 1u;
  int ew = lw;
  unsigned ebits = lbits;
  auto next_needed = [&](int& w, unsigned& bits) __attribute__((always_inline)) -> int {
    while (bits == 0u) {
      if (++w >= G.need_words) return -1;
      bits = __builtin_amdgcn_readfirstlane(B.nmask[w]);
    }
    const int i = __builtin_ctz(bits);
    bits &= bits - 1u;
    return 32 * w + i;
  };
  // Stream the needed blocks in order through the ring; a candidate pair is
  // evaluated at the position of its first block, whose NBP - 1 successors
  // in the stream are its other blocks (all needed, hence consecutive).
  // Every position issues exactly one load (past the last needed block, a
  // load of nothing that returns zeros without touching memory), so the
  // number of loads in flight after each block is known statically.
  auto fetch = [&](int r) __attribute__((always_inline)) -> half8 {
    return r >= 0 ? load_block(M, L, g, G.kbA0 + r) : load_nothing(L);
  };
  half8 ring[RING];
#pragma unroll
  for (int x = 0; x < RING - 1; ++x) ring[x] = fetch(next_needed(lw, lbits));
  for (int i0 = pos_lo; i0 < pos_hi; i0 += RING) {
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      ring[(u + RING - 1) % RING] = fetch(next_needed(lw, lbits));
      const int m = i0 + u < pos_hi ? next_needed(ew, ebits) : -1;
      if (m >= 0 && m < G.npairs && is_cand(B.pmask, m)) {
        half8 blk[NBP];
#pragma unroll
        for (int b = 0; b < NBP; ++b) blk[b] = ring[(u + b) % RING];
        if constexpr (!kMfma) {
          wave_sync();
#pragma unroll
          for (int b = 0; b < NBP; ++b) ring_store(ring_lds, i16, g, G.kbA0 + m + b, blk[b]);
          wave_sync();
        }
        floatx4 a0, a1;
        pair_cost<kEng, NBP>(M, sA, ring_lds, lane, m, blk, a0, a1);
        if (is_cand(B.tmask, 2 * m)) tile_epi(a0, 2 * m);
        if (is_cand(B.tmask, 2 * m + 1)) tile_epi(a1, 2 * m + 1);
      }
    }
  }
}

// Lane merge, state update (a6) and reflectivity / background (a7) of
// block idx from its merged moments.
template <int kEng, int NBP>
__device__ __forceinline__ void resolve_finish(const DevModel& M, const TileGeom& G,
                                               const StepIO& io, const TileBound* __restrict__ bound,
                                               int idx, const float* sh_irf, Moments mo, int lane) {
  constexpr int U = 8 * NBP - 7;  // taps per lane, as in resolve_prep
  const int i16 = lane & 15, g = lane >> 4;
  const LanePix L = lane_pixel(M, G, io.hist, io.faulty, idx, i16, g);
  const uint16_t* row = io.hist + (size_t)L.p * M.T;
  // the four lanes of each pixel
#pragma unroll
  for (int xm = 16; xm <= 32; xm <<= 1) {
    Moments o;
    o.R = __shfl_xor(mo.R, xm);
    o.ref = __shfl_xor(mo.ref, xm);
    o.S0 = __shfl_xor(mo.S0, xm);
    o.S1 = __shfl_xor(mo.S1, xm);
    o.S2 = __shfl_xor(mo.S2, xm);
    merge_moments(mo, o);
  }
  const float mu = mo.S1 / mo.S0;
  const int dstar = (int)mo.ref;
  const float mean = mo.ref + mu;
  const float var = fmaxf(mo.S2 / mo.S0 - mu * mu, 0.f);
  const float K = L.valid ? bound[L.p].y : 0.f;

  // ============================ a6 + a7 ============================
  const float pi_now = L.faulty ? 0.5f : (io.pi_in && L.valid ? io.pi_in[L.p] : 1.0f);
  const bool detected = pi_now > 0.5f;
  float r_hat = 0.f, b_hat = K / (float)M.T;
  if (L.faulty) b_hat = io.pb[L.p];
  // window taps j = g + 4 u of the pixel, kept in registers
  float ws[U], wz[U];
  float S = 0.f, Kw = 0.f, nw = 0.f;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = g + 4 * u;
    const int t = dstar - M.c + j;
    const bool in = j < M.W && t >= 0 && t < M.T;
    wz[u] = (in && L.has_data) ? half_bits_to_float(row[t]) : 0.f;
    ws[u] = in ? sh_irf[j] : 0.f;
    S += ws[u];
    Kw += wz[u];
    nw += in ? 1.f : 0.f;
  }
  S = group_sum<16, 32>(S);
  Kw = group_sum<16, 32>(Kw);
  nw = group_sum<16, 32>(nw);
  if (L.has_data && detected) {
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

  if (L.valid && g == 0) {
    const int p = L.p;
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

// The resolve role of a workgroup: blocks w * nr + j for its wavefronts w.
template <int kEng, int NBP>
__device__ __forceinline__ void resolve_group(const DevModel& M, const TileGeom& G,
                                              const TileJob& J, int j, const half8* sA,
                                              const float* sh_irf, const float* sh_h,
                                              unsigned char* smem, int wave, int lane) {
  int* s_need = reinterpret_cast<int*>(smem + G.lds_share);
  float* s_part = reinterpret_cast<float*>(smem + G.lds_share + 16);  // [4 waves][5][64 lanes]
  const int idx = wave * J.nr + j;
  const bool mine = idx < G.nblk;
  const BlockLds B = block_lds(G, smem + G.lds_fixed + wave * G.lds_per_wave);
  int nneed = 0;
  if (mine) nneed = resolve_prep<kEng, NBP>(M, G, J.io, J.rbound, idx, sh_h, B, lane);
  if (lane == 0) s_need[wave] = nneed;
  __syncthreads();
  // work items: 0 = the wavefront's own block when it is not shared, then
  // the shared blocks in wavefront order (quarter w of the stream on
  // wavefront w); one call site keeps the code compact
  Moments mo{-INFINITY, 0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < 5; ++it) {
    const int d = it == 0 ? wave : it - 1;
    const int nd = it == 0 ? nneed : s_need[d];
    const int didx = d * J.nr + j;
    if (didx >= G.nblk) continue;
    if (it == 0 ? nd > kSplitMin : nd <= kSplitMin) continue;  // uniform over the workgroup for it > 0
    const BlockLds D = block_lds(G, smem + G.lds_fixed + d * G.lds_per_wave);
    Moments part{-INFINITY, 0.f, 0.f, 0.f, 0.f};
    const int lo = it == 0 ? 0 : (wave * nd) / 4, hi = it == 0 ? nd : ((wave + 1) * nd) / 4;
    resolve_range<kEng, NBP>(M, G, J.io, didx, sA, D, B.ring, lo, hi, part, lane);
    if (it == 0) {
      mo = part;
      continue;
    }
    float* sp = s_part + wave * 5 * 64;
    sp[0 * 64 + lane] = part.R;
    sp[1 * 64 + lane] = part.ref;
    sp[2 * 64 + lane] = part.S0;
    sp[3 * 64 + lane] = part.S1;
    sp[4 * 64 + lane] = part.S2;
    __syncthreads();
    if (wave == d) {
      mo = Moments{s_part[lane], s_part[64 + lane], s_part[128 + lane], s_part[192 + lane],
                   s_part[256 + lane]};
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        const float* q = s_part + w * 5 * 64;
        merge_moments(mo, Moments{q[lane], q[64 + lane], q[128 + lane], q[192 + lane], q[256 + lane]});
      }
    }
    __syncthreads();
  }
  if (mine) resolve_finish<kEng, NBP>(M, G, J.io, J.rbound, idx, sh_irf, mo, lane);
}

// LDS of the workgroup: irf and irf^beta (fp32), the A operands, then each
// wavefront's masks, halo and (VALU engine) histogram ring.
template <int kEng, int NBP>
__device__ __forceinline__ void tile_prologue(const DevModel& M, const TileGeom& G,
                                              unsigned char* smem) {
  float* sh_irf = reinterpret_cast<float*>(smem);
  float* sh_h = sh_irf + M.W;
  for (int j = threadIdx.x; j < M.W; j += blockDim.x) {
    sh_irf[j] = M.irf[j];
    sh_h[j] = M.h[j];
  }
  if constexpr (kEng != kEngValu) {
    half8* sA = reinterpret_cast<half8*>(smem + G.lds_a);
    for (int e = threadIdx.x; e < 2 * 2 * NBP * 64; e += blockDim.x) {
      const int ln = e & 63, b = (e >> 6) % NBP, tau = (e / (64 * NBP)) & 1, part = e / (128 * NBP);
      const int g = ln >> 4, i16 = ln & 15;
      const _Float16* src = part ? M.h16lo : M.h16hi;
      const bool scale = part == 0 && kEng == kEngMfma16x2;
      half8 v;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int j = 32 * b + 8 * g + s - 16 * tau - i16 - G.o;
        const _Float16 x = (j >= 0 && j < M.W) ? src[j] : (_Float16)0.f;
        v[s] = scale ? x * (_Float16)2048.f : x;
      }
      sA[e] = v;  // e == ((part * 2 + tau) * NBP + b) * 64 + ln
    }
  }
  __syncthreads();
}

// One launch: workgroups alternate between the two roles while both have
// work left. Resolve workgroup j takes blocks w * nr + j (w = its
// wavefronts); bound workgroup j's wavefront w takes blocks 4 j + w + 4 nb k.
template <int kEng, int NBP>
__global__ void __launch_bounds__(256, NBP <= 3 ? 4 : 2) k_tile(DevModel M, TileGeom G, TileJob J) {
  extern __shared__ __align__(16) unsigned char smem[];
  tile_prologue<kEng, NBP>(M, G, smem);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float* sh_irf = reinterpret_cast<const float*>(smem);
  const float* sh_h = sh_irf + M.W;
  const half8* sA = reinterpret_cast<const half8*>(smem + G.lds_a);
  unsigned char* wbase = smem + G.lds_fixed + wave * G.lds_per_wave;

  const int i = blockIdx.x, both = J.nr < J.nb ? J.nr : J.nb;
  bool resolve;
  int j;
  if (i < 2 * both) {
    resolve = (i & 1) == 0;
    j = i >> 1;
  } else {
    resolve = J.nr > J.nb;
    j = i - both;
  }
  if (resolve) {
    resolve_group<kEng, NBP>(M, G, J, j, sA, sh_irf, sh_h, smem, wave, lane);
  } else {
    half8 Ahi[2][NBP];
    if constexpr (kEng != kEngValu) {
#pragma unroll
      for (int tau = 0; tau < 2; ++tau)
#pragma unroll
        for (int b = 0; b < NBP; ++b) Ahi[tau][b] = a_op(sA, NBP, 0, tau, b, lane);
    }
    _Float16* ring_lds = reinterpret_cast<_Float16*>(wbase + G.off_ring);
    for (int idx = 4 * j + wave; idx < G.nblk; idx += 4 * J.nb)
      bound_block<kEng, NBP>(M, G, J.bhist, J.bfaulty, J.bbound, idx, Ahi, ring_lds, lane);
  }
}

// a3 alone: the exact cost of every grid depth written out.
template <int kEng, int NBP>
__global__ void __launch_bounds__(256) k_tile_cost(DevModel M, TileGeom G, const uint16_t* hist,
                                                   float* __restrict__ ell) {
  extern __shared__ __align__(16) unsigned char smem[];
  tile_prologue<kEng, NBP>(M, G, smem);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i16 = lane & 15, g = lane >> 4;
  const int idx = blockIdx.x * 4 + wave;
  if (idx >= G.nblk) return;
  const half8* sA = reinterpret_cast<const half8*>(smem + G.lds_a);
  _Float16* ring_lds = reinterpret_cast<_Float16*>(smem + G.lds_fixed + wave * G.lds_per_wave + G.off_ring);
  const LanePix L = lane_pixel(M, G, hist, nullptr, idx, i16, g);
  const float sc = M.scale2 * (kEng == kEngMfma16x2 ? (1.0f / 2048.0f) : 1.0f) * kLn2;
  const int dhi = M.d_lo + M.D - 1;
  for (int m = 0; m < G.npairs; ++m) {
    half8 blk[NBP];
#pragma unroll
    for (int b = 0; b < NBP; ++b) blk[b] = load_block(M, L, g, G.kbA0 + m + b);
    if constexpr (kEng == kEngValu) {
      wave_sync();
#pragma unroll
      for (int b = 0; b < NBP; ++b) ring_store(ring_lds, i16, g, G.kbA0 + m + b, blk[b]);
      wave_sync();
    }
    floatx4 c0, c1;
    pair_cost<kEng, NBP>(M, sA, ring_lds, lane, m, blk, c0, c1);
    if (L.valid) {
#pragma unroll
      for (int tau = 0; tau < 2; ++tau) {
        const int dbase = M.d_lo + 32 * m + 16 * tau + 4 * g;
        const floatx4 acc = tau ? c1 : c0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (dbase + q <= dhi) ell[(size_t)L.p * M.D + (dbase + q - M.d_lo)] = acc[q] * sc;
      }
    }
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
  G.pair_words = (G.npairs + 31) / 32;
  G.need_words = (G.npairs + G.nbp - 1 + 31) / 32;
  G.nkb = (M.T + 31) / 32;
  G.kb_last = G.kbA0 + G.npairs - 1 + G.nbp - 1;
  G.nbc = (M.cols + 3) / 4;
  G.nblk = ((M.rows + 3) / 4) * G.nbc;
  // byte offsets inside one 4x4 block's rows must fit the 32-bit buffer offset
  if ((long long)(3 * M.cols + 4) * M.T * 2 >= 0x7fffffffLL) return false;
  // workgroup: irf and irf^beta (fp32), the A operands, the resolve role's
  // shared counts and partial moments; then one region per wavefront: masks,
  // component tile ranges, halo, components and (VALU engine) the ring
  G.lds_a = ((8 * M.W + 15) / 16) * 16;
  G.lds_share = G.lds_a + (engine == kEngValu ? 0 : 2 * 2 * G.nbp * 64 * 16);
  G.lds_fixed = G.lds_share + 16 + 4 * 5 * 64 * 4;
  G.off_trange = ((4 * (G.mask_words + G.pair_words + G.need_words) + 15) / 16) * 16;
  G.off_halo = G.off_trange + 80;
  G.off_comp = G.off_halo + kHaloBytes;
  G.off_ring = G.off_comp + kCompBytes;
  G.lds_per_wave = G.off_ring + (engine == kEngValu ? 16 * kRingT * 2 : 0);
  if (engine == kEngValu && 32 * G.nbp > kRingT) return false;
  return (size_t)G.lds_fixed + 4 * (size_t)G.lds_per_wave <= 65536;
}

int tile_workgroups(const DevModel& M) {
  const int nblk = ((M.rows + 3) / 4) * ((M.cols + 3) / 4);
  return (nblk + 3) / 4;
}

template <int kEng>
static hipError_t launch_eng(const DevModel& M, const TileGeom& G, const TileJob& J, hipStream_t s) {
  const int both = J.nr < J.nb ? J.nr : J.nb;
  const dim3 grid(J.nr + J.nb - both + both), block(256);
  if (grid.x == 0) return hipSuccess;
  const size_t lds = G.lds_fixed + 4 * (size_t)G.lds_per_wave;
  switch (G.nbp) {
    case 2: hipLaunchKernelGGL((k_tile<kEng, 2>), grid, block, lds, s, M, G, J); break;
    case 3: hipLaunchKernelGGL((k_tile<kEng, 3>), grid, block, lds, s, M, G, J); break;
    case 4: hipLaunchKernelGGL((k_tile<kEng, 4>), grid, block, lds, s, M, G, J); break;
    case 5: hipLaunchKernelGGL((k_tile<kEng, 5>), grid, block, lds, s, M, G, J); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tile(const DevModel& M, int engine, const TileJob& job, hipStream_t s) {
  TileGeom G;
  if (!tile_geometry(M, engine, G)) return hipErrorInvalidValue;
  switch (engine) {
    case kEngValu: return launch_eng<kEngValu>(M, G, job, s);
    case kEngMfma16: return launch_eng<kEngMfma16>(M, G, job, s);
    case kEngMfma16x2: return launch_eng<kEngMfma16x2>(M, G, job, s);
  }
  return hipErrorInvalidValue;
}

template <int kEng>
static hipError_t launch_cost_eng(const DevModel& M, const TileGeom& G, const uint16_t* hist,
                                  float* ell, hipStream_t s) {
  const dim3 grid((G.nblk + 3) / 4), block(256);
  const size_t lds = G.lds_fixed + 4 * (size_t)G.lds_per_wave;
  switch (G.nbp) {
    case 2: hipLaunchKernelGGL((k_tile_cost<kEng, 2>), grid, block, lds, s, M, G, hist, ell); break;
    case 3: hipLaunchKernelGGL((k_tile_cost<kEng, 3>), grid, block, lds, s, M, G, hist, ell); break;
    case 4: hipLaunchKernelGGL((k_tile_cost<kEng, 4>), grid, block, lds, s, M, G, hist, ell); break;
    case 5: hipLaunchKernelGGL((k_tile_cost<kEng, 5>), grid, block, lds, s, M, G, hist, ell); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
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
  switch (engine) {
    case kEngValu: return launch_cost_eng<kEngValu>(M, G, hist, ell, s);
    case kEngMfma16: return launch_cost_eng<kEngMfma16>(M, G, hist, ell, s);
    case kEngMfma16x2: return launch_cost_eng<kEngMfma16x2>(M, G, hist, ell, s);
  }
  return hipErrorInvalidValue;
}

bool tile_supported(const DevModel& M, int engine) {
  TileGeom G;
  return tile_geometry(M, engine, G);
}

}  // namespace r3d
