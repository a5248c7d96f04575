// Per-frame step on fp16 histograms, one wavefront per 4x4 pixel block, in
// one pass over the histograms.
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
// Posterior (a4, a5). Before the stream, each pixel's prior mixture comes
// from the previous states of the block's 6x6 halo, and the exact cost at a
// reference depth d_ref (the rounded mean of the pixel's own prior component)
// is gathered in fp32. With L = ell + log f the log2 pseudo-posterior,
// Llb = ell(d_ref) + log f(d_ref) <= L*, and with a margin Lambda = ell(d_ref)
// + kLambdaGap, every depth d where ell(d) <= Lambda and every prior component
// is below X = log f(d_ref) - 64 - log2(9) - kLambdaGap satisfies
// L(d) < Llb - 64 <= L* - 64: d cannot be the argmax, and its weight
// exp2(L - L*) is below 2^-64 of the largest one. The skipped depths
// together weigh below D 2^-64 <= 2^-49 of the maximum (D <= 2^15; the
// maximum adds 1 to the weight sum), 25 bits under the fp32 resolution of
// the sums, and their share of the second moment is below 2^-64 D^3 bin^2
// (2^-28 bin^2 at D = 4096).
// Per component, q_k >= X holds on an interval; the 16-bin tiles meeting any
// pixel's interval are candidates. The stream computes the fp16-hi cost of
// every pair of tiles; a pair is evaluated (low part added: the exact cost)
// when it holds a candidate tile or when some pixel's fp16-hi cost, widened
// by its rounding, could exceed Lambda (then with every component of the
// mixture). The argmax and the centred moments are accumulated online
// (running maximum with rescaled, re-centred sums; the four lanes of a pixel
// merge with a symmetric rule, so all of them hold bit-identical results).
// Dense blocks are shared by the wavefronts of a workgroup (see the shared
// blocks section). Then the state update (a6) and the reflectivity /
// background MLE (a7).
#include "r3d_device.hpp"
#include "r3d_tile.hpp"

namespace r3d {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort2 __attribute__((ext_vector_type(2)));
typedef _Float16 half2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kRingT = 256;            // LDS ring per pixel (fp16 bins), VALU engine
constexpr int kRingStride = kRingT + 8;  // its row stride: 16 bytes of padding spread the pixels
                                         // over the LDS banks
constexpr float kCullMargin2 = 64.f;  // log2 units: skipped weights below 2^-64 of the largest
constexpr float kLog2Nine = 3.16992500144231236f;
constexpr float kLiveGap = 40.f;        // log2 units
constexpr unsigned kOob = 0x80000000u;  // buffer offset past every record: loads return zeros
constexpr int kBufWord3 = 0x00020000;   // raw buffer descriptor, 32-bit data format
constexpr int kHaloBytes = 448;         // 6x6 halo of (m, v, pi), 108 floats
constexpr int kCompBytes = 9 * 16 * 16;  // (m, k2, w2, 0) of 9 components x 16 pixels

// blocks in flight per wavefront, beyond the blocks of the current pair
template <int kEng> constexpr int kTilePF = kEng == kEngValu ? 3 : 5;
// wavefronts per workgroup of the step (the vector-FMA engine keeps an LDS
// ring per wavefront, so it stays at 4)
template <int kEng> constexpr int kWavesOf = kEng == kEngValu ? 4 : kTileWaves;
constexpr float kLambdaGap = 32.f;  // log2 units: cost margin above ell(d_ref)
// absolute slack of the fp16-hi cost in the split engine's raw units (hi
// scaled by 2^11): 256 taps x count 2048 x 2^-25 x 2^11
constexpr float kHiSlack = 256.f * 2048.f * 0x1p-25f * 2048.f;

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
  unsigned off_row;  // byte offset of the lane's 8 bins of block 0
  unsigned off;      // off_row, or past the records without data
  unsigned klim;     // blocks kb < klim hold this lane's 8 bins (0 without data)
};

// Mark the lane's pixel faulty (or not): a faulty pixel's photons are ignored.
__device__ __forceinline__ void lane_set_faulty(const DevModel& M, LanePix& L, int g, bool f) {
  L.faulty = L.valid && f;
  L.has_data = L.valid && !f;
  L.off = L.has_data ? L.off_row : kOob;
  L.klim = L.has_data ? (unsigned)((M.T - 8 * g + 31) / 32) : 0u;
}

// The lane's pixel without its faulty flag (taken as not faulty).
__device__ __forceinline__ LanePix lane_pixel_nf(const DevModel& M, const TileGeom& G,
                                                 const uint16_t* hist, int idx, int i16, int g) {
  LanePix L;
  int br, bc;
  block_of(idx, G.nblk / G.nbc, G.nbc, br, bc);
  L.br = __builtin_amdgcn_readfirstlane(br);
  L.bc = __builtin_amdgcn_readfirstlane(bc);
  const int pr = 4 * L.br + (i16 >> 2), pc = 4 * L.bc + (i16 & 3);
  L.valid = pr < M.rows && pc < M.cols && pr * M.cols + pc < M.P;
  L.p = L.valid ? pr * M.cols + pc : 0;
  const int p0 = __builtin_amdgcn_readfirstlane((4 * L.br) * M.cols + 4 * L.bc);
  const long long rec = (long long)(M.P - p0) * M.T * 2;
  L.hbuf = __builtin_amdgcn_make_buffer_rsrc((void*)(hist + (size_t)p0 * M.T), (short)0,
                                             (int)(rec < 0x7fffffffLL ? rec : 0x7fffffffLL),
                                             kBufWord3);
  L.off_row = (unsigned)(((L.p - p0) * M.T + 8 * g) * 2);
  lane_set_faulty(M, L, g, false);
  return L;
}

__device__ __forceinline__ LanePix lane_pixel(const DevModel& M, const TileGeom& G,
                                              const uint16_t* hist, const uint8_t* faulty,
                                              int idx, int i16, int g) {
  LanePix L = lane_pixel_nf(M, G, hist, idx, i16, g);
  lane_set_faulty(M, L, g, L.valid && faulty && faulty[L.p]);
  return L;
}

// Block kb (bins 32 kb .. 32 kb + 31) of the lane's pixel, 8 bins per lane.
__device__ __forceinline__ half8 load_block(const DevModel& M, const LanePix& L, int g, int kb) {
  const unsigned off = (unsigned)kb < L.klim ? L.off + 64u * (unsigned)kb : kOob;
  return __builtin_bit_cast(half8, __builtin_amdgcn_raw_buffer_load_b128(L.hbuf, off, 0, 0));
}

// Bin t of the lane's pixel as a float; zero for t outside [0, T) or a lane
// without data (the load is issued unconditionally, so that a run of them
// is in flight at once).
__device__ __forceinline__ float load_bin(const DevModel& M, const LanePix& L, int g, int t, bool use) {
  const unsigned off = (use && (unsigned)t < (unsigned)M.T && L.off != kOob)
                           ? L.off + 2u * (unsigned)(t - 8 * g) : kOob;
  const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(L.hbuf, off, 0, 0);
  return (float)__builtin_bit_cast(_Float16, b);
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

// fp32 cost of both tiles of pair m from the LDS ring (VALU engine): the
// lane computes its depths d = d_lo + 32 m + 16 tau + 4 g + q (q < 4) of
// tile tau as register blocks. With s = (d_lo - c) mod 4 and the taps
// shifted by s (hs[j'] = irf^beta[j' - s], zero outside the W taps, padded
// to a multiple of 4), every window starts on a multiple of 4 bins: each
// step takes 4 taps from one broadcast LDS read and 4 new bins of each
// window from one 8-byte LDS read, for 32 FMAs. Every accumulator adds its
// taps in increasing order, one FMA each, as the definition reads.
__device__ __forceinline__ int valu_shift(const DevModel& M) { return ((M.d_lo - M.c) % 4 + 4) % 4; }
__device__ __forceinline__ int valu_taps(const DevModel& M) { return (M.W + valu_shift(M) + 3) & ~3; }

__device__ __forceinline__ void valu_pair(const DevModel& M, const float* hs, const _Float16* ring_lds,
                                          int i16, int g, int m, floatx4& c0, floatx4& c1) {
  typedef _Float16 half4 __attribute__((ext_vector_type(4)));
  const int s = valu_shift(M), wp = valu_taps(M);
  const int ta = M.d_lo - M.c + 32 * m + 4 * g - s;  // a multiple of 4
  const _Float16* rp = ring_lds + i16 * kRingStride;
  auto ld4 = [&](int t) __attribute__((always_inline)) -> floatx4 {
    const half4 v = *reinterpret_cast<const half4*>(rp + (t & (kRingT - 1)));
    return floatx4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  };
  floatx4 x0 = ld4(ta), x1 = ld4(ta + 16);
  floatx4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0;
#pragma unroll 2
  for (int jb = 0; jb < wp; jb += 4) {
    const floatx4 y0 = ld4(ta + jb + 4), y1 = ld4(ta + jb + 20);
    const floatx4 h = *reinterpret_cast<const floatx4*>(hs + jb);
    const float w0[8] = {x0[0], x0[1], x0[2], x0[3], y0[0], y0[1], y0[2], y0[3]};
    const float w1[8] = {x1[0], x1[1], x1[2], x1[3], y1[0], y1[1], y1[2], y1[3]};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a0[q] = fmaf(h[k], w0[q + k], a0[q]);
        a1[q] = fmaf(h[k], w1[q + k], a1[q]);
      }
    x0 = y0;
    x1 = y1;
  }
  c0 = a0;
  c1 = a1;
}

__device__ __forceinline__ void ring_store(_Float16* ring_lds, int i16, int g, int kb, half8 v) {
  *reinterpret_cast<half8*>(ring_lds + i16 * kRingStride + ((32 * kb + 8 * g) & (kRingT - 1))) = v;
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
    valu_pair(M, reinterpret_cast<const float*>(sA), ring_lds, lane & 15, lane >> 4, m, c0, c1);
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
    C.k2[k] = 0.5f * kLog2e * fast_rcp(V);
    C.w2[k] = M.lognu2[k] - 0.5f * (kLog2TwoPi + fast_log2(V));
  }
  merge_components(C);
}

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

// Merge the four lanes of each pixel (lanes i16, i16 + 16, i16 + 32,
// i16 + 48); all four end with the same moments.
__device__ __forceinline__ void lane_merge(Moments& mo) {
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
}

// Per-wavefront LDS region of a resolved block.
struct BlockLds {
  unsigned *tmask, *pmask;  // candidate tiles, candidate pairs (then one zero word)
  int* trange;  // [0..8] first and [9..17] last tile of each component's live range
  float* halo;
  float* comp;  // (m, k2, w2, 0) of component k of pixel i16 at comp[4 (16 k + i16)]
  _Float16* ring;
};

__device__ __forceinline__ BlockLds block_lds(const TileGeom& G, unsigned char* wbase) {
  BlockLds B;
  B.tmask = reinterpret_cast<unsigned*>(wbase);
  B.pmask = B.tmask + G.mask_words;
  B.trange = reinterpret_cast<int*>(wbase + G.off_trange);
  B.halo = reinterpret_cast<float*>(wbase + G.off_halo);
  B.comp = reinterpret_cast<float*>(wbase + G.off_comp);
  B.ring = reinterpret_cast<_Float16*>(wbase + G.off_ring);
  return B;
}

// Prior, reference cost and candidate tiles of block idx into its LDS
// region; returns the lane's cost margin Lambda (log2 units) and the
// components live for some pixel (wave-uniform). after_gather() is called
// once the state and reference-cost loads are issued (the caller's first
// histogram loads then queue behind them), after_masks() once the candidate
// masks are complete.
template <int kEng, int NBP, typename AfterGather, typename AfterMasks>
__device__ __forceinline__ void step_prep(const DevModel& M, const TileGeom& G, const StepIO& io,
                                          LanePix& L, const float* sh_h, const BlockLds& B,
                                          int lane, float& Lam, unsigned& wave_live,
                                          AfterGather&& after_gather, AfterMasks&& after_masks) {
  constexpr bool kMfma = kEng != kEngValu;
  constexpr bool kSplit = kEng == kEngMfma16x2;
  // taps per lane (j = g + 4 u): W <= 32 NBP - 30 by construction of NBP, so u < 8 NBP - 7
  constexpr int U = 8 * NBP - 7;
  const int i16 = lane & 15, g = lane >> 4;
  const int dhi = M.d_lo + M.D - 1;

  // One round of independent loads (unconditional, from clamped indices, so
  // that they are all in flight together): the pixel's own state and faulty
  // flag, and the previous states of the block's 6x6 halo.
  const float pm_own = io.pm[L.p], ppi_own = io.ppi[L.p];
  const bool f_own = io.faulty ? io.faulty[L.p] != 0 : false;
  const int hl = lane < 36 ? lane : 0;
  const int hr = 4 * L.br - 1 + hl / 6, hc = 4 * L.bc - 1 + hl % 6;
  const bool hin = hr >= 0 && hr < M.rows && hc >= 0 && hc < M.cols;
  const int hq = hin ? hr * M.cols + hc : 0;
  float hm = io.pm[hq], hv = io.pv[hq], hp = io.ppi[hq];
  // keep these loads ahead of the histogram loads issued below
  asm volatile("" ::: "memory");
  if (!hin) {
    hm = 0.f;
    hv = 1.f;
    hp = -1.f;
  }
  lane_set_faulty(M, L, g, f_own);
  // reference depth: the rounded mean of the pixel's own prior component
  const float mown = (L.valid && ppi_own > 0.5f) ? pm_own : M.m_flat;
  const int dref = (int)fminf(fmaxf(rintf(mown), (float)M.d_lo), (float)dhi);
  // exact cost at d_ref by an fp32 gather (the lane takes taps j = g + 4 u)
  float zr[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = g + 4 * u;
    const int t = dref - M.c + j;
    zr[u] = load_bin(M, L, g, t, j < M.W);
  }
  after_gather();
  if (lane < 36) {
    B.halo[lane] = hm;
    B.halo[36 + lane] = hv;
    B.halo[72 + lane] = hp;
  }
  wave_sync();

  Comps C;
  halo_components(M, B.halo, i16, C);

  wave_live = 0u;
#pragma unroll
  for (int k = 0; k < 9; ++k) wave_live |= (__any(L.valid && (C.live >> k & 1u)) ? 1u : 0u) << k;
  // X = Llb - 64 - Lambda - log2(9), with Llb = ell(d_ref) + log f(d_ref) and
  // Lambda = ell(d_ref) + kLambdaGap: the reference cost cancels, so the
  // candidate tiles do not wait for its gather
  const float theta = L.valid
      ? log_prior2(C, (float)dref, wave_live) - kCullMargin2 - kLambdaGap - kLog2Nine
      : INFINITY;

  // Component k is "live" on depths where q_k >= theta - kLiveGap: at a
  // candidate depth of a pair whose costs stay below Lambda some component
  // reaches theta, so components below theta - kLiveGap change f by less
  // than 9 * 2^-kLiveGap relative and are skipped there.
  // The block keeps, per component, the tile range covering every pixel's
  // live interval (LDS min / max over the pixels).
  // Each lane group takes its own components (k = g, g + 4, and k = 8 for
  // the first group), so the loop runs three times rather than nine; the
  // LDS minima, maxima and or-ed bits do not depend on which lane adds them.
  if (lane < 9) {
    B.trange[lane] = 0x7fffffff;
    B.trange[9 + lane] = -1;
  }
  // candidate tiles and pairs (LDS bit masks, or-ed by the lanes)
  const int nwords = G.mask_words + G.pair_words + 1;  // the pair bits are read 64 at a time
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
  // component g + 4 it of the lane's group (it < 2), component 8 (it == 2)
  auto pick = [&](const float (&a)[9], int it) __attribute__((always_inline)) -> float {
    if (it == 2) return a[8];
    const float x0 = a[4 * it], x1 = a[4 * it + 1], x2 = a[4 * it + 2], x3 = a[4 * it + 3];
    return g == 0 ? x0 : (g == 1 ? x1 : (g == 2 ? x2 : x3));
  };
  if (L.valid) {
#pragma unroll
    for (int it = 0; it < 3; ++it) {
      if (it == 2 && g != 0) continue;
      const int k = it == 2 ? 8 : g + 4 * it;
      const float w2 = pick(C.w2, it), mk = pick(C.m, it), rk = fast_rcp(pick(C.k2, it));
      if (w2 >= theta - kLiveGap) {
        const float R = __builtin_amdgcn_sqrtf((w2 - theta + kLiveGap) * rk) + 2.0f;
        const float lo = fmaxf(mk - R, (float)M.d_lo);
        const float hi = fminf(mk + R, (float)dhi);
        if (lo <= hi) {
          atomicMin(&B.trange[k], ((int)floorf(lo) - M.d_lo) >> 4);
          atomicMax(&B.trange[9 + k], ((int)ceilf(hi) - M.d_lo) >> 4);
        }
      }
      if (w2 >= theta) {
        const float R = __builtin_amdgcn_sqrtf((w2 - theta) * rk) + 2.0f;
        const float lo = fmaxf(floorf(mk - R), (float)M.d_lo);
        const float hi = fminf(ceilf(mk + R), (float)dhi);
        if (lo <= hi) {
          const int ta = ((int)lo - M.d_lo) >> 4, tb = ((int)hi - M.d_lo) >> 4;
          set_bits(B.tmask, ta, tb);
          set_bits(B.pmask, ta >> 1, tb >> 1);
        }
      }
    }
  }
  wave_sync();
  after_masks();
  // the reference cost, whose gather has been in flight meanwhile
  float lref = 0.f;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = g + 4 * u;
    if (j < M.W) lref = fmaf(sh_h[j], zr[u], lref);
  }
  lref = group_sum<16, 32>(lref);
  Lam = lref * M.scale2 + kLambdaGap;
  // the pixels' components, component-major
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      *reinterpret_cast<float4*>(B.comp + 4 * (16 * k + i16)) = make_float4(C.m[k], C.k2[k], C.w2[k], 0.f);
    }
  }
  wave_sync();
}

// State update (a6) and reflectivity / background (a7) of block idx from
// its moments (already merged over the four lanes of each pixel).
template <int kEng, int NBP>
__device__ __forceinline__ void step_finish(const DevModel& M, const StepIO& io, const LanePix& L,
                                            const float* sh_irf, Moments mo, float K, int lane) {
  constexpr int U = 8 * NBP - 7;  // taps per lane, as in step_prep
  const int g = lane >> 4;
  const float mu = mo.S1 / mo.S0;
  const int dstar = (int)mo.ref;
  const float mean = mo.ref + mu;
  // the depth point estimate is the posterior mean (Sec. II-E): the MLE
  // places the IRF at its nearest bin
  const int dmle = (int)fminf(fmaxf(rintf(mean), (float)M.d_lo), (float)(M.d_lo + M.D - 1));
  const float var = fmaxf(mo.S2 / mo.S0 - mu * mu, 0.f);

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
    const int t = dmle - M.c + j;
    const bool in = j < M.W && t >= 0 && t < M.T;
    wz[u] = load_bin(M, L, g, t, in);
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

// ============================ shared blocks ============================
// A dense block (candidate tiles on many of its pairs: a frame border, a
// flat or wide prior) can be shared by the wavefronts of its workgroup.
// The dense block with the most candidate pairs owns the workgroup's share
// region (a choice made by the data alone): its wavefront publishes the
// margins and a list of the block's chunks of pairs: chunk 0 (its first
// blocks are already in the owner's ring), the heavy chunks (those holding
// candidate pairs, whose evaluations dominate the time), then the light
// ones, each group in chunk order. The owner takes chunks from the front of
// the list; the other wavefronts, once their own blocks are done, take the
// heavy chunks left from the back of the heavy part, then light ones from
// the back of the list, so that no heavy chunk is left for last. Each
// chunk's moments go to a slot of their own and are merged in chunk order,
// so the result does not depend on which wavefront took which chunk.
struct ShareLds {
  unsigned* ctl;  // [0] wavefronts decided, [1] owner wavefront + 1 (0: none),
                  // [2] chunk claims, positions in the list (owner's next | end of the
                  // others' heavy part << 8 | end of the others' light part << 16 |
                  // end of the heavy part << 24), [3] live components,
                  // [4 + w] wavefront w's decision (0: pending, 1: not dense, 2 + its
                  // candidate pairs: dense)
  float* lam;     // [16] cost margin of each pixel
  unsigned* K;    // [16] photon count of each pixel (integer sums: exact in any order)
  unsigned* order;  // [kMaxChunks] the list of chunks
  unsigned* heavy;  // [kMaxChunks] chunk holds candidate pairs (1) or not (0)
  float* slot;    // [kMaxChunks][5][16] moments of each chunk
};

// control words: 4, then one decision per wavefront, padded to 8 words
constexpr int kCtlWords = (4 + kTileWaves + 7) / 8 * 8;
constexpr int kShareBytes = (kCtlWords + 32 + 2 * kMaxChunks + kMaxChunks * 5 * 16) * 4;

__device__ __forceinline__ ShareLds share_lds(const TileGeom& G, unsigned char* smem) {
  ShareLds S;
  S.ctl = reinterpret_cast<unsigned*>(smem + G.off_share);
  S.lam = reinterpret_cast<float*>(S.ctl + kCtlWords);
  S.K = S.ctl + kCtlWords + 16;
  S.order = S.ctl + kCtlWords + 32;
  S.heavy = S.order + kMaxChunks;
  S.slot = reinterpret_cast<float*>(S.heavy + kMaxChunks);
  return S;
}

__device__ __forceinline__ void put_moments(float* s, const Moments& mo, int i16) {
  s[i16] = mo.R;
  s[16 + i16] = mo.ref;
  s[32 + i16] = mo.S0;
  s[48 + i16] = mo.S1;
  s[64 + i16] = mo.S2;
}

__device__ __forceinline__ Moments get_moments(const float* s, int i16) {
  return Moments{s[i16], s[16 + i16], s[32 + i16], s[48 + i16], s[64 + i16]};
}

// ============================ one wavefront ============================
// The wavefront's tasks: its own block (whole, or in chunks when it owns the
// shared block), then chunks of the shared block. Each task streams its
// pairs through the register ring (the blocks of the current pair plus
// kTilePF prefetched ones): photon count and count validation on every
// block, the exact cost of both tiles of every pair, the posterior on the
// pairs that need it. After the workgroup barrier each wavefront finishes its
// own block (a6, a7).
template <int kEng, int NBP>
__device__ __forceinline__ void step_wave(const DevModel& M, const TileGeom& G, const StepIO& io,
                                          int idx, int wave, const half8* sA, const float* sh_irf,
                                          const float* sh_h, unsigned char* smem, int lane) {
  constexpr bool kMfma = kEng != kEngValu;
  constexpr bool kSplit = kEng == kEngMfma16x2;
  constexpr int RING = NBP + kTilePF<kEng>;
  const int i16 = lane & 15, g = lane >> 4;
  const int dhi = M.d_lo + M.D - 1;
  const float cs2 = M.scale2 * (kSplit ? (1.0f / 2048.0f) : 1.0f);  // raw cost -> log2 units
  constexpr int NW = kWavesOf<kEng>;
  const int ngrp = (G.nblk + NW - 1) / NW;  // workgroups; wavefront w takes block w * ngrp + j
  const bool active = idx < G.nblk;
  unsigned char* wown = smem + G.lds_fixed + wave * G.lds_per_wave;
  _Float16* ring_lds = block_lds(G, wown).ring;
  const ShareLds S = share_lds(G, smem);

  // current task: pairs [mb, me) of the block of L and B; c = its chunk, or
  // -1 for a whole block
  // (the faulty flag of the own block is read with the prior's loads)
  LanePix L = lane_pixel_nf(M, G, io.hist, active ? idx : 0, i16, g);
  BlockLds B = block_lds(G, wown);
  int mb = 0, me = G.npairs, c = -1, kb_end = G.kb_last;
  auto fetch = [&](int kb) __attribute__((always_inline)) -> half8 {
    return load_block(M, L, g, kb <= kb_end ? kb : -1);
  };
  half8 ring[RING];
  half8 Ahi[2][NBP];
  if constexpr (kMfma) {
#pragma unroll
    for (int tau = 0; tau < 2; ++tau)
#pragma unroll
      for (int b = 0; b < NBP; ++b) Ahi[tau][b] = a_op(sA, NBP, 0, tau, b, lane);
  }
  float Lam = 0.f;
  unsigned wave_live = 0u;
  // the first blocks are in flight while the prior is prepared; the block's
  // decision (below) is published as soon as its candidate masks are built
  bool dense = false;
  unsigned mine = 1u;
  if (active)
    step_prep<kEng, NBP>(
        M, G, io, L, sh_h, B, lane, Lam, wave_live,
        [&]() __attribute__((always_inline)) {
#pragma unroll
          for (int x = 0; x < RING - 1; ++x) ring[x] = fetch(G.kbA0 + x);
        },
        [&]() __attribute__((always_inline)) {
          int ncand = 0;
          for (int w = 0; w < G.pair_words; ++w)
            ncand += __builtin_popcount(__builtin_amdgcn_readfirstlane(B.pmask[w]));
          dense = G.nchunks >= 2 && 64 * ncand >= G.npairs;
          // decision: 1 for a plain block, 2 + its candidate pairs for a dense one
          mine = dense ? 2u + (unsigned)ncand : 1u;
          if (lane == 0)
            __hip_atomic_store(&S.ctl[4 + wave], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        });
  const bool own_faulty = L.faulty;
  // of the dense blocks (candidate tiles on at least a 64th of their pairs:
  // most blocks but the plainest) the one with the most candidate pairs (the
  // lowest-numbered wavefront's among equals) is shared, so that the
  // workgroup's wavefronts end together: a dense wavefront waits (bounded)
  // for the decisions of the others, which finish their preparation at about
  // the same time. The owner publishes the margins, then every wavefront
  // with a block counts itself decided.
  bool owner = false;
  if (active) {
    if (dense) {
      owner = true;
      for (int v = 0; v < NW && owner; ++v) {
        if (v == wave || v * ngrp + (int)blockIdx.x >= G.nblk) continue;  // itself, or no block
        unsigned dv = 0u;
        for (int n = 0; n < (1 << 20) && dv == 0u; ++n) {
          dv = __builtin_amdgcn_readfirstlane(
              __hip_atomic_load(&S.ctl[4 + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
          if (dv == 0u) __builtin_amdgcn_s_sleep(4);
        }
        // a denser block, an as dense lower-numbered one, or no answer keeps
        // this one unshared
        owner = dv != 0u && (dv < mine || (dv == mine && v > wave));
      }
    }
    if (owner) {
      if (g == 0) {
        S.lam[i16] = Lam;
        S.K[i16] = 0u;
      }
      if (lane == 0) {
        S.ctl[1] = (unsigned)wave + 1u;
        S.ctl[3] = wave_live;
      }
      // the list: lane k tests chunk k for candidate pairs, then places it
      unsigned hk = 0u;
      if (lane < G.nchunks) {
        const int a = lane * G.chunk, b = min(a + G.chunk, G.npairs);
        for (int w = a >> 5; w <= (b - 1) >> 5; ++w) {
          const int lo = max(a - 32 * w, 0), hi = min(b - 32 * w, 32);
          const unsigned msk = (hi == 32 ? 0xffffffffu : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
          hk |= (B.pmask[w] & msk) != 0u ? 1u : 0u;
        }
        S.heavy[lane] = hk;
      }
      wave_sync();
      if (lane < G.nchunks) {
        // position: chunk 0 first, then (heavy first, chunk index)
        int pos = 0;
        if (lane > 0) {
          pos = 1;
          for (int j = 1; j < G.nchunks; ++j) {
            const unsigned hj = S.heavy[j];
            pos += (hj > hk || (hj == hk && j < lane)) ? 1 : 0;
          }
        }
        S.order[pos] = (unsigned)lane;
      }
      // the list's heavy part is [0, nh); chunk 0 is the owner's
      const unsigned nh =
          1u + (unsigned)__builtin_popcountll(__ballot(lane >= 1 && lane < G.nchunks && hk != 0u));
      if (lane == 0) S.ctl[2] = 1u | (nh << 8) | ((unsigned)G.nchunks << 16) | (nh << 24);
      // the owner's ring runs on from one chunk into the next (kb_end stays
      // at the end of the block)
      c = 0;
      me = G.chunk < G.npairs ? G.chunk : G.npairs;
    }
    if (lane == 0) __hip_atomic_fetch_add(&S.ctl[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  int nactive = 0;
  for (int w = 0; w < NW; ++w) nactive += (w * ngrp + (int)blockIdx.x < G.nblk) ? 1 : 0;

  // take a chunk of the shared block (-1 once none is left; each chunk is
  // taken once): while heavy ones are left, the owner from the front of the
  // list and the others from the back of its heavy part; then the owner from
  // the front of the light part and the others from the back of the list
  auto claim = [&](bool front) __attribute__((always_inline)) -> int {
    int got = -1;
    if (lane == 0) {
      unsigned old = __hip_atomic_load(&S.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      for (;;) {
        const unsigned f = old & 0xffu, hb = (old >> 8) & 0xffu, b = (old >> 16) & 0xffu,
                       nh = old >> 24;
        unsigned pos, next;
        if (f < hb) {
          pos = front ? f : hb - 1u;
          next = front ? old + 1u : old - 0x100u;
        } else {
          const unsigned f2 = f > nh ? f : nh;
          if (f2 >= b) break;
          pos = front ? f2 : b - 1u;
          next = front ? ((old & ~0xffu) | (f2 + 1u)) : old - 0x10000u;
        }
        const unsigned seen = atomicCAS(&S.ctl[2], old, next);
        if (seen == old) {
          got = (int)S.order[pos];
          break;
        }
        old = seen;
      }
    }
    return __builtin_amdgcn_readfirstlane(got);
  };
  auto is_cand = [&](const unsigned* mk, int i) __attribute__((always_inline)) -> bool {
    return (__builtin_amdgcn_readfirstlane(mk[i >> 5]) >> (i & 31)) & 1u;
  };
  // the margin test on the raw cost bits: a pair is evaluated for the lane's
  // pixel when the largest raw cost of its 8 depths reaches thr, the margin
  // taken back through the fp16-hi widening (the split engine) and lowered
  // by 2^-20 relative so that the rounding of this conversion only adds
  // evaluations; lanes without a pixel never reach it
  auto margin_bits = [&](float lam) __attribute__((always_inline)) -> unsigned {
    float thr = kSplit ? (lam / cs2 - kHiSlack) * (1.0f / (1.0f + 0x1p-9f)) : lam / cs2;
    thr *= 1.0f - 0x1p-20f;
    return !L.valid ? 0x7f800000u : (thr > 0.f ? __float_as_uint(thr) : 0u);
  };
  unsigned thr = margin_bits(Lam);

  // first: the task is the wavefront's own block, whose first ring blocks
  // are already loaded (a wavefront without a block starts with a chunk)
  bool have = active, first = active, helping = false;
  int pend = -1;  // a chunk the owner took that does not follow its ring
  for (;;) {
    if (have) {
      if (!first) {
#pragma unroll
        for (int x = 0; x < RING - 1; ++x) ring[x] = fetch(G.kbA0 + mb + x);
      }
      const int* trange = B.trange;
      const float* comp = B.comp;
      Moments mo{-INFINITY, 0.f, 0.f, 0.f, 0.f};
      auto tile_epi = [&](const floatx4& acc, int dt, bool all) __attribute__((always_inline)) {
        const int dbase = M.d_lo + 16 * dt + 4 * g;
        unsigned tmk = wave_live;
        if (!all) {
          const int TAv = lane < 9 ? trange[lane] : 1, TBv = lane < 9 ? trange[9 + lane] : 0;
          tmk = (unsigned)__ballot(TAv <= dt && dt <= TBv) & 0x1ffu;
        }
        // log2 f by a log-sum-exp over the live components: their maximum,
        // then the sum of exp2 of each below it (one exp2 per component)
        const float4* cp = reinterpret_cast<const float4*>(comp) + i16;
        float lp[4];
        if (__builtin_popcount(tmk) <= 1) {
          const float4 c = cp[16 * (tmk ? __builtin_ctz(tmk) : 0)];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float e = (float)(dbase + q) - c.x;
            lp[q] = tmk ? fmaf(-e * e, c.y, c.z) : -INFINITY;
          }
        } else {
          float mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY}, sm[4] = {0.f, 0.f, 0.f, 0.f};
          for (unsigned bits = tmk; bits; bits &= bits - 1u) {
            const float4 c = cp[16 * __builtin_ctz(bits)];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float e = (float)(dbase + q) - c.x;
              mx[q] = fmaxf(mx[q], fmaf(-e * e, c.y, c.z));
            }
          }
          // a pixel with none of these components alive keeps -inf
#pragma unroll
          for (int q = 0; q < 4; ++q) mx[q] = mx[q] == -INFINITY ? 0.f : mx[q];
          for (unsigned bits = tmk; bits; bits &= bits - 1u) {
            const float4 c = cp[16 * __builtin_ctz(bits)];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float e = (float)(dbase + q) - c.x;
              sm[q] += fast_exp2(fmaf(-e * e, c.y, c.z) - mx[q]);
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) lp[q] = mx[q] + fast_log2(sm[q]);
        }
        float Lq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) Lq[q] = (L.valid && dbase + q <= dhi) ? fmaf(acc[q], cs2, lp[q]) : -INFINITY;
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
          // the four depths d0 + q in closed form: with e0 = d0 - ref and
          // T_k = sum_q q^k w_q, sum_q w_q e_q = e0 T0 + T1 and
          // sum_q w_q e_q^2 = e0 (e0 T0 + 2 T1) + T2
          float w[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = fast_exp2(Lq[q] - mo.R);
          const float T0 = (w[0] + w[1]) + (w[2] + w[3]);
          const float T1 = fmaf(3.f, w[3], fmaf(2.f, w[2], w[1]));
          const float T2 = fmaf(9.f, w[3], fmaf(4.f, w[2], w[1]));
          const float e0 = (float)dbase - mo.ref;
          mo.S0 += T0;
          mo.S1 += fmaf(e0, T0, T1);
          mo.S2 += fmaf(e0, fmaf(e0, T0, 2.f * T1), T2);
        }
      };

      // photon count by fp32 dot products with ones (exact integer sums),
      // count validation by the packed maximum of the raw fp16 bits
      float Kv = 0.f;
      ushort2 vmax = {0, 0};
      unsigned vfrac = 0u;
      auto account = [&](half8 v) __attribute__((always_inline)) {
        const ushort8 u = __builtin_bit_cast(ushort8, v);
        const ushort2 m01 = __builtin_elementwise_max(ushort2{u[0], u[1]}, ushort2{u[2], u[3]});
        const ushort2 m23 = __builtin_elementwise_max(ushort2{u[4], u[5]}, ushort2{u[6], u[7]});
        vmax = __builtin_elementwise_max(vmax, __builtin_elementwise_max(m01, m23));
        // non-integral counts: the fractional parts' bits, paired into 32-bit
        // words and or-ed (16-bit or chains cost a spill at this register
        // budget)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          vfrac |= __builtin_bit_cast(unsigned, half2{(_Float16)__builtin_amdgcn_fracth(v[2 * s]),
                                                      (_Float16)__builtin_amdgcn_fracth(v[2 * s + 1])});
        const half2 one2 = {(_Float16)1.f, (_Float16)1.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) Kv = __builtin_amdgcn_fdot2(half2{v[2 * s], v[2 * s + 1]}, one2, Kv, false);
      };
      // the task's moments and photon count, lane-merged, to the own region
      // (cc < 0) or to chunk cc's slot
      auto flush = [&](int cc) __attribute__((always_inline)) {
        const float K = group_sum<16, 32>(Kv);
        Moments mm = mo;
        lane_merge(mm);
        if (g == 0) {
          if (cc < 0) {
            float* own = block_lds(G, wown).halo;  // the halo is dead once the prior is built
            put_moments(own, mm, i16);
            own[80 + i16] = K;
          } else {
            put_moments(S.slot + cc * 80, mm, i16);
            atomicAdd(&S.K[i16], (unsigned)K);
          }
        }
        mo = Moments{-INFINITY, 0.f, 0.f, 0.f, 0.f};
        Kv = 0.f;
      };
      if (first) {
        // blocks of [0, T) that no depth window reaches still hold photons
        for (int kb = 0; kb < G.nkb; ++kb) {
          if (kb >= G.kbA0 && kb <= G.kb_last) continue;
          account(load_block(M, L, g, kb));
        }
      }
      // the owner runs on through chunks that follow each other in the list
      // without reloading the ring: at each chunk end (chunks are whole ring
      // rounds) it flushes and takes the next chunk from the front; one that
      // does not follow becomes its next task
      const bool run_on = owner;
      bool flushed = false;
      for (int m0 = mb; m0 < me; m0 += RING) {
        // candidate-pair bits of pairs m0 .. m0 + RING - 1 (< 41 bits past
        // pbase)
        const int pbase = m0 & ~31;
        const unsigned long long pbits =
            (unsigned long long)__builtin_amdgcn_readfirstlane(B.pmask[pbase >> 5]) |
            ((unsigned long long)__builtin_amdgcn_readfirstlane(B.pmask[(pbase >> 5) + 1]) << 32);
#pragma unroll
        for (int u = 0; u < RING; ++u) {
          const int m = m0 + u;
          ring[(u + RING - 1) % RING] = fetch(G.kbA0 + m + RING - 1);
          if (m < me) {
            half8 blk[NBP];
#pragma unroll
            for (int b = 0; b < NBP; ++b) blk[b] = ring[(u + b) % RING];
            if constexpr (!kMfma) {
              wave_sync();
#pragma unroll
              for (int b = 0; b < NBP; ++b) ring_store(ring_lds, i16, g, G.kbA0 + m + b, blk[b]);
              wave_sync();
            }
            // every block of the band counted once: the first NBP - 1 with
            // pair 0, then the last block of each pair
            if (m == 0) {
#pragma unroll
              for (int b = 0; b < NBP - 1; ++b) account(blk[b]);
            }
            account(blk[NBP - 1]);
            // cost of both tiles: the fp16-hi contraction (A operands in
            // registers) on every pair, the low part only where the pair is
            // evaluated
            floatx4 a0, a1;
            if constexpr (kMfma) {
              a0 = floatx4{0.f, 0.f, 0.f, 0.f};
              a1 = a0;
#pragma unroll
              for (int b = 0; b < NBP; ++b) {
                a0 = mfma16(Ahi[0][b], blk[b], a0);
                a1 = mfma16(Ahi[1][b], blk[b], a1);
              }
            } else {
              valu_pair(M, reinterpret_cast<const float*>(sA), ring_lds, i16, g, m, a0, a1);
            }
            // a pixel whose cost in this pair may exceed its margin needs the
            // pair evaluated with every component (the cost is >= 0: compare
            // bits); the fp16-hi cost is widened by its rounding (2^-11 per
            // tap and below 2^-25 absolute per subnormal tap, times counts <=
            // 2048 and at most 256 taps)
            const unsigned pm = __builtin_elementwise_max(
                __builtin_elementwise_max(
                    __builtin_elementwise_max(__float_as_uint(a0[0]), __float_as_uint(a0[1])),
                    __builtin_elementwise_max(__float_as_uint(a0[2]), __float_as_uint(a0[3]))),
                __builtin_elementwise_max(
                    __builtin_elementwise_max(__float_as_uint(a1[0]), __float_as_uint(a1[1])),
                    __builtin_elementwise_max(__float_as_uint(a1[2]), __float_as_uint(a1[3]))));
            const bool all = __any(pm >= thr);
            if (all || ((pbits >> (m - pbase)) & 1u)) {
              if constexpr (kSplit) {
                // the low-part operands are all read before the first product
                half8 Alo[2][NBP];
#pragma unroll
                for (int b = 0; b < NBP; ++b) {
                  Alo[0][b] = a_op(sA, NBP, 1, 0, b, lane);
                  Alo[1][b] = a_op(sA, NBP, 1, 1, b, lane);
                }
                floatx4 l0 = {0.f, 0.f, 0.f, 0.f}, l1 = l0;
#pragma unroll
                for (int b = 0; b < NBP; ++b) {
                  l0 = mfma16(Alo[0][b], blk[b], l0);
                  l1 = mfma16(Alo[1][b], blk[b], l1);
                }
                a0 = a0 + l0;
                a1 = a1 + l1;
              }
              for (int tau = 0; tau < 2; ++tau)
                if (all || is_cand(B.tmask, 2 * m + tau)) tile_epi(tau ? a1 : a0, 2 * m + tau, all);
            }
          }
        }
        if (run_on && m0 + RING == me && me < G.npairs) {
          flush(c);
          const int nc = claim(true);
          if (nc != c + 1) {
            flushed = true;
            pend = nc;
            break;
          }
          c = nc;
          me = me + G.chunk < G.npairs ? me + G.chunk : G.npairs;
        }
      }
      // above 2048, negative (sign bit set) or not an integer
      const unsigned bad = (vmax[0] > 0x6800u || vmax[1] > 0x6800u || vfrac != 0) ? kErrOverflow : 0u;
      if (bad) atomicOr(M.err, bad);
      if (!flushed) flush(c);
      first = false;
    }
    if (!helping && !owner) {
      helping = true;
      // wait (bounded) until every wavefront with a block has decided; a
      // wavefront that gives up leaves the chunks to the others, which take
      // all of them
      bool decided = false;
      for (int n = 0; n < (1 << 20) && !decided; ++n) {
        decided = (int)__builtin_amdgcn_readfirstlane(
                      __hip_atomic_load(&S.ctl[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) >= nactive;
        if (!decided) __builtin_amdgcn_s_sleep(4);
      }
      const unsigned ow = decided ? __builtin_amdgcn_readfirstlane(S.ctl[1]) : 0u;
      if (ow == 0u) break;
      const int oi = (int)ow - 1;
      L = lane_pixel(M, G, io.hist, io.faulty, oi * ngrp + (int)blockIdx.x, i16, g);
      B = block_lds(G, smem + G.lds_fixed + oi * G.lds_per_wave);
      thr = margin_bits(S.lam[i16]);
      wave_live = __builtin_amdgcn_readfirstlane(S.ctl[3]);
    }
    c = pend >= 0 ? pend : claim(owner);
    pend = -1;
    if (c < 0) break;
    mb = c * G.chunk;
    me = mb + G.chunk < G.npairs ? mb + G.chunk : G.npairs;
    // the owner's ring may run on into the next chunk: it loads to the end
    kb_end = owner ? G.kb_last : G.kbA0 + me + NBP - 2;
    have = true;
  }
  __syncthreads();
  if (active) {
    Moments mo;
    float K;
    if (owner) {
      mo = Moments{-INFINITY, 0.f, 0.f, 0.f, 0.f};
      for (int k = 0; k < G.nchunks; ++k) merge_moments(mo, get_moments(S.slot + k * 80, i16));
      K = (float)S.K[i16];
    } else {
      const float* own = block_lds(G, wown).halo;
      mo = get_moments(own, i16);
      K = own[80 + i16];
    }
    LanePix Lo = lane_pixel_nf(M, G, io.hist, idx, i16, g);
    lane_set_faulty(M, Lo, g, own_faulty);
    step_finish<kEng, NBP>(M, io, Lo, sh_irf, mo, K, lane);
  }
}

// LDS of the workgroup: irf and irf^beta (fp32), irf^beta's fp16 hi and lo
// parts, the A operands, then each wavefront's region and the shared chunk
// region. The fp16 parts are staged in LDS first (one coalesced load per
// tap), so that the A operands are built from LDS rather than from scattered
// 2-byte global loads.
template <int kEng, int NBP>
__device__ __forceinline__ void tile_prologue(const DevModel& M, const TileGeom& G,
                                              unsigned char* smem) {
  float* sh_irf = reinterpret_cast<float*>(smem);
  float* sh_h = sh_irf + M.W;
  _Float16* sh16 = reinterpret_cast<_Float16*>(sh_h + M.W);  // [0, W) hi, [W, 2W) lo
  for (int j = threadIdx.x; j < M.W; j += blockDim.x) {
    sh_irf[j] = M.irf[j];
    sh_h[j] = M.h[j];
    sh16[j] = M.h16hi[j];
    sh16[M.W + j] = M.h16lo[j];
  }
  if constexpr (kEng == kEngValu) {
    // the VALU engine's taps, shifted by (d_lo - c) mod 4 and zero-padded
    float* hs = reinterpret_cast<float*>(smem + G.lds_a);
    const int sh = ((M.d_lo - M.c) % 4 + 4) % 4, wp = (M.W + sh + 3) & ~3;
    for (int j = threadIdx.x; j < wp; j += blockDim.x) {
      const int k = j - sh;
      hs[j] = (k >= 0 && k < M.W) ? M.h[k] : 0.f;
    }
  } else {
    __syncthreads();
    half8* sA = reinterpret_cast<half8*>(smem + G.lds_a);
    for (int e = threadIdx.x; e < 2 * 2 * NBP * 64; e += blockDim.x) {
      const int ln = e & 63, b = (e >> 6) % NBP, tau = (e / (64 * NBP)) & 1, part = e / (128 * NBP);
      const int g = ln >> 4, i16 = ln & 15;
      const _Float16* src = sh16 + (part ? M.W : 0);
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

// One frame: wavefront w of workgroup j takes block w * (workgroups) + j, so
// the border blocks (first in block order) fall on wavefront 0 of distinct
// workgroups and each can be shared by its workgroup.
template <int kEng, int NBP>
__global__ void __launch_bounds__(64 * kWavesOf<kEng>, NBP <= 3 ? 4 : 2) k_tile_step(DevModel M, TileGeom G,
                                                                      StepIO io) {
  extern __shared__ __align__(16) unsigned char smem[];
  {
    // Workgroups are dispatched in order, so a frame's grid fills the
    // compute units a quarter at a time (a 256x256 frame: four workgroups
    // per unit, one from each quarter), and each SIMD favours its older
    // wavefronts. The first quarter holds the frame-border blocks (the
    // heaviest: every tile of theirs is evaluated) and keeps the highest
    // priority; the last quarter, which the age order would serve last,
    // comes next; the middle two share the lowest (152 against 155 us per
    // launch of the 256x256 x 4096-bin frames).
    const unsigned q = blockIdx.x * 4u / gridDim.x;
    if (q == 0u)
      __builtin_amdgcn_s_setprio(3);
    else if (q == 3u)
      __builtin_amdgcn_s_setprio(2);
    else
      __builtin_amdgcn_s_setprio(1);
  }
  if (threadIdx.x < 4 + kWavesOf<kEng>) {
    // no wavefront decided yet, no shared block, no decisions
    if (threadIdx.x < 2 || threadIdx.x >= 4) reinterpret_cast<unsigned*>(smem + G.off_share)[threadIdx.x] = 0u;
  }
  tile_prologue<kEng, NBP>(M, G, smem);
  // the wavefront index is uniform: say so, so that everything derived from
  // it (the block, its buffer descriptor, the task switches) stays scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int idx = wave * ((G.nblk + kWavesOf<kEng> - 1) / kWavesOf<kEng>) + (int)blockIdx.x;
  const float* sh_irf = reinterpret_cast<const float*>(smem);
  const float* sh_h = sh_irf + M.W;
  const half8* sA = reinterpret_cast<const half8*>(smem + G.lds_a);
  step_wave<kEng, NBP>(M, G, io, idx, wave, sA, sh_irf, sh_h, smem, lane);
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

// ============================ minimum divergence ============================
// Minimum beta-divergence depth estimates, with no prior. The single-band
// estimate maximises the cost ell(d) (Sec. II-B, last paragraph); the
// multispectral one maximises sum_l log(c_l(d) / K_l), c_l the band's
// correlation with its own irf^beta and K_l its photon count (Appendix,
// eq. div_MSL), bands without photons left out. One wavefront per 4x4 pixel
// block streams each band's histograms once through a register ring (each
// 32-bin block loaded once, kTilePF pairs ahead for one band, one for
// several), computes every pair's exact cost (split fp16 on the matrix
// cores, or fp32) and reduces it to a running argmax per lane (the lowest
// depth among equal values), merged over the pixel's four lanes. The
// photon counts and the count validation (integers in [0, 2048]) ride on
// the stream. The kernel holds kNBL bands' rings and operands (one, two or
// kMaxBands); every ring load is issued unconditionally, a band past the
// last reading nothing, so that the compiler's wait counts stay exact
// across the unrolled ring (a load under a branch costs a wait for every
// load in flight).
template <int kEng, int NBP, bool kMsl, int kNBL>
__global__ void __launch_bounds__(256) k_mindiv(MindivArgs A) {
  static_assert(kMsl ? (kNBL >= 1 && kNBL <= kMaxBands) : kNBL == 1, "bands held");
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = kMsl ? A.nb : 1;
  for (int l = 0; l < nb; ++l) tile_prologue<kEng, NBP>(A.M[l], A.G[l], smem + l * A.lds_band);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i16 = lane & 15, g = lane >> 4;
  const DevModel& M0 = A.M[0];
  const TileGeom& G0 = A.G[0];
  const int idx = blockIdx.x * 4 + wave;
  if (idx >= G0.nblk) return;
  _Float16* ring_lds = reinterpret_cast<_Float16*>(smem + nb * A.lds_band) + wave * 16 * kRingStride;
  constexpr int NBL = kNBL;
  constexpr int RING = NBP + (kMsl ? 1 : kTilePF<kEng>);

  // photon counts by fp16 dot products with ones (exact integer sums), count
  // validation by the packed maximum of the raw fp16 bits and the or of the
  // fractional parts
  ushort2 vmax = {0, 0};
  unsigned vfrac = 0u;
  auto account = [&](half8 v, float& kv) __attribute__((always_inline)) {
    const ushort8 u = __builtin_bit_cast(ushort8, v);
    const ushort2 m01 = __builtin_elementwise_max(ushort2{u[0], u[1]}, ushort2{u[2], u[3]});
    const ushort2 m23 = __builtin_elementwise_max(ushort2{u[4], u[5]}, ushort2{u[6], u[7]});
    vmax = __builtin_elementwise_max(vmax, __builtin_elementwise_max(m01, m23));
#pragma unroll
    for (int q = 0; q < 8; ++q)
      vfrac |= (unsigned)__builtin_bit_cast(unsigned short, (_Float16)__builtin_amdgcn_fracth(v[q]));
    const half2 one2 = {(_Float16)1.f, (_Float16)1.f};
#pragma unroll
    for (int q = 0; q < 4; ++q) kv = __builtin_amdgcn_fdot2(half2{v[2 * q], v[2 * q + 1]}, one2, kv, false);
  };

  float Kv[NBL];
  LanePix Lb[NBL];
#pragma unroll
  for (int l = 0; l < NBL; ++l) {
    Kv[l] = 0.f;
    if (l >= nb) {
      // a band past the last: its ring loads read nothing
      Lb[l] = Lb[0];
      Lb[l].klim = 0u;
      continue;
    }
    Lb[l] = lane_pixel(A.M[l], A.G[l], A.hist[l], nullptr, idx, i16, g);
    // blocks of [0, T) that no depth window reaches still hold photons
    const TileGeom& Gl = A.G[l];
    for (int kb = 0; kb < Gl.nkb; ++kb)
      if (kb < Gl.kbA0 || kb > Gl.kb_last) account(load_block(A.M[l], Lb[l], g, kb), Kv[l]);
  }

  const bool valid = Lb[0].valid;
  float best = -INFINITY;
  int bidx = 0;
  // one band on the matrix cores: the fp16-hi A operands stay in registers
  // (the low parts are read from LDS), halving the LDS reads of each pair
  constexpr bool kHiRegs = !kMsl && kEng != kEngValu;
  half8 Ahi[2][NBP];
  if constexpr (kHiRegs) {
    const half8* sA0 = reinterpret_cast<const half8*>(smem + G0.lda_band);
#pragma unroll
    for (int tau = 0; tau < 2; ++tau)
#pragma unroll
      for (int b = 0; b < NBP; ++b) Ahi[tau][b] = a_op(sA0, NBP, 0, tau, b, lane);
  }
  // One pass over the band blocks: the running argmax of the cost (one band)
  // or of the sum over the bands in ``mask`` (per pixel), counting the
  // photons when ``counting``.
  half8 ring[NBL][RING];
  auto stream = [&](unsigned mask, bool counting) __attribute__((always_inline)) {
    best = -INFINITY;
    bidx = 0;
#pragma unroll
    for (int l = 0; l < NBL; ++l) {
#pragma unroll
      for (int x = 0; x < RING - 1; ++x) {
        const int kb = A.G[l].kbA0 + x;
        ring[l][x] = load_block(A.M[l], Lb[l], g, kb <= A.G[l].kb_last ? kb : -1);
      }
    }
  for (int m0 = 0; m0 < G0.npairs; m0 += RING) {
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      const int m = m0 + u;
#pragma unroll
      for (int l = 0; l < NBL; ++l) {
        const int kb = A.G[l].kbA0 + m + RING - 1;
        ring[l][(u + RING - 1) % RING] = load_block(A.M[l], Lb[l], g, kb <= A.G[l].kb_last ? kb : -1);
      }
      if (m < G0.npairs) {
        floatx4 J0 = {0.f, 0.f, 0.f, 0.f}, J1 = J0;
#pragma unroll
        for (int l = 0; l < NBL; ++l) {
          if (l >= nb) continue;
          const DevModel& Ml = A.M[l];
          const TileGeom& Gl = A.G[l];
          half8 blk[NBP];
#pragma unroll
          for (int b = 0; b < NBP; ++b) blk[b] = ring[l][(u + b) % RING];
          if (counting) {
            // every block of the band counted once: the first NBP - 1 with
            // pair 0, then the last block of each pair
            if (m == 0) {
#pragma unroll
              for (int b = 0; b < NBP - 1; ++b) account(blk[b], Kv[l]);
            }
            account(blk[NBP - 1], Kv[l]);
          }
          if constexpr (kEng == kEngValu) {
            wave_sync();
#pragma unroll
            for (int b = 0; b < NBP; ++b) ring_store(ring_lds, i16, g, Gl.kbA0 + m + b, blk[b]);
            wave_sync();
          }
          const half8* sA = reinterpret_cast<const half8*>(smem + l * A.lds_band + Gl.lda_band);
          floatx4 c0, c1;
          if constexpr (kHiRegs) {
            floatx4 h0 = {0.f, 0.f, 0.f, 0.f}, h1 = h0;
#pragma unroll
            for (int b = 0; b < NBP; ++b) {
              h0 = mfma16(Ahi[0][b], blk[b], h0);
              h1 = mfma16(Ahi[1][b], blk[b], h1);
            }
            if constexpr (kEng == kEngMfma16x2) {
              half8 Alo[2][NBP];
#pragma unroll
              for (int b = 0; b < NBP; ++b) {
                Alo[0][b] = a_op(sA, NBP, 1, 0, b, lane);
                Alo[1][b] = a_op(sA, NBP, 1, 1, b, lane);
              }
              floatx4 l0 = {0.f, 0.f, 0.f, 0.f}, l1 = l0;
#pragma unroll
              for (int b = 0; b < NBP; ++b) {
                l0 = mfma16(Alo[0][b], blk[b], l0);
                l1 = mfma16(Alo[1][b], blk[b], l1);
              }
              c0 = h0 + l0;
              c1 = h1 + l1;
            } else {
              c0 = h0;
              c1 = h1;
            }
          } else {
            pair_cost<kEng, NBP>(Ml, sA, ring_lds, lane, m, blk, c0, c1);
          }
          if constexpr (kMsl) {
            const bool use = (mask >> l) & 1u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              J0[q] += !use ? 0.f : (c0[q] > 0.f ? fast_log2(c0[q]) : -INFINITY);
              J1[q] += !use ? 0.f : (c1[q] > 0.f ? fast_log2(c1[q]) : -INFINITY);
            }
          } else {
            J0 = c0;
            J1 = c1;
          }
        }
        // depths past the grid (only the last pair reaches them) are -inf
        if (m == G0.npairs - 1) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int o = 32 * m + 4 * g + q;
            J0[q] = o < M0.D ? J0[q] : -INFINITY;
            J1[q] = o + 16 < M0.D ? J1[q] : -INFINITY;
          }
        }
        // the pair's maximum over the lane's eight depths and the first
        // depth that attains it (depth offsets: 16 tau + q past 32 m + 4 g),
        // then the running one; strict comparisons keep the lowest depth
        // among equal values
        int off[2];
        float mt[2];
#pragma unroll
        for (int tau = 0; tau < 2; ++tau) {
          const floatx4 J = tau ? J1 : J0;
          mt[tau] = __builtin_fmaxf(__builtin_fmaxf(J[0], J[1]), __builtin_fmaxf(J[2], J[3]));
          off[tau] = 16 * tau + (J[0] == mt[tau] ? 0 : J[1] == mt[tau] ? 1 : J[2] == mt[tau] ? 2 : 3);
        }
        const bool hi = mt[1] > mt[0];
        const float mp = hi ? mt[1] : mt[0];
        if (mp > best) {
          best = mp;
          bidx = 32 * m + 4 * g + (hi ? off[1] : off[0]);
        }
      }
    }
  }
  };
  // Several bands: the pass assumes every band of every pixel holds photons;
  // a block where some band of some pixel has none (that band leaves the
  // sum) runs the pass again with the pixels' own bands.
  stream(kMsl ? (1u << A.nb) - 1u : 1u, true);
  float Kb[NBL];
  unsigned mask = 0u;
#pragma unroll
  for (int l = 0; l < NBL; ++l) {
    Kb[l] = group_sum<16, 32>(Kv[l]);
    if (l < nb) mask |= (Kb[l] > 0.f ? 1u : 0u) << l;
  }
  if constexpr (kMsl) {
    if (__any(valid && mask != (1u << A.nb) - 1u)) stream(mask, false);
  }
  // above 2048, negative (sign bit set) or not an integer
  if (vmax[0] > 0x6800u || vmax[1] > 0x6800u || vfrac != 0) atomicOr(M0.err, kErrOverflow);
  group_argmax<16, 32>(best, bidx);
  if (valid && g == 0) {
    float val;
    if constexpr (kMsl) {
      // log2 of the raw cost is log2 c_l + 11 for the split engine (its
      // high part is scaled by 2^11)
      const float sh = kEng == kEngMfma16x2 ? 11.f : 0.f;
      float off = 0.f;
#pragma unroll
      for (int l = 0; l < NBL; ++l)
        if (l < A.nb && ((mask >> l) & 1u)) off += sh + fast_log2(Kb[l]);
      val = best == -INFINITY ? -INFINITY : (best - off) * kLn2;
    } else {
      (void)Kb;
      val = best * M0.scale2 * (kEng == kEngMfma16x2 ? (1.0f / 2048.0f) : 1.0f) * kLn2;
    }
    A.argmax[Lb[0].p] = M0.d_lo + bidx;
    if (A.value) A.value[Lb[0].p] = val;
  }
}

static int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// LDS bytes of the VALU engine's shifted taps (padded to a multiple of 4,
// plus one spare group)
static int valu_hs_bytes(const DevModel& M) { return ((4 * (M.W + 8) + 15) / 16) * 16; }

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
  G.nkb = (M.T + 31) / 32;
  G.kb_last = G.kbA0 + G.npairs - 1 + G.nbp - 1;
  G.nbc = (M.cols + 3) / 4;
  G.nblk = ((M.rows + 3) / 4) * G.nbc;
  // byte offsets inside one 4x4 block's rows must fit the 32-bit buffer offset
  if ((long long)(3 * M.cols + 4) * M.T * 2 >= 0x7fffffffLL) return false;
  // workgroup: irf and irf^beta (fp32) and the A operands; then one region
  // per wavefront: masks, component tile ranges, halo, components and (VALU
  // engine) the ring
  G.lds_a = ((12 * M.W + 15) / 16) * 16;  // irf, irf^beta (fp32), fp16 hi and lo
  G.lds_fixed = G.lds_a + (engine == kEngValu ? valu_hs_bytes(M) : 2 * 2 * G.nbp * 64 * 16);
  G.off_trange = ((4 * (G.mask_words + G.pair_words + 1) + 15) / 16) * 16;
  G.off_halo = G.off_trange + 80;
  G.off_comp = G.off_halo + kHaloBytes;
  G.off_ring = G.off_comp + kCompBytes;
  G.lds_per_wave = G.off_ring + (engine == kEngValu ? 16 * kRingStride * 2 : 0);
  G.waves = engine == kEngValu ? kWavesOf<kEngValu> : kWavesOf<kEngMfma16x2>;
  G.off_share = G.lds_fixed + G.waves * G.lds_per_wave;
  G.lds_total = G.off_share + kShareBytes;
  // chunks of a whole number of ring rounds (RING pairs), at most
  // kMaxChunks of them: the owner of a shared block streams on from one
  // chunk into the next at the end of a round, and the ring's first
  // RING - 1 blocks, loaded before the block's chunking is known, lie in
  // the band of its first chunk
  const int ring = G.nbp + (engine == kEngValu ? kTilePF<kEngValu> : kTilePF<kEngMfma16x2>);
  G.chunk = ring * ((G.npairs + kMaxChunks * ring - 1) / (kMaxChunks * ring));
  G.nchunks = (G.npairs + G.chunk - 1) / G.chunk;
  if (engine == kEngValu && 32 * G.nbp > kRingT) return false;
  return G.lds_total <= 65536;
}


template <int kEng>
static hipError_t launch_step_eng(const DevModel& M, const TileGeom& G, const StepIO& io,
                                  hipStream_t s) {
  const size_t lds = G.lds_total;
  const dim3 grid((G.nblk + G.waves - 1) / G.waves), block(64 * G.waves);
  if (G.nblk < 1) return hipErrorInvalidValue;
  switch (G.nbp) {
    case 2: hipLaunchKernelGGL((k_tile_step<kEng, 2>), grid, block, lds, s, M, G, io); break;
    case 3: hipLaunchKernelGGL((k_tile_step<kEng, 3>), grid, block, lds, s, M, G, io); break;
    case 4: hipLaunchKernelGGL((k_tile_step<kEng, 4>), grid, block, lds, s, M, G, io); break;
    case 5: hipLaunchKernelGGL((k_tile_step<kEng, 5>), grid, block, lds, s, M, G, io); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step_tile(const DevModel& M, int engine, const StepIO& io, hipStream_t s) {
  TileGeom G;
  if (!tile_geometry(M, engine, G)) return hipErrorInvalidValue;
  switch (engine) {
    case kEngValu: return launch_step_eng<kEngValu>(M, G, io, s);
    case kEngMfma16: return launch_step_eng<kEngMfma16>(M, G, io, s);
    case kEngMfma16x2: return launch_step_eng<kEngMfma16x2>(M, G, io, s);
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

template <int kEng, bool kMsl, int kNBL>
static hipError_t launch_mindiv_eng(const MindivArgs& A, int nbp, size_t lds, hipStream_t s) {
  const dim3 grid((A.G[0].nblk + 3) / 4), block(256);
  switch (nbp) {
#define R3D_MD_CASE(N)                                                                  \
  case N:                                                                               \
    if (lds > 65536)                                                                    \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mindiv<kEng, N, kMsl, kNBL>), \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);        \
    hipLaunchKernelGGL((k_mindiv<kEng, N, kMsl, kNBL>), grid, block, lds, s, A);             \
    break;
    R3D_MD_CASE(2)
    R3D_MD_CASE(3)
    R3D_MD_CASE(4)
    R3D_MD_CASE(5)
#undef R3D_MD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// the multispectral kernel holds the registers of two bands, or of all
template <int kEng>
static hipError_t launch_mindiv_bands(const MindivArgs& A, bool msl, int nbp, size_t lds, hipStream_t s) {
  if (!msl) return launch_mindiv_eng<kEng, false, 1>(A, nbp, lds, s);
  return A.nb <= 2 ? launch_mindiv_eng<kEng, true, 2>(A, nbp, lds, s)
                   : launch_mindiv_eng<kEng, true, kMaxBands>(A, nbp, lds, s);
}

hipError_t launch_mindiv(const DevModel* M, const uint16_t* const* hist, int nb, int engine,
                         bool msl, int32_t* argmax, float* value, hipStream_t s) {
  if (nb < 1 || nb > kMaxBands || (!msl && nb != 1)) return hipErrorInvalidValue;
  MindivArgs A{};
  A.nb = nb;
  A.argmax = argmax;
  A.value = value;
  int nbp = 2;
  for (int l = 0; l < nb; ++l) {
    A.M[l] = M[l];
    A.hist[l] = hist[l];
    if (!tile_geometry(M[l], engine, A.G[l])) return hipErrorInvalidValue;
    nbp = A.G[l].nbp > nbp ? A.G[l].nbp : nbp;
  }
  // every band's A operands are built for the widest band (extra blocks
  // carry zero taps); each band region holds its staging and A operands
  int band = 0;
  for (int l = 0; l < nb; ++l) {
    A.G[l].nbp = nbp;
    A.G[l].lda_band = ((12 * M[l].W + 15) / 16) * 16;
    const int need = A.G[l].lda_band + (engine == kEngValu ? valu_hs_bytes(M[l]) : 2 * 2 * nbp * 64 * 16);
    band = need > band ? need : band;
  }
  for (int l = 0; l < nb; ++l) A.G[l].lds_a = A.G[l].lda_band;
  A.lds_band = band;
  const size_t lds = (size_t)nb * band + (engine == kEngValu ? 4 * 16 * kRingStride * 2 : 0);
  const int lds_max = M[0].lds_max > 0 ? M[0].lds_max : 65536;
  if (lds > (size_t)lds_max) return hipErrorInvalidValue;
  switch (engine) {
    case kEngValu: return launch_mindiv_bands<kEngValu>(A, msl, nbp, lds, s);
    case kEngMfma16: return launch_mindiv_bands<kEngMfma16>(A, msl, nbp, lds, s);
    case kEngMfma16x2: return launch_mindiv_bands<kEngMfma16x2>(A, msl, nbp, lds, s);
  }
  return hipErrorInvalidValue;
}

bool tile_supported(const DevModel& M, int engine) {
  TileGeom G;
  return tile_geometry(M, engine, G);
}

}  // namespace r3d
