// Reverse-mode adjoint of one frame of the filter (differentiation of
// Algorithm 1 with respect to beta, the IRF taps, sigma_rw2 and nu).
//
// Forward, per pixel (Sec. II-B, eq. beta_div2; Sec. III-A, eq. predict;
// Sec. II-C, eq. approx_post):
//   L(d)  = s A(d) + log f(d),   s = (beta+1)/beta,  A(d) = sum_j irf_j^beta z[d-c+j]
//   log f = log sum_k exp(q_k),  q_k = log nu_k - log(2 pi V_k)/2 - (d-m_k)^2/(2 V_k),
//           V_k = v_k + sigma_rw2
//   w(d)  = exp(L(d)) / sum exp(L),  mean = sum w d,  var = sum w (d-mean)^2.
// Given the adjoints mbar, vbar of mean and var:
//   g(d) = dJ/dL(d) = w(d) [mbar (d-mean) + vbar ((d-mean)^2 - var)]
// and, with the responsibilities r_k = exp(q_k - log f):
//   dJ/dbeta  += sum_d g (-A/beta^2 + s B),  B(d) = sum_j irf_j^beta ln(irf_j) z[d-c+j]
//   dJ/dirf_j += s beta irf_j^(beta-1) sum_d g(d) z[d-c+j]
//   dJ/dm_k    = sum_d g r_k (d-m_k) / V_k
//   dJ/dV_k    = sum_d g r_k ((d-m_k)^2 - V_k) / (2 V_k^2)   (-> sigma_rw2 and v_k)
//   dJ/dnu_k  += sum_d g r_k / nu_k = sum_d g exp(q_k - log nu_k - log f),
// the last form also for a zero weight, where it is the one-sided derivative
// (the component's unweighted density over f).
// One wavefront per pixel, on the candidate depths of the forward step
// (depths outside carry exactly zero weight in fp32): the frame's mean,
// variance and log2 normaliser come from the forward step; pass 2 forms
// g(d), accumulates the sums and keeps g in LDS, pass 3 correlates g with the
// non-empty bins for the tap sums. The
// adjoints of the neighbours' states are written per (component, pixel) and
// gathered per neighbour by k_adjoint_gather, and the parameter sums are
// reduced per block then over blocks in a fixed order: no atomics, so the
// gradient is bit-reproducible.
#include "r3d_adjoint.hpp"
#include "r3d_pixel.hpp"

namespace r3d {

namespace {

constexpr int kAdjU = kMaxW / 64;  // taps per lane

__host__ __device__ inline int adj_fixed_words(int W) { return (2 * W + 3) & ~3; }
__host__ __device__ inline int adj_wave_words(int T, int D) {
  return pixel_lds_words(T) + ((D + 3) & ~3);
}

// Both tap sums of depth d in one gather (same bin order as cost_gather).
__device__ __forceinline__ void cost_gather2(const DevModel& M, const unsigned* hist,
                                             const unsigned* nzmask, const float* tapA,
                                             const float* tapB, int d, bool sparse, float& A,
                                             float& B) {
  A = 0.f;
  B = 0.f;
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
        const float z = packed_count(hist, tb);
        A = fmaf(tapA[tb - t0], z, A);
        B = fmaf(tapB[tb - t0], z, B);
      }
      t = base + 32;
    }
  } else {
    const int jlo = t0 < 0 ? -t0 : 0;
    const int jhi = (M.T - t0) < M.W ? (M.T - t0) : M.W;
    for (int j = jlo; j < jhi; ++j) {
      const float z = packed_count(hist, t0 + j);
      A = fmaf(tapA[j], z, A);
      B = fmaf(tapB[j], z, B);
    }
  }
}

__device__ __forceinline__ void adjoint_pixel(const DevModel& M, const AdjIO& io, int p, int lane,
                                              unsigned* hist, float* gbuf, const float* sh_h,
                                              const float* sh_hl, float (&accT)[kThetaFixed],
                                              float (&accG)[kAdjU]) {
  const int nwords = (M.T + 1) >> 1;
  unsigned* nzmask = hist + nwords;
  {
    uint4* z4 = reinterpret_cast<uint4*>(hist);
    const int n4 = pixel_lds_words(M.T) >> 2;
    for (int w = lane; w < n4; w += 64) z4[w] = make_uint4(0u, 0u, 0u, 0u);
  }
  wave_fence();
  const bool faulty = io.faulty && io.faulty[p];
  float K = 0.f;
  unsigned bad = 0u;
  if (!faulty) K = csr_histogram(M, io.row_ptr, io.toa, p, lane, hist, nzmask, bad);
  if (bad) atomicOr(M.err, bad);
  wave_fence();

  Comps C;
  float Vk[9];
  unsigned nb;
  build_components_raw(M, io.pm, io.pv, io.ppi, p, C, Vk, nb);
  const unsigned live = __builtin_amdgcn_readfirstlane(C.live);
  nb = __builtin_amdgcn_readfirstlane(nb);
  float R[9], Rl[9];
  int dlo_c, dhi_c;
  candidate_range(M, C, live, K, faulty, lane, R, Rl, dlo_c, dhi_c);
  const bool sparse = 3.f * K <= (float)M.T;

  // the frame's moments and normaliser, as the forward step computed them
  const float mean = io.mean[p];
  const float var = io.var[p];
  const float lz = io.lognorm[p];

  // ---- pass 2: g(d) and the sums ----
  const float mb = io.gm[p];
  const float vb = io.gv ? io.gv[p] : 0.f;
  const float s_nat = M.scale2 * kLn2;
  const float s_prime = -1.f / (M.beta * M.beta);
  float a0[9], a1[9], a2[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) a0[k] = a1[k] = a2[k] = 0.f;
  float ab = 0.f;
  for (int d0 = dlo_c; d0 <= dhi_c; d0 += 64) {
    unsigned cand, cmask;
    chunk_masks(C, R, Rl, d0, cand, cmask);
    const int d = d0 + lane;
    const bool in = d <= dhi_c;
    if (cand == 0u) {  // no weight anywhere in the chunk
      if (in) gbuf[d - dlo_c] = 0.f;
      continue;
    }
    if (!in) continue;
    float A = 0.f, B = 0.f;
    if (!faulty) cost_gather2(M, hist, nzmask, sh_h, sh_hl, d, sparse, A, B);
    float q[9], ek[9];
    float mx = -INFINITY;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float e = (float)d - C.m[k];
      q[k] = C.w2[k] - e * e * C.k2[k];
      if (live & (1u << k)) mx = fmaxf(mx, q[k]);
    }
    float ssum = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      ek[k] = (live & (1u << k)) ? fast_exp2(q[k] - mx) : 0.f;
      ssum += ek[k];
    }
    const float L2 = fmaf(A, M.scale2, mx + fast_log2(ssum));
    const float w = fast_exp2(L2 - lz);
    const float del = (float)d - mean;
    const float g = w * fmaf(mb, del, vb * fmaf(del, del, -var));
    gbuf[d - dlo_c] = g;
    ab = fmaf(g, fmaf(s_prime, A, s_nat * B), ab);
    const float gr = g * fast_rcp(ssum);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float t = gr * ek[k];
      const float e = (float)d - C.m[k];
      a0[k] += t;
      a1[k] = fmaf(t, e, a1[k]);
      a2[k] = fmaf(t * e, e, a2[k]);
    }
  }
  wave_fence();



  // ---- pass 3: tap sums G_j = sum_d g(d) z[d - c + j] over non-empty bins ----
  if (!faulty && dlo_c <= dhi_c) {
    const int nmw = (M.T + 31) >> 5;
    for (int wb = 0; wb < nmw; ++wb) {
      unsigned bits = __builtin_amdgcn_readfirstlane(nzmask[wb]);
      while (bits) {
        const int t = (wb << 5) + __builtin_ctz(bits);
        bits &= bits - 1u;
        const float z = packed_count(hist, t);
#pragma unroll
        for (int u = 0; u < kAdjU; ++u) {
          const int j = lane + 64 * u;
          const int d = t + M.c - j;
          if (j < M.W && d >= dlo_c && d <= dhi_c) accG[u] = fmaf(z, gbuf[d - dlo_c], accG[u]);
        }
      }
    }
  }
  wave_fence();

  // ---- wavefront sums and outputs ----
  ab = group_sum<1, 32>(ab);
  float sig_bar = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    float mbar = 0.f, vbar = 0.f;
    if (live & (1u << k)) {
      const float s0 = group_sum<1, 32>(a0[k]);
      const float s1 = group_sum<1, 32>(a1[k]);
      const float s2 = group_sum<1, 32>(a2[k]);
      const float V = Vk[k];
      mbar = s1 / V;
      vbar = (s2 / V - s0) / (2.f * V);
      sig_bar += vbar;
      accT[2 + k] += s0 / M.nu[k];
    }
    if (lane == 0) {
      const bool own = (nb >> k) & 1u;
      io.cm[(size_t)k * M.P + p] = own ? mbar : 0.f;
      io.cv[(size_t)k * M.P + p] = own ? vbar : 0.f;
    }
  }
  accT[0] += ab;
  accT[1] += sig_bar;

  // ---- pass 4, zero-weight components only (wave-uniform): the one-sided
  // derivative in nu_k, sum_d g(d) exp2(q_k - log2 nu_k - log2 f) with
  // q_k - log2 nu_k the component's unweighted log2 density ----
  const unsigned zw = ~live & 0x1ffu;
  if (zw) {
    float an[9], wz[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) an[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k)  // log2 V = log2(log2(e) / 2) - log2 k2
      wz[k] = (zw >> k & 1u) ? -0.5f * (kLog2TwoPi + fast_log2(0.5f * kLog2e) - fast_log2(C.k2[k])) : 0.f;
    for (int d = dlo_c + lane; d <= dhi_c; d += 64) {
      const float g = gbuf[d - dlo_c];
      if (g == 0.f) continue;
      float q[9];
      float mx = -INFINITY;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const float e = (float)d - C.m[k];
        q[k] = C.w2[k] - e * e * C.k2[k];
        if (live & (1u << k)) mx = fmaxf(mx, q[k]);
      }
      float ssum = 0.f;
#pragma unroll
      for (int k = 0; k < 9; ++k) ssum += (live & (1u << k)) ? fast_exp2(q[k] - mx) : 0.f;
      const float gr = g * fast_rcp(ssum);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        if (!(zw >> k & 1u)) continue;
        const float e = (float)d - C.m[k];
        an[k] = fmaf(gr, fast_exp2(wz[k] - e * e * C.k2[k] - mx), an[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (zw >> k & 1u) accT[2 + k] += group_sum<1, 32>(an[k]);
  }
}

// 4 wavefronts per SIMD (128 VGPRs, a few spills): the pixel passes are
// latency-bound, and twice the wavefronts in flight halves the stalls
__global__ void __launch_bounds__(256, 4) k_adjoint(DevModel M, AdjIO io) {
  extern __shared__ __align__(16) float smem[];
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int W = M.W;
  float* sh_h = smem;
  float* sh_hl = smem + W;
  const int fixed = adj_fixed_words(W);
  const int per_wave = adj_wave_words(M.T, M.D);
  unsigned* hist = reinterpret_cast<unsigned*>(smem + fixed) + (size_t)wave * per_wave;
  float* gbuf = reinterpret_cast<float*>(hist + pixel_lds_words(M.T));
  const int npar = kThetaFixed + W;
  float* red = smem + fixed + (size_t)nw * per_wave;  // [nw][npar]
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    const float h = M.h[j], f = M.irf[j];
    sh_h[j] = h;
    sh_hl[j] = f > 0.f ? h * logf(f) : 0.f;
  }
  __syncthreads();
  float accT[kThetaFixed];
#pragma unroll
  for (int i = 0; i < kThetaFixed; ++i) accT[i] = 0.f;
  float accG[kAdjU];
#pragma unroll
  for (int u = 0; u < kAdjU; ++u) accG[u] = 0.f;
  for (int p = blockIdx.x * nw + wave; p < M.P; p += gridDim.x * nw)
    adjoint_pixel(M, io, p, lane, hist, gbuf, sh_h, sh_hl, accT, accG);
  float* mine = red + (size_t)wave * npar;
  if (lane == 0)
    for (int i = 0; i < kThetaFixed; ++i) mine[i] = accT[i];
#pragma unroll
  for (int u = 0; u < kAdjU; ++u) {
    const int j = lane + 64 * u;
    if (j < W) mine[kThetaFixed + j] = accG[u];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npar; i += blockDim.x) {
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += red[(size_t)w * npar + i];
    io.part[(size_t)blockIdx.x * npar + i] = s;
  }
}

__global__ void k_adjoint_gather(int rows, int cols, const float* __restrict__ cm,
                                 const float* __restrict__ cv, const float* __restrict__ gm_prev,
                                 const float* __restrict__ gv_prev, float* __restrict__ am,
                                 float* __restrict__ av) {
  const int P = rows * cols;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  const int r = q / cols, c = q - r * cols;
  float sm = gm_prev ? gm_prev[q] : 0.f;
  float sv = gv_prev ? gv_prev[q] : 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    // pixel p whose stencil position k is q
    const int pr = r - (k / 3 - 1), pc = c - (k % 3 - 1);
    if (pr >= 0 && pr < rows && pc >= 0 && pc < cols) {
      const size_t i = (size_t)k * P + pr * cols + pc;
      sm += cm[i];
      sv += cv[i];
    }
  }
  am[q] = sm;
  av[q] = sv;
}

// One workgroup per parameter: each thread sums a fixed stride of the block
// partials in fp64, then a fixed-order tree over the threads (the same
// order every run, so the gradient stays bit-reproducible).
constexpr int kReduceThreads = 256;

__global__ void __launch_bounds__(kReduceThreads) k_theta_reduce(DevModel M, const float* __restrict__ part,
                                                                 int blocks, double* __restrict__ grad) {
  __shared__ double red[kReduceThreads];
  const int npar = kThetaFixed + M.W;
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < blocks; b += kReduceThreads) s += (double)part[(size_t)b * npar + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    s = red[0];
    if (i >= kThetaFixed) {
      const double beta = M.beta;
      const double s_nat = (beta + 1.0) / beta;
      const double f = M.irf[i - kThetaFixed];
      s = f > 0.0 ? s * s_nat * beta * pow(f, beta - 1.0) : 0.0;
    }
    grad[i] += s;
  }
}

__global__ void k_fill_f32(float* x, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void k_fill_f64(double* x, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    x[i] = v;
}

}  // namespace

AdjGeom adjoint_geometry(const DevModel& M) {
  AdjGeom g{0, 0, 0};
  const size_t cap = 65536;
  const size_t fixed = (size_t)adj_fixed_words(M.W) * 4;
  const size_t per_wave = ((size_t)adj_wave_words(M.T, M.D) + kThetaFixed + M.W) * 4;
  if (fixed + per_wave > cap) return g;
  size_t nw = (cap - fixed) / per_wave;
  if (nw > 4) nw = 4;
  g.waves = (int)nw;
  const int need = (M.P + g.waves - 1) / g.waves;
  g.blocks = need < 2048 ? need : 2048;
  g.lds = fixed + nw * per_wave;
  return g;
}

hipError_t launch_adjoint(const DevModel& M, const AdjIO& io, const AdjGeom& g, hipStream_t s) {
  if (g.waves == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adjoint, dim3(g.blocks), dim3(64 * g.waves), g.lds, s, M, io);
  return hipGetLastError();
}

hipError_t launch_adjoint_gather(const DevModel& M, const float* cm, const float* cv,
                                 const float* gm_prev, const float* gv_prev, float* am, float* av,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_gather, dim3((M.P + 255) / 256), dim3(256), 0, s, M.rows, M.cols,
                     cm, cv, gm_prev, gv_prev, am, av);
  return hipGetLastError();
}

hipError_t launch_theta_reduce(const DevModel& M, const float* part, int blocks, double* grad,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_theta_reduce, dim3(kThetaFixed + M.W), dim3(kReduceThreads), 0, s, M, part,
                     blocks, grad);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* x, size_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t b = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_f32, dim3(b < 4096 ? b : 4096), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* x, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t b = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_f64, dim3(b < 4096 ? b : 4096), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

}  // namespace r3d
