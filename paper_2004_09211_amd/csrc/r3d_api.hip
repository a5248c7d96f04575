// C ABI of libr3d: parameter validation, context management and launches.
// Every entry point validates synchronously, then enqueues on the caller's
// stream; nothing here synchronises except create/destroy and the explicit
// device-status query.
#include <cmath>
#include <cstring>
#include <new>
#include <algorithm>
#include <mutex>
#include <vector>

#include "r3d_internal.hpp"
#include "r3d_tile.hpp"
#include "r3d_adjoint.hpp"
#include "r3d_batch.hpp"
#include "r3d_pixel.hpp"

struct r3d_ctx {
  int device = 0;
  r3d_params prm{};
  std::vector<double> irf;
  r3d::DevModel dm{};
  float* d_h = nullptr;
  float* d_irf = nullptr;
  _Float16* d_h16 = nullptr;  // [2*W]: hi then lo
  unsigned* d_err = nullptr;
};

namespace {

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

r3d_status check_params(const r3d_params* p) {
  if (!p) return R3D_EINVAL;
  if (p->rows < 1 || p->cols < 1) return R3D_EINVAL;
  if ((int64_t)p->rows * p->cols > (int64_t)1 << 30) return R3D_EUNSUPPORTED;
  if (p->T < 1 || p->T > 32767) return R3D_EINVAL;
  if (p->D < 1 || p->D > 32768) return R3D_EINVAL;
  // grid depths stay exact in fp32 and d_lo + D - 1 cannot overflow
  if (p->d_lo < -(1 << 20) || p->d_lo > (1 << 20)) return R3D_EINVAL;
  if (p->W < 1 || p->W > r3d::kMaxW) return R3D_EINVAL;
  if (p->c < 0 || p->c >= p->W) return R3D_EINVAL;
  if (!p->irf) return R3D_EINVAL;
  if (!finite_pos(p->beta) || !finite_pos(p->sigma_rw2)) return R3D_EINVAL;
  if (!std::isfinite(p->d_min) || !std::isfinite(p->d_max) || !(p->d_max > p->d_min))
    return R3D_EINVAL;
  double s = 0.0;
  for (int j = 0; j < p->W; ++j) {
    if (!std::isfinite(p->irf[j]) || p->irf[j] < 0.0) return R3D_EINVAL;
    s += p->irf[j];
  }
  if (!(s > 0.0)) return R3D_EINVAL;
  double n = 0.0;
  for (int k = 0; k < 9; ++k) {
    if (!std::isfinite(p->nu[k]) || p->nu[k] < 0.0) return R3D_EINVAL;
    n += p->nu[k];
  }
  if (!(n > 0.0)) return R3D_EINVAL;
  if (p->precision < R3D_FP32 || p->precision > R3D_FP16X2_MFMA) return R3D_EINVAL;
  return R3D_OK;
}

r3d_status check_state(const r3d_state* s) {
  if (!s || !s->m || !s->v || !s->pi || !s->b) return R3D_EINVAL;
  return R3D_OK;
}

bool same_buffer(const r3d_state* a, const r3d_state* b) {
  const float* pa[4] = {a->m, a->v, a->pi, a->b};
  const float* pb[4] = {b->m, b->v, b->pi, b->b};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      if (pa[i] == pb[j]) return true;
  return false;
}

r3d::StepIO make_io(const float* pi_in, const uint8_t* faulty, const r3d_state* prev,
                    const r3d_state* next, const r3d_out* out) {
  r3d::StepIO io{};
  io.pi_in = pi_in;
  io.faulty = faulty;
  io.pm = prev->m;
  io.pv = prev->v;
  io.ppi = prev->pi;
  io.pb = prev->b;
  io.nm = next->m;
  io.nv = next->v;
  io.npi = next->pi;
  io.nb = next->b;
  if (out) {
    io.depth = out->depth;
    io.var = out->var;
    io.intensity = out->intensity;
    io.background = out->background;
    io.pi0_next = out->pi0_next;
    io.argmax = out->argmax;
  }
  return io;
}

r3d_status hip_status(hipError_t e) {
  if (e == hipSuccess) return R3D_OK;
  if (e == hipErrorInvalidValue) return R3D_EUNSUPPORTED;
  if (e == hipErrorOutOfMemory) return R3D_ENOMEM;
  return R3D_EHIP;
}

void free_ctx(r3d_ctx* c) {
  if (!c) return;
  if (c->d_h) (void)hipFree(c->d_h);
  if (c->d_irf) (void)hipFree(c->d_irf);
  if (c->d_h16) (void)hipFree(c->d_h16);
  if (c->d_err) (void)hipFree(c->d_err);
  delete c;
}

}  // namespace

// Device tables of r3d_batch_run_noalloc (sequence descriptors, chunk prefix,
// frame pointers, work counter, done counters): a fixed array in every GPU's
// memory, held until the process ends. Host code uses the address that
// hipGetSymbolAddress returns for the current device, never the array's name.
constexpr size_t kBatchScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kBatchScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};
// host staging of the tables; guarded by g_stage_mu until their upload ends
std::mutex g_stage_mu;
alignas(256) unsigned char g_stage[kBatchScratchBytes];

// The scratch array's device address on the current device, resolved once
// per device (with that device current).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* r3d_status_string(r3d_status s) {
  switch (s) {
    case R3D_OK: return "ok";
    case R3D_EINVAL: return "invalid argument";
    case R3D_ERANGE: return "photon time of arrival outside [0, T)";
    case R3D_EOVERFLOW: return "histogram count not an integer in [0, 2048]";
    case R3D_ENOMEM: return "device allocation failed";
    case R3D_EHIP: return "HIP runtime error";
    case R3D_EUNSUPPORTED: return "unsupported size or option";
    case R3D_ETIMEDOUT: return "a batched work item waited past its spin limit";
    case R3D_ETOOBIG: return "batch tables larger than the 4 MiB static scratch array";
  }
  return "unknown status";
}

r3d_status r3d_create(const r3d_params* params, r3d_ctx** out) {
  if (!out) return R3D_EINVAL;
  *out = nullptr;
  r3d_status st = check_params(params);
  if (st != R3D_OK) return st;
  r3d_ctx* c = new (std::nothrow) r3d_ctx();
  if (!c) return R3D_ENOMEM;
  c->prm = *params;
  c->irf.assign(params->irf, params->irf + params->W);
  c->prm.irf = nullptr;
  void* scratch_dev = nullptr;  // resolves the device's scratch address once
  if (hipGetDevice(&c->device) != hipSuccess || scratch_address(&scratch_dev) != hipSuccess) {
    free_ctx(c);
    return R3D_EHIP;
  }
  const int W = params->W;
  double* d_irf64 = nullptr;
  if (hipMalloc(&c->d_h, W * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->d_irf, W * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->d_h16, 2 * W * sizeof(_Float16)) != hipSuccess ||
      hipMalloc(&c->d_err, sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&d_irf64, (W + 1) * sizeof(double)) != hipSuccess) {
    if (d_irf64) (void)hipFree(d_irf64);
    free_ctx(c);
    return R3D_ENOMEM;
  }
  // the largest irf^beta, taken on the device with the same power function
  // as the per-pixel IRF step (d_irf64[W])
  double hmax = 0.0;
  hipError_t e = hipMemcpy(d_irf64, c->irf.data(), W * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->d_err, 0, sizeof(unsigned));
  if (e == hipSuccess)
    e = r3d::launch_prepare_irf(d_irf64, W, params->beta, c->d_h, c->d_irf, c->d_h16,
                                c->d_h16 + W, d_irf64 + W, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&hmax, d_irf64 + W, sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d_irf64);
  if (e != hipSuccess) {
    free_ctx(c);
    return R3D_EHIP;
  }

  r3d::DevModel& m = c->dm;
  m.rows = params->rows;
  m.cols = params->cols;
  m.P = params->rows * params->cols;
  m.T = params->T;
  m.d_lo = params->d_lo;
  m.D = params->D;
  m.W = W;
  m.c = params->c;
  m.beta = (float)params->beta;
  m.beta_d = params->beta;
  m.scale2 = (float)((params->beta + 1.0) / params->beta * 1.4426950408889634);
  m.hmax = (float)(hmax * (1.0 + 1e-6));
  m.m_flat = (float)(0.5 * (params->d_min + params->d_max));
  const double span = params->d_max - params->d_min;
  m.v_flat = (float)(span * span / 12.0);
  m.sigma_rw2 = (float)params->sigma_rw2;
  for (int k = 0; k < 9; ++k) {
    m.nu[k] = (float)params->nu[k];
    m.lognu2[k] = params->nu[k] > 0.0 ? (float)std::log2(params->nu[k]) : -INFINITY;
  }
  m.h = c->d_h;
  m.irf = c->d_irf;
  m.h16hi = c->d_h16;
  m.h16lo = c->d_h16 + W;
  m.err = c->d_err;
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) !=
      hipSuccess) {
    free_ctx(c);
    return R3D_EHIP;
  }
  m.lds_max = lds_max;
  if (!r3d::plain_supported(m)) {
    free_ctx(c);
    return R3D_EUNSUPPORTED;
  }
  *out = c;
  return R3D_OK;
}

void r3d_destroy(r3d_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  free_ctx(ctx);
}

r3d_status r3d_state_init(r3d_ctx* ctx, const r3d_state* st, void* stream) {
  if (!ctx || check_state(st) != R3D_OK) return R3D_EINVAL;
  return hip_status(r3d::launch_state_init(ctx->dm, st->m, st->v, st->pi, st->b,
                                           (hipStream_t)stream));
}

r3d_status r3d_histogram(r3d_ctx* ctx, const int32_t* row_ptr, const int16_t* toa,
                         uint16_t* hist, void* stream) {
  if (!ctx || !row_ptr || !hist) return R3D_EINVAL;
  return hip_status(r3d::launch_histogram(ctx->dm, row_ptr, toa, hist, (hipStream_t)stream));
}

r3d_status r3d_cost(r3d_ctx* ctx, const uint16_t* hist, int32_t npix, float* ell, void* stream) {
  if (!ctx || !hist || !ell || npix < 0) return R3D_EINVAL;
  if (npix == 0) return R3D_OK;
  if (ctx->prm.precision == R3D_FP32)
    return hip_status(r3d::launch_cost_plain(ctx->dm, hist, npix, ell, (hipStream_t)stream));
  return hip_status(r3d::launch_cost_tile(ctx->dm, ctx->prm.precision, hist, npix, ell,
                                          (hipStream_t)stream));
}

r3d_status r3d_step_csr(r3d_ctx* ctx, const int32_t* row_ptr, const int16_t* toa,
                        const float* pi_in, const uint8_t* faulty, const r3d_state* prev,
                        const r3d_state* next, const r3d_out* out, void* stream) {
  if (!ctx || !row_ptr) return R3D_EINVAL;
  if (check_state(prev) != R3D_OK || check_state(next) != R3D_OK) return R3D_EINVAL;
  if (same_buffer(prev, next)) return R3D_EINVAL;
  if (ctx->prm.precision != R3D_FP32) return R3D_EUNSUPPORTED;
  r3d::StepIO io = make_io(pi_in, faulty, prev, next, out);
  io.row_ptr = row_ptr;
  io.toa = toa;
  return hip_status(r3d::launch_step_plain(ctx->dm, io, false, (hipStream_t)stream));
}

r3d_status r3d_step_hist(r3d_ctx* ctx, const uint16_t* hist, const float* pi_in,
                         const uint8_t* faulty, const r3d_state* prev, const r3d_state* next,
                         const r3d_out* out, void* stream) {
  if (!ctx || !hist) return R3D_EINVAL;
  if (check_state(prev) != R3D_OK || check_state(next) != R3D_OK) return R3D_EINVAL;
  if (same_buffer(prev, next)) return R3D_EINVAL;
  r3d::StepIO io = make_io(pi_in, faulty, prev, next, out);
  io.hist = hist;
  const int engine = ctx->prm.precision;  // r3d_precision values are the engine ids
  const hipStream_t s = (hipStream_t)stream;
  if (r3d::tile_supported(ctx->dm, engine) && ((uintptr_t)hist & 15u) == 0)
    return hip_status(r3d::launch_step_tile(ctx->dm, engine, io, s));
  if (engine != R3D_FP32) return R3D_EUNSUPPORTED;
  return hip_status(r3d::launch_step_plain(ctx->dm, io, true, s));
}

r3d_status r3d_run_hist(r3d_ctx* ctx, const uint16_t* const* hist, int32_t nframes,
                        const float* pi_in, const uint8_t* faulty, const r3d_state* state,
                        const r3d_out* out, void* stream) {
  if (!ctx || !hist || !state || nframes < 1) return R3D_EINVAL;
  if (check_state(&state[0]) != R3D_OK || check_state(&state[1]) != R3D_OK) return R3D_EINVAL;
  if (same_buffer(&state[0], &state[1])) return R3D_EINVAL;
  for (int n = 0; n < nframes; ++n) {
    if (!hist[n]) return R3D_EINVAL;
    if ((uintptr_t)hist[n] & 15u) return R3D_EUNSUPPORTED;
  }
  const int engine = ctx->prm.precision;
  if (!r3d::tile_supported(ctx->dm, engine)) return R3D_EUNSUPPORTED;
  const hipStream_t s = (hipStream_t)stream;
  const size_t P = (size_t)ctx->dm.P;
  for (int f = 0; f < nframes; ++f) {
    const size_t o = (size_t)f * P;
    r3d_out of{};
    if (out) {
      of.depth = out->depth ? out->depth + o : nullptr;
      of.var = out->var ? out->var + o : nullptr;
      of.intensity = out->intensity ? out->intensity + o : nullptr;
      of.background = out->background ? out->background + o : nullptr;
      of.pi0_next = out->pi0_next ? out->pi0_next + o : nullptr;
      of.argmax = out->argmax ? out->argmax + o : nullptr;
    }
    r3d::StepIO io = make_io(pi_in ? pi_in + o : nullptr, faulty, &state[f % 2], &state[(f + 1) % 2], &of);
    io.hist = hist[f];
    const r3d_status st = hip_status(r3d::launch_step_tile(ctx->dm, engine, io, s));
    if (st != R3D_OK) return st;
  }
  return R3D_OK;
}

r3d_status r3d_step_pirf(r3d_ctx* ctx, const int32_t* row_ptr, const int16_t* toa,
                         const uint16_t* hist, const double* irf_pix, const int32_t* c_pix,
                         const float* pi_in, const uint8_t* faulty, const r3d_state* prev,
                         const r3d_state* next, const r3d_out* out, void* stream) {
  if (!ctx || !irf_pix) return R3D_EINVAL;
  if ((row_ptr != nullptr) == (hist != nullptr)) return R3D_EINVAL;  // exactly one input form
  if (check_state(prev) != R3D_OK || check_state(next) != R3D_OK) return R3D_EINVAL;
  if (same_buffer(prev, next)) return R3D_EINVAL;
  r3d::StepIO io = make_io(pi_in, faulty, prev, next, out);
  io.row_ptr = row_ptr;
  io.toa = toa;
  io.hist = hist;
  return hip_status(r3d::launch_step_pirf(ctx->dm, io, hist != nullptr, irf_pix, c_pix,
                                          (hipStream_t)stream));
}

r3d_status r3d_min_divergence(r3d_ctx* ctx, const uint16_t* hist, int32_t* argmax, float* value,
                              void* stream) {
  if (!ctx || !hist || !argmax) return R3D_EINVAL;
  if ((uintptr_t)hist & 15u) return R3D_EUNSUPPORTED;
  const uint16_t* h[1] = {hist};
  return hip_status(r3d::launch_mindiv(&ctx->dm, h, 1, ctx->prm.precision, false, argmax, value,
                                       (hipStream_t)stream));
}

r3d_status r3d_min_divergence_gauss(r3d_ctx* ctx, const int32_t* row_ptr, const int16_t* toa,
                                    double sigma, float* depth, float* value, int32_t* grid_argmax,
                                    void* stream) {
  if (!ctx || !row_ptr || !toa || !depth) return R3D_EINVAL;
  if (!(sigma > 0.0) || !(sigma <= (double)ctx->prm.T)) return R3D_EINVAL;
  return hip_status(r3d::launch_gauss_mindiv(ctx->dm, row_ptr, toa, sigma, depth, value, grid_argmax,
                                             (hipStream_t)stream));
}

r3d_status r3d_min_divergence_msl(r3d_ctx* const* bands, int32_t nbands,
                                  const uint16_t* const* hist, int32_t* argmax, float* value,
                                  void* stream) {
  if (!bands || !hist || !argmax || nbands < 1) return R3D_EINVAL;
  if (nbands > r3d::kMaxBands) return R3D_EUNSUPPORTED;
  r3d::DevModel M[r3d::kMaxBands];
  const r3d_params& p0 = bands[0] ? bands[0]->prm : r3d_params{};
  for (int l = 0; l < nbands; ++l) {
    if (!bands[l] || !hist[l]) return R3D_EINVAL;
    const r3d_params& p = bands[l]->prm;
    if (p.rows != p0.rows || p.cols != p0.cols || p.T != p0.T || p.d_lo != p0.d_lo ||
        p.D != p0.D || p.beta != p0.beta || p.precision != p0.precision)
      return R3D_EINVAL;
    if ((uintptr_t)hist[l] & 15u) return R3D_EUNSUPPORTED;
    M[l] = bands[l]->dm;
    M[l].err = bands[0]->d_err;  // one error word for the call
  }
  return hip_status(r3d::launch_mindiv(M, hist, nbands, p0.precision, true, argmax, value,
                                       (hipStream_t)stream));
}

}  // extern "C"

struct r3d_batch {
  r3d::SeqDesc* d_seqs = nullptr;
  int* d_prefix = nullptr;
  void** d_ptrs = nullptr;  // every sequence's row_ptr and toa pointer arrays
  unsigned* d_queue = nullptr;
  int* d_done = nullptr;
  unsigned* d_err = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void free_batch(r3d_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_seqs) (void)hipFree(b->d_seqs);
  if (b->d_prefix) (void)hipFree(b->d_prefix);
  if (b->d_ptrs) (void)hipFree(b->d_ptrs);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->d_done) (void)hipFree(b->d_done);
  if (b->d_err) (void)hipFree(b->d_err);
  delete b;
}

r3d_status device_bits(unsigned bits) {
  if (bits & r3d::kErrIrf) return R3D_EINVAL;
  if (bits & r3d::kErrTimeout) return R3D_ETIMEDOUT;
  if (bits & r3d::kErrRange) return R3D_ERANGE;
  if (bits & r3d::kErrOverflow) return R3D_EOVERFLOW;
  return R3D_OK;
}

// First pass over a batch: argument checks and the length of its frame
// pointer table.
r3d_status batch_count(const r3d_sequence* seqs, int32_t nseq, const r3d_batch_options* opt,
                       size_t& nptrs) {
  if (!seqs || nseq < 1) return R3D_EINVAL;
  if (opt && opt->blocks < 0) return R3D_EINVAL;
  nptrs = 0;
  for (int s = 0; s < nseq; ++s) {
    const r3d_sequence& q = seqs[s];
    if (!q.ctx || q.nframes < 1 || !q.row_ptr || !q.toa || q.chunk_rows < 0) return R3D_EINVAL;
    if (check_state(&q.state[0]) != R3D_OK || check_state(&q.state[1]) != R3D_OK) return R3D_EINVAL;
    if (same_buffer(&q.state[0], &q.state[1])) return R3D_EINVAL;
    if (q.ctx->prm.precision != R3D_FP32) return R3D_EUNSUPPORTED;
    for (int n = 0; n < q.nframes; ++n)
      if (!q.row_ptr[n] || !q.toa[n]) return R3D_EINVAL;
    nptrs += 2 * (size_t)q.nframes;
  }
  return R3D_OK;
}

// Second pass: the sequence descriptors, the chunk prefix [nseq + 1] and the
// frame pointer table, written to host memory; d_ptrs is the device address
// the table will have (the descriptors point into it). Fills the geometry
// except its device pointers.
r3d_status batch_fill(const r3d_sequence* seqs, int32_t nseq, const r3d_batch_options* opt,
                      r3d::SeqDesc* desc, int* prefix, void** ptrs, void** d_ptrs,
                      r3d::BatchGeom& G) {
  size_t np = 0;
  int tmax = 1, fmax = 1;
  prefix[0] = 0;
  for (int s = 0; s < nseq; ++s) {
    const r3d_sequence& q = seqs[s];
    const r3d::DevModel& M = q.ctx->dm;
    r3d::SeqDesc& d = desc[s];
    d = r3d::SeqDesc{};
    d.M = M;
    d.nframes = q.nframes;
    d.chunk_rows = q.chunk_rows > 0 ? q.chunk_rows : (256 + M.cols - 1) / M.cols;
    if (d.chunk_rows > M.rows) d.chunk_rows = M.rows;
    d.nchunks = (M.rows + d.chunk_rows - 1) / d.chunk_rows;
    d.done_off = prefix[s];
    prefix[s + 1] = prefix[s] + d.nchunks;
    d.row_ptr = reinterpret_cast<const int32_t* const*>(d_ptrs + np);
    for (int n = 0; n < q.nframes; ++n) ptrs[np++] = (void*)q.row_ptr[n];
    d.toa = reinterpret_cast<const int16_t* const*>(d_ptrs + np);
    for (int n = 0; n < q.nframes; ++n) ptrs[np++] = (void*)q.toa[n];
    for (int i = 0; i < 2; ++i) {
      d.st_m[i] = q.state[i].m;
      d.st_v[i] = q.state[i].v;
      d.st_pi[i] = q.state[i].pi;
      d.st_b[i] = q.state[i].b;
    }
    d.depth = q.out.depth;
    d.var = q.out.var;
    d.intensity = q.out.intensity;
    d.background = q.out.background;
    d.pi0_next = q.out.pi0_next;
    d.argmax = q.out.argmax;
    d.pi_in = q.pi_in;
    d.faulty = q.faulty;
    tmax = std::max(tmax, M.T);
    fmax = std::max(fmax, q.nframes);
  }
  const uint32_t spin_limit = opt ? opt->spin_limit : 0u;
  G = r3d::BatchGeom{};
  G.nseq = nseq;
  G.chunks_total = prefix[nseq];
  G.hist_words = r3d::pixel_lds_words(tmax);
  if (r3d::batch_lds_bytes(G) > 65536) return R3D_EUNSUPPORTED;
  const long long nitems = (long long)fmax * G.chunks_total;
  if (nitems >= (1LL << 31)) return R3D_EUNSUPPORTED;
  G.nitems = (unsigned)nitems;
  G.spin_limit = spin_limit ? spin_limit : (1u << 22);
  G.ndone = G.chunks_total;
  return R3D_OK;
}

int batch_blocks(const r3d::BatchGeom& G, const r3d_batch_options* opt, hipError_t& e) {
  const int req = opt ? opt->blocks : 0;
  if (req > 0) return req;
  int dev = 0, ncu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  return std::max(1, ncu) * r3d::batch_blocks_per_cu(G);
}

}  // namespace

extern "C" {

r3d_status r3d_batch_create(const r3d_sequence* seqs, int32_t nseq,
                            const r3d_batch_options* opt, r3d_batch** out) {
  if (!out) return R3D_EINVAL;
  *out = nullptr;
  size_t nptrs = 0;
  r3d_status st = batch_count(seqs, nseq, opt, nptrs);
  if (st != R3D_OK) return st;
  std::vector<r3d::SeqDesc> host(nseq);
  std::vector<int> prefix(nseq + 1, 0);
  std::vector<void*> ptrs(nptrs);
  r3d_batch* b = new (std::nothrow) r3d_batch();
  if (!b) return R3D_ENOMEM;
  if (hipMalloc(&b->d_ptrs, nptrs * sizeof(void*)) != hipSuccess) {
    free_batch(b);
    return R3D_ENOMEM;
  }
  r3d::BatchGeom G{};
  st = batch_fill(seqs, nseq, opt, host.data(), prefix.data(), ptrs.data(), b->d_ptrs, G);
  if (st != R3D_OK) {
    free_batch(b);
    return st;
  }
  if (hipMalloc(&b->d_seqs, nseq * sizeof(r3d::SeqDesc)) != hipSuccess ||
      hipMalloc(&b->d_prefix, (nseq + 1) * sizeof(int)) != hipSuccess ||
      hipMalloc(&b->d_queue, sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&b->d_done, G.ndone * sizeof(int)) != hipSuccess ||
      hipMalloc(&b->d_err, sizeof(unsigned)) != hipSuccess) {
    free_batch(b);
    return R3D_ENOMEM;
  }
  G.chunk_prefix = b->d_prefix;
  G.queue = b->d_queue;
  G.done = b->d_done;
  G.err = b->d_err;
  hipError_t e = hipSuccess;
  const int blocks = batch_blocks(G, opt, e);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_seqs, host.data(), nseq * sizeof(r3d::SeqDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_prefix, prefix.data(), (nseq + 1) * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_ptrs, ptrs.data(), nptrs * sizeof(void*), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->d_err, 0, sizeof(unsigned));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = r3d::launch_batch(b->d_seqs, G, blocks, b->cap);
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_batch(b);
    return R3D_EHIP;
  }
  *out = b;
  return R3D_OK;
}

r3d_status r3d_batch_launch(r3d_batch* b, void* stream) {
  if (!b) return R3D_EINVAL;
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? R3D_OK : R3D_EHIP;
}

r3d_status r3d_batch_status(r3d_batch* b, void* stream) {
  if (!b) return R3D_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return R3D_EHIP;
  unsigned bits = 0;
  if (hipMemcpy(&bits, b->d_err, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
    return R3D_EHIP;
  if (hipMemset(b->d_err, 0, sizeof(unsigned)) != hipSuccess) return R3D_EHIP;
  return device_bits(bits);
}

void r3d_batch_destroy(r3d_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_batch(b);
}

r3d_status r3d_batch_run_noalloc(const r3d_sequence* seqs, int32_t nseq,
                                 const r3d_batch_options* opt, void* stream) {
  size_t nptrs = 0;
  r3d_status st = batch_count(seqs, nseq, opt, nptrs);
  if (st != R3D_OK) return st;
  // table sections in the scratch array, 256-byte aligned
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_prefix = up((size_t)nseq * sizeof(r3d::SeqDesc));
  const size_t o_ptrs = up(o_prefix + (size_t)(nseq + 1) * sizeof(int));
  const size_t o_queue = up(o_ptrs + nptrs * sizeof(void*));
  const size_t o_done = o_queue + 256;
  if (o_done > kBatchScratchBytes) return R3D_ETOOBIG;
  void* addr = nullptr;
  if (scratch_address(&addr) != hipSuccess) return R3D_EHIP;
  unsigned char* base = static_cast<unsigned char*>(addr);
  const hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_stage_mu);
  r3d::BatchGeom G{};
  st = batch_fill(seqs, nseq, opt, reinterpret_cast<r3d::SeqDesc*>(g_stage),
                  reinterpret_cast<int*>(g_stage + o_prefix),
                  reinterpret_cast<void**>(g_stage + o_ptrs),
                  reinterpret_cast<void**>(base + o_ptrs), G);
  if (st != R3D_OK) return st;
  if (o_done + (size_t)G.ndone * sizeof(int) > kBatchScratchBytes) return R3D_ETOOBIG;
  G.chunk_prefix = reinterpret_cast<const int*>(base + o_prefix);
  G.queue = reinterpret_cast<unsigned*>(base + o_queue);
  G.done = reinterpret_cast<int*>(base + o_done);
  G.err = seqs[0].ctx->d_err;
  hipError_t e = hipSuccess;
  const int blocks = batch_blocks(G, opt, e);
  // the staging area serves the next call: its upload ends before the
  // launch (the work counter and done counters are cleared by the launch)
  if (e == hipSuccess) e = hipMemcpyAsync(base, g_stage, o_queue, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess)
    e = r3d::launch_batch(reinterpret_cast<const r3d::SeqDesc*>(base), G, blocks, s);
  return e == hipSuccess ? R3D_OK : R3D_EHIP;
}

}  // extern "C"

namespace {

// Workspace of the differentiable filter (offsets in bytes, 256-aligned).
struct GradLayout {
  int N = 0, E = 0, nseg = 0, npar = 0;
  size_t P = 0, state_bytes = 0;
  size_t ckpt = 0, seg = 0, lnz = 0, am = 0, av = 0, cm = 0, cv = 0, pib = 0, bb = 0, part = 0;
  size_t bytes = 0;
  r3d::AdjGeom geo{};
};

bool grad_layout(const r3d::DevModel& M, int N, int E, GradLayout& L) {
  L.geo = r3d::adjoint_geometry(M);
  if (L.geo.waves == 0) return false;
  L.N = N;
  L.E = E;
  L.nseg = (N + E - 1) / E;
  L.P = (size_t)M.P;
  L.npar = r3d::kThetaFixed + M.W;
  L.state_bytes = 4 * L.P * sizeof(float);  // m, v, pi, b
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  L.ckpt = take(L.nseg * L.state_bytes);
  L.seg = take((size_t)E * L.state_bytes);
  L.lnz = take((size_t)E * L.P * sizeof(float));
  L.am = take(2 * L.P * sizeof(float));
  L.av = take(2 * L.P * sizeof(float));
  L.cm = take(9 * L.P * sizeof(float));
  L.cv = take(9 * L.P * sizeof(float));
  L.pib = take(2 * L.P * sizeof(float));
  L.bb = take(2 * L.P * sizeof(float));
  L.part = take((size_t)L.geo.blocks * L.npar * sizeof(float));
  L.bytes = off;
  return true;
}

r3d_state state_at(char* base, size_t off, size_t P) {
  float* f = reinterpret_cast<float*>(base + off);
  return r3d_state{f, f + P, f + 2 * P, f + 3 * P};
}

hipError_t copy_state(const r3d_state& dst, const r3d_state& src, size_t P, hipStream_t s) {
  const float* a[4] = {src.m, src.v, src.pi, src.b};
  float* b[4] = {dst.m, dst.v, dst.pi, dst.b};
  for (int i = 0; i < 4; ++i) {
    const hipError_t e =
        hipMemcpyAsync(b[i], a[i], P * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

r3d_status check_frames(const r3d_frames* f) {
  if (!f || f->nframes < 1 || !f->row_ptr || !f->toa) return R3D_EINVAL;
  for (int n = 0; n < f->nframes; ++n)
    if (!f->row_ptr[n] || !f->toa[n]) return R3D_EINVAL;
  return R3D_OK;
}

hipError_t forward_frame(const r3d::DevModel& M, const r3d_frames* f, int n, const r3d_state& prev,
                         const r3d_state& next, hipStream_t s, float* lognorm = nullptr) {
  const float* pin = f->pi_in ? f->pi_in + (size_t)n * M.P : nullptr;
  r3d::StepIO io = make_io(pin, f->faulty, &prev, &next, nullptr);
  io.lognorm = lognorm;
  io.row_ptr = f->row_ptr[n];
  io.toa = f->toa[n];
  return r3d::launch_step_plain(M, io, false, s);
}

}  // namespace

extern "C" {

r3d_status r3d_grad_workspace_size(const r3d_ctx* ctx, int32_t nframes, int32_t ckpt_every,
                                   size_t* bytes) {
  if (!ctx || !bytes || nframes < 1 || ckpt_every < 1) return R3D_EINVAL;
  GradLayout L;
  if (!grad_layout(ctx->dm, nframes, ckpt_every, L)) return R3D_EUNSUPPORTED;
  *bytes = L.bytes;
  return R3D_OK;
}

r3d_status r3d_filter_forward(r3d_ctx* ctx, const r3d_frames* frames, int32_t ckpt_every,
                              const r3d_state* init, float* mean, float* var, void* workspace,
                              size_t workspace_bytes, void* stream) {
  if (!ctx || !mean || !var || !workspace || ckpt_every < 1) return R3D_EINVAL;
  if (check_frames(frames) != R3D_OK || check_state(init) != R3D_OK) return R3D_EINVAL;
  const r3d::DevModel& M = ctx->dm;
  GradLayout L;
  if (!grad_layout(M, frames->nframes, ckpt_every, L)) return R3D_EUNSUPPORTED;
  if (workspace_bytes < L.bytes) return R3D_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  char* base = static_cast<char*>(workspace);
  float* pib = reinterpret_cast<float*>(base + L.pib);
  float* bb = reinterpret_cast<float*>(base + L.bb);
  r3d_state prev = *init;
  hipError_t e = hipSuccess;
  for (int n = 0; n < L.N && e == hipSuccess; ++n) {
    if (n % L.E == 0) e = copy_state(state_at(base, L.ckpt + (n / L.E) * L.state_bytes, L.P), prev,
                                     L.P, s);
    const r3d_state next{mean + (size_t)n * L.P, var + (size_t)n * L.P, pib + (n & 1) * L.P,
                         bb + (n & 1) * L.P};
    if (e == hipSuccess) e = forward_frame(M, frames, n, prev, next, s);
    prev = next;
  }
  return hip_status(e);
}

r3d_status r3d_filter_backward(r3d_ctx* ctx, const r3d_frames* frames, int32_t ckpt_every,
                               const float* grad_mean, const float* grad_var, void* workspace,
                               size_t workspace_bytes, double* grad, void* stream) {
  if (!ctx || !grad_mean || !grad || !workspace || ckpt_every < 1) return R3D_EINVAL;
  if (check_frames(frames) != R3D_OK) return R3D_EINVAL;
  const r3d::DevModel& M = ctx->dm;
  GradLayout L;
  if (!grad_layout(M, frames->nframes, ckpt_every, L)) return R3D_EUNSUPPORTED;
  if (workspace_bytes < L.bytes) return R3D_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  char* base = static_cast<char*>(workspace);
  const size_t P = L.P;
  float* am[2] = {reinterpret_cast<float*>(base + L.am), reinterpret_cast<float*>(base + L.am) + P};
  float* av[2] = {reinterpret_cast<float*>(base + L.av), reinterpret_cast<float*>(base + L.av) + P};
  float* cm = reinterpret_cast<float*>(base + L.cm);
  float* cv = reinterpret_cast<float*>(base + L.cv);
  float* part = reinterpret_cast<float*>(base + L.part);
  const int N = L.N;

  hipError_t e = r3d::launch_fill_f64(grad, (size_t)L.npar, 0.0, s);
  int cur = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(am[cur], grad_mean + (size_t)(N - 1) * P, P * sizeof(float),
                       hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = grad_var ? hipMemcpyAsync(av[cur], grad_var + (size_t)(N - 1) * P, P * sizeof(float),
                                  hipMemcpyDeviceToDevice, s)
                 : r3d::launch_fill_f32(av[cur], P, 0.f, s);
  for (int sg = L.nseg - 1; sg >= 0 && e == hipSuccess; --sg) {
    const int f0 = sg * L.E;
    const int f1 = std::min(N, f0 + L.E);
    const r3d_state ck = state_at(base, L.ckpt + sg * L.state_bytes, P);
    // recompute the segment's frames: the state after each, and each
    // frame's posterior normaliser (its moments are the state after it)
    float* lnz = reinterpret_cast<float*>(base + L.lnz);
    r3d_state prev = ck;
    for (int n = f0; n < f1 && e == hipSuccess; ++n) {
      const r3d_state next = state_at(base, L.seg + (n - f0) * L.state_bytes, P);
      e = forward_frame(M, frames, n, prev, next, s, lnz + (size_t)(n - f0) * P);
      prev = next;
    }
    for (int n = f1 - 1; n >= f0 && e == hipSuccess; --n) {
      const r3d_state before =
          n == f0 ? ck : state_at(base, L.seg + (n - 1 - f0) * L.state_bytes, P);
      const r3d_state after = state_at(base, L.seg + (n - f0) * L.state_bytes, P);
      r3d::AdjIO io{};
      io.row_ptr = frames->row_ptr[n];
      io.toa = frames->toa[n];
      io.faulty = frames->faulty;
      io.pm = before.m;
      io.pv = before.v;
      io.ppi = before.pi;
      io.mean = after.m;
      io.var = after.v;
      io.lognorm = lnz + (size_t)(n - f0) * P;
      io.gm = am[cur];
      io.gv = av[cur];
      io.cm = cm;
      io.cv = cv;
      io.part = part;
      e = r3d::launch_adjoint(M, io, L.geo, s);
      if (e == hipSuccess) e = r3d::launch_theta_reduce(M, part, L.geo.blocks, grad, s);
      if (e == hipSuccess && n > 0) {
        e = r3d::launch_adjoint_gather(M, cm, cv, grad_mean + (size_t)(n - 1) * P,
                                       grad_var ? grad_var + (size_t)(n - 1) * P : nullptr,
                                       am[cur ^ 1], av[cur ^ 1], s);
        cur ^= 1;
      }
    }
  }
  return hip_status(e);
}

r3d_status r3d_last_device_status(r3d_ctx* ctx, void* stream) {
  if (!ctx) return R3D_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return R3D_EHIP;
  unsigned bits = 0;
  if (hipMemcpy(&bits, ctx->d_err, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
    return R3D_EHIP;
  if (hipMemset(ctx->d_err, 0, sizeof(unsigned)) != hipSuccess) return R3D_EHIP;
  return device_bits(bits);
}

}  // extern "C"
