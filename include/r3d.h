/*
 * r3d.h - C ABI of the R3DSP per-frame hot path on AMD Instinct MI355X (gfx950).
 *
 * R3DSP is the online single-photon lidar reconstruction of Legros et al.,
 * "Robust 3D reconstruction of dynamic scenes from single-photon lidar using
 * Beta-divergences" (arXiv:2004.09211). For every pixel of a frame the
 * library
 *   (a1) histograms the photon times of arrival (ToAs) of the pixel (Sec. II-A,
 *        discrete Poisson model),
 *   (a3) evaluates the beta-divergence log pseudo-likelihood on the depth grid,
 *        ell(d) = (beta+1)/beta * sum_j irf[j]^beta * z[d - c + j]
 *        (Sec. II-B, eq. beta_div2 and its histogram form),
 *   (a4) builds the spatio-temporal prior: a Gaussian mixture over the 3x3
 *        neighbourhood of the previous frame convolved with a Gaussian random
 *        walk, with flat components for undetected or out-of-frame neighbours
 *        (Sec. III-A, eq. predict),
 *   (a5) normalises the pseudo-posterior on the grid and extracts its argmax,
 *        mean and variance (Sec. II-C, eq. approx_post; Sec. III-A, eq. KL_div),
 *   (a6) writes the new Gaussian state and the depth (NaN when undetected),
 *   (a7) estimates background and reflectivity (Sec. II-E, eq. lik_bg_poisson),
 * and the prior presence probability of the next frame (Sec. III-B,
 * eq. prior_detect), i.e. one iteration of Algorithm 1 for every pixel.
 *
 * Units: every time and depth is in histogram bins. A surface at depth d puts
 * tap j of the IRF into bin t = d - c + j, c being the tap of the IRF maximum.
 * The depth grid is d = d_lo .. d_lo + D - 1; bins outside [0, T) count zero.
 *
 * Memory: every array argument of a step is DEVICE memory owned by the
 * caller; the library keeps no caller pointer past the call. The library owns
 * only its context (the uploaded IRF, its powers and an error word).
 * Streams: calls enqueue on the given stream (a hipStream_t passed as void*,
 * NULL = the default stream) and never synchronise, except r3d_create,
 * r3d_last_device_status and r3d_destroy. A context is used by one stream at a
 * time.
 * Errors: parameter and shape errors are returned synchronously before any
 * launch. Data-dependent faults found by a kernel (a ToA outside [0, T), an
 * fp16 count that is not an integer in [0, 2048] or has its sign bit set, an
 * invalid per-pixel IRF) set the context's device error word, read back by
 * r3d_last_device_status; the affected outputs are then undefined.
 */
#ifndef R3D_H
#define R3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    R3D_OK = 0,
    R3D_EINVAL = -1,        /* bad parameter, shape or NULL pointer             */
    R3D_ERANGE = -2,        /* a ToA outside [0, T) (device-detected)           */
    R3D_EOVERFLOW = -3,     /* an fp16 count not an integer in [0, 2048], or -0 */
    R3D_ENOMEM = -4,        /* device allocation failed                         */
    R3D_EHIP = -5,          /* a HIP runtime call failed                        */
    R3D_EUNSUPPORTED = -6,  /* size or option outside what the kernels support  */
    R3D_ETIMEDOUT = -7,     /* a batched item waited past its spin limit        */
    R3D_ETOOBIG = -8        /* tables beyond r3d_batch_run_noalloc's scratch    */
} r3d_status;

/* How the cost correlation (a3) is evaluated.
 * R3D_FP32: fp32 vector FMAs (the plain form).
 * R3D_FP16_MFMA: banded Toeplitz contraction on the matrix cores with fp16
 *   counts and fp16 irf^beta, fp32 accumulation (histogram input only).
 * R3D_FP16X2_MFMA: as above with irf^beta split into an fp16 high part and an
 *   fp16 low part (two contractions), about 22 significant bits. */
typedef enum {
    R3D_FP32 = 0,
    R3D_FP16_MFMA = 1,
    R3D_FP16X2_MFMA = 2
} r3d_precision;

typedef struct r3d_ctx r3d_ctx;

/* Model parameters (Algorithm 1 fixed inputs plus the observation model). */
typedef struct {
    int32_t rows, cols;     /* frame size, P = rows*cols, pixel p = row*cols + col */
    int32_t T;              /* timing bins per histogram, 1 <= T <= 32767          */
    int32_t d_lo, D;        /* depth grid d_lo .. d_lo+D-1, 1 <= D <= 32768        */
    double  d_min, d_max;   /* bounds of the flat prior component, d_max > d_min   */
    double  beta;           /* beta-divergence parameter, beta > 0                 */
    int32_t W, c;           /* IRF taps (1..256) and tap of its maximum (0..W-1)   */
    const double *irf;      /* HOST pointer, W non-negative taps, used verbatim    */
    double  nu[9];          /* 3x3 mixture weights, row-major, centre nu[4], >= 0  */
    double  sigma_rw2;      /* random-walk variance, > 0                           */
    int32_t precision;      /* r3d_precision                                       */
} r3d_params;

/* Filter state of one frame, device arrays of P floats each (caller-owned):
 * q = N(m, v) per pixel, presence probability pi, background level b. */
typedef struct {
    float *m, *v, *pi, *b;
} r3d_state;

/* Per-pixel outputs of one frame, device arrays of P elements (caller-owned).
 * Any pointer may be NULL to skip that output. depth is the posterior mean
 * where pi > 0.5 and NaN elsewhere; var the posterior variance; argmax the
 * grid depth of the pseudo-posterior maximum (lowest on ties); intensity and
 * background the reflectivity / background estimates; pi0_next the prior
 * presence probability of the next frame. */
typedef struct {
    float   *depth, *var, *intensity, *background, *pi0_next;
    int32_t *argmax;
} r3d_out;

/* Create a context on the current HIP device: validates the parameters,
 * uploads irf and the modified IRF irf^beta of Sec. II-B (the taps the
 * cost correlates with the histogram). Synchronous. Returns R3D_EINVAL on
 * a bad parameter (beta <= 0 (Sec. II-B requires beta > 0), sigma_rw2 <= 0,
 * W out of range, c outside [0, W), negative or all-zero irf or nu,
 * d_max <= d_min, empty sizes, d_lo outside [-2^20, 2^20]). */
r3d_status r3d_create(const r3d_params *params, r3d_ctx **out);

/* Destroy a context and free its device memory (synchronises the device
 * first). NULL is ignored. */
void r3d_destroy(r3d_ctx *ctx);

/* Initial state of Algorithm 1 (Sec. III-B, its initialisation of q and of
 * the presence probabilities, whose values the paper leaves open): every
 * pixel flat, m = (d_min+d_max)/2, v = (d_max-d_min)^2/12 (the flat
 * Gaussian of Sec. III-A), pi = 0.5, b = 0. st: four device arrays of P. */
r3d_status r3d_state_init(r3d_ctx *ctx, const r3d_state *st, void *stream);

/* a1 alone: per-pixel photon-count histogram of a CSR photon list (Sec. II-A:
 * z_t counts the pixel's ToAs in bin t, eq. lik_ideal_poisson), written as
 * fp16 [P][T] (IEEE binary16 bits). row_ptr: int32[P+1], non-decreasing,
 * row_ptr[0] = 0; toa: int16[row_ptr[P]], any order inside a pixel. Counts
 * are exact up to 2048; a larger count sets R3D_EOVERFLOW, a ToA outside
 * [0, T) sets R3D_ERANGE (device error word). */
r3d_status r3d_histogram(r3d_ctx *ctx, const int32_t *row_ptr, const int16_t *toa,
                         uint16_t *hist, void *stream);

/* a3 alone, for inspection and tests: the log pseudo-likelihood
 * ell(d) = (beta+1)/beta * sum_j irf[j]^beta z[d-c+j] (Sec. II-B, histogram
 * form of eq. beta_div2; Sec. II-C, eq. beta_CE) for npix pixels of an fp16
 * histogram [npix][T] (device), written as float [npix][D] (device) in
 * natural-log units, with the context's precision. */
r3d_status r3d_cost(r3d_ctx *ctx, const uint16_t *hist, int32_t npix, float *ell,
                    void *stream);

/* One frame of Algorithm 1 from CSR photon lists (a1..a7 fused).
 * pi_in: float[P] presence probabilities of this frame from the caller's
 * detector, or NULL (every pixel detected, pi = 1). faulty: uint8[P] mask of
 * pixels without observations, or NULL; a faulty pixel keeps its prior as
 * pseudo-posterior and gets pi = 0.5 (Sec. III-B). prev is read, next is
 * written; they must not alias. Only R3D_FP32 evaluates photon lists. */
r3d_status r3d_step_csr(r3d_ctx *ctx, const int32_t *row_ptr, const int16_t *toa,
                        const float *pi_in, const uint8_t *faulty,
                        const r3d_state *prev, const r3d_state *next,
                        const r3d_out *out, void *stream);

/* One frame of Algorithm 1 from fp16 histograms [P][T] (IEEE binary16 bits,
 * integer counts 0..2048). Same semantics as r3d_step_csr; the cost is
 * evaluated with the context's precision. */
r3d_status r3d_step_hist(r3d_ctx *ctx, const uint16_t *hist,
                         const float *pi_in, const uint8_t *faulty,
                         const r3d_state *prev, const r3d_state *next,
                         const r3d_out *out, void *stream);

/* Consecutive frames of fp16 histograms through Algorithm 1 (Sec. III-B),
 * each frame exactly as r3d_step_hist computes it (bit-identical results):
 * one launch of the tile kernel per frame on the given stream, with no host
 * round trip between frames.
 * hist: HOST array of nframes DEVICE pointers, each fp16 [P][T] as for
 * r3d_step_hist and 16-byte aligned (else R3D_EUNSUPPORTED). Frame n reads
 * state[n % 2] and writes state[(n + 1) % 2]; state[0] holds the state before
 * the first frame; the two states must not alias. pi_in: device
 * [nframes * P], frame-major, or NULL (every pixel detected). faulty: device
 * [P] mask applied to every frame, or NULL. out: device arrays of
 * nframes * P elements, frame-major; any pointer may be NULL.
 * R3D_EUNSUPPORTED when T is not a multiple of 8 or the IRF is too long for
 * the tile kernels (r3d_step_hist then still runs R3D_FP32 contexts).
 * Asynchronous. The context keeps no per-call buffers for this call: only
 * its error word is shared with other calls. */
r3d_status r3d_run_hist(r3d_ctx *ctx, const uint16_t *const *hist, int32_t nframes,
                        const float *pi_in, const uint8_t *faulty, const r3d_state *state,
                        const r3d_out *out, void *stream);

/* Synchronise the stream, then read and clear the device error word: the
 * data checks of the calls above (a ToA outside the timing window (0, T) of
 * Sec. II-A: R3D_ERANGE; a histogram count that is not an integer in
 * [0, 2048]: R3D_EOVERFLOW; an invalid per-pixel IRF: R3D_EINVAL). Returns
 * R3D_OK or the first kind recorded. */
r3d_status r3d_last_device_status(r3d_ctx *ctx, void *stream);

/* ---------------------------------------------------------------------------
 * Minimum-divergence (pseudo-ML) depth estimates: the cost alone, no prior.
 * ------------------------------------------------------------------------- */

/* Minimum beta-divergence depth of each pixel (Sec. II-B, last paragraph:
 * eq. beta_div2 minimised over d without prior information, i.e. the depth
 * maximising the histogram correlation ell(d)). hist: device fp16 [P][T]
 * (integer counts in [0, 2048], 16-byte aligned, T a multiple of 8).
 * argmax: device int32 [P], the first grid depth of the maximum (d_lo when
 * ell vanishes everywhere); value: device float [P] or NULL, ell there in
 * natural-log units. Evaluated with the context's precision. Asynchronous;
 * count errors set R3D_EOVERFLOW in the device error word. */
r3d_status r3d_min_divergence(r3d_ctx *ctx, const uint16_t *hist, int32_t *argmax, float *value,
                              void *stream);

/* Minimum multispectral beta-divergence depth of each pixel (Appendix,
 * eq. div_MSL): maximises sum over bands of log(c_l(d) / K_l), c_l the
 * correlation of band l's histogram with its own irf_l^beta and K_l its
 * photon count; bands without photons are left out. bands: HOST array of
 * nbands contexts (1 <= nbands <= 4), one per band with its own IRF and peak
 * tap, sharing rows, cols, T, d_lo, D, beta and precision (else R3D_EINVAL).
 * hist: HOST array of nbands DEVICE pointers, fp16 [P][T] as for
 * r3d_min_divergence. argmax: device int32 [P] (d_lo when the objective is
 * -inf everywhere); value: device float [P] or NULL, the objective there
 * (natural log, -inf when some band's correlation vanishes everywhere).
 * Count errors are recorded in the first band's error word. */
r3d_status r3d_min_divergence_msl(r3d_ctx *const *bands, int32_t nbands,
                                  const uint16_t *const *hist, int32_t *argmax, float *value,
                                  void *stream);

/* Continuous minimum-divergence depth of each pixel for a Gaussian IRF
 * (Sec. II-B, eq. beta_div2 in its photon form with f0(y|d) = N(y; d,
 * sigma^2) of unit integral; Sec. V: the correlation may be continuous and a
 * Gaussian IRF simplifies the updates). The photon sum is, up to a constant
 * factor, sum_k exp(-beta (y_k - d)^2 / (2 sigma^2)) with the ToAs y_k taken
 * as bin indices; it is maximised over real d in [d_lo, d_lo + D - 1] by the
 * stationarity fixed point d = sum w_k y_k / sum w_k started from the first
 * grid maximiser (the local maximum of that maximiser's basin; a basin whose
 * peak lies beyond the span ends at the span's end). Uses the context's
 * rows, cols, T, d_lo, D and beta; its IRF is not used. row_ptr, toa: CSR
 * photon lists as for r3d_step_csr. sigma: the IRF's standard deviation in
 * bins, 0 < sigma <= T (else R3D_EINVAL). depth: device float [P]; value:
 * device float [P] or NULL, (beta+1)/beta * sum_k f0(y_k|d)^beta at the
 * depth (natural-log units); grid_argmax: device int32 [P] or NULL, the grid
 * maximiser. Evaluated in fp32; terms below 2^-40 of one photon's peak are
 * dropped, so a pixel without photons, or whose photons all lie beyond that
 * radius, sigma sqrt(80 / (beta log2(e))) bins, of every grid depth, gets
 * d_lo and 0. Asynchronous; a ToA outside [0, T) sets R3D_ERANGE in the
 * device error word. */
r3d_status r3d_min_divergence_gauss(r3d_ctx *ctx, const int32_t *row_ptr, const int16_t *toa,
                                    double sigma, float *depth, float *value,
                                    int32_t *grid_argmax, void *stream);

/* ---------------------------------------------------------------------------
 * Pixel-dependent IRFs (Sec. II-A: the method applies when the shape of the
 * IRF depends on the pixel).
 * ------------------------------------------------------------------------- */

/* One frame of Algorithm 1 as r3d_step_csr / r3d_step_hist, every pixel with
 * its own IRF: the cost, the candidate bound and the background /
 * reflectivity estimate use the pixel's taps. Exactly one input form:
 * row_ptr + toa (CSR photon lists, as r3d_step_csr; hist NULL) or hist
 * (device fp16 [P][T], any T; row_ptr and toa NULL). irf_pix: device double
 * [P][W] (the context's W), row p the IRF of pixel p, non-negative with a
 * positive tap, used verbatim; c_pix: device int32 [P], the tap of each
 * pixel's IRF maximum (its depth reference, Sec. II-D), or NULL for the
 * context's c. irf^beta is taken per pixel exactly as the context's IRF, so
 * equal rows give the results of r3d_step_csr / r3d_step_hist. Evaluated in
 * fp32 (one wavefront per pixel) whatever the context's precision. An
 * invalid row or peak tap sets R3D_EINVAL in the device error word and
 * leaves that pixel's outputs unwritten. Asynchronous. */
r3d_status r3d_step_pirf(r3d_ctx *ctx, const int32_t *row_ptr, const int16_t *toa,
                         const uint16_t *hist, const double *irf_pix, const int32_t *c_pix,
                         const float *pi_in, const uint8_t *faulty, const r3d_state *prev,
                         const r3d_state *next, const r3d_out *out, void *stream);

/* ---------------------------------------------------------------------------
 * Batched sequences in one persistent launch.
 *
 * Many independent sequences of photon-list frames (each with its own
 * context: resolution, bins, IRF, beta, ...) are run through Algorithm 1 by
 * one persistent kernel. Work items are (frame, sequence, band of image
 * rows); an item of frame n starts once frame n-1 of its band and of the two
 * neighbouring bands is done (the 3x3 prior of Sec. III-A reads one halo row),
 * so frames of different sequences and bands overlap freely. The launch
 * (a small counter reset plus the persistent kernel) is captured once into a
 * HIP graph at creation and replayed by r3d_batch_launch.
 * ------------------------------------------------------------------------- */
typedef struct {
    r3d_ctx *ctx;                  /* model of this sequence (precision R3D_FP32)        */
    int32_t nframes;               /* >= 1                                               */
    const int32_t *const *row_ptr; /* HOST array of nframes DEVICE pointers, int32[P+1]  */
    const int16_t *const *toa;     /* HOST array of nframes DEVICE pointers              */
    r3d_state state[2];            /* device; frame n reads state[n % 2] and writes
                                      state[(n+1) % 2]; state[0] must hold the initial
                                      state when the batch is launched                    */
    r3d_out out;                   /* device arrays of nframes*P elements, frame-major;
                                      any pointer may be NULL                             */
    const float *pi_in;            /* device [nframes*P] presence probabilities or NULL  */
    const uint8_t *faulty;         /* device [P] mask or NULL                            */
    int32_t chunk_rows;            /* image rows per work item, 0 = library default      */
} r3d_sequence;

typedef struct r3d_batch r3d_batch;

/* Launch options of a batch; a NULL pointer or zero fields take defaults. */
typedef struct {
    uint32_t spin_limit;  /* dependency polls per item before R3D_ETIMEDOUT is
                             recorded and the item proceeds (0 = a default far
                             above any legitimate wait)                         */
    int32_t blocks;       /* persistent workgroups (0 = compute units times the
                             workgroups that fit on one)                        */
} r3d_batch_options;

/* Validate the sequences, upload their descriptors (the pointers are kept:
 * the caller's buffers must stay allocated while the batch exists), size the
 * work queue and capture the launch into a graph. Synchronous. Histogram
 * lengths up to 7468 bins; R3D_EUNSUPPORTED for longer ones or a context
 * whose precision is not R3D_FP32. */
r3d_status r3d_batch_create(const r3d_sequence *seqs, int32_t nseq,
                            const r3d_batch_options *opt, r3d_batch **out);

/* Replay the captured launch on the stream (asynchronous). */
r3d_status r3d_batch_launch(r3d_batch *batch, void *stream);

/* Synchronise the stream, then read and clear the batch's device error word
 * (R3D_OK, R3D_ETIMEDOUT, R3D_ERANGE or R3D_EOVERFLOW). */
r3d_status r3d_batch_status(r3d_batch *batch, void *stream);

/* Destroy a batch (synchronises the device first). NULL is ignored. */
void r3d_batch_destroy(r3d_batch *batch);

/* For callers that cannot allocate device memory (serving loops that must
 * not call hipMalloc or hipFree): the batch of r3d_batch_create run once on
 * the stream, without creating a batch object and without any allocation.
 * The sequence descriptors, frame pointer table, work counter and done
 * counters live in a static device array of 4 MiB per GPU (held until the
 * process ends); tables larger than that (about 336 bytes per sequence, 16
 * per frame and 4 per chunk of rows, in 256-byte aligned sections) return
 * R3D_ETOOBIG before anything is enqueued. Arguments,
 * checks and results are those of r3d_batch_create + r3d_batch_launch; the
 * outputs are bit-identical. Device errors (R3D_ETIMEDOUT, R3D_ERANGE,
 * R3D_EOVERFLOW) are recorded in seqs[0].ctx's error word: read them with
 * r3d_last_device_status(seqs[0].ctx, stream). The call blocks until its
 * tables are uploaded (it synchronises the stream once, before the launch),
 * then returns with the batch running. Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other host threads, other streams)
 * race and give undefined results. Not for use under stream capture. */
r3d_status r3d_batch_run_noalloc(const r3d_sequence *seqs, int32_t nseq,
                                 const r3d_batch_options *opt, void *stream);

/* ---------------------------------------------------------------------------
 * Differentiable filter.
 *
 * r3d_filter_forward runs Algorithm 1 over a sequence of photon-list frames
 * and returns every frame's posterior mean and variance (the Gaussian state
 * of eq. KL_div, Sec. III-A). r3d_filter_backward returns the gradient of a
 * scalar loss J of those outputs, given dJ/dmean and dJ/dvar, with respect to
 * the model parameters: beta (Sec. II-B), the IRF taps, sigma_rw2 and the 3x3
 * weights nu (Sec. III-A, eq. predict). The posterior mean is the
 * soft-argmax of the log pseudo-posterior at temperature one bin (Sec. II-C,
 * eq. approx_post). Presence probabilities (pi_in) and faulty masks are
 * inputs, not differentiated. The backward keeps only a checkpoint state
 * every ckpt_every frames from the forward and recomputes the states inside
 * each segment; the result does not depend on ckpt_every (bit-identical).
 * Both calls are asynchronous on the stream and need the same workspace.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t nframes;               /* >= 1                                                  */
    const int32_t *const *row_ptr; /* HOST array of nframes DEVICE pointers, int32[P+1]     */
    const int16_t *const *toa;     /* HOST array of nframes DEVICE pointers                 */
    const float *pi_in;            /* device [nframes*P] presence probabilities, or NULL    */
    const uint8_t *faulty;         /* device [P] mask, or NULL                              */
} r3d_frames;

/* Device workspace bytes for a sequence of nframes with this checkpoint
 * interval (R3D_EUNSUPPORTED when the model's T, D, W do not fit the
 * adjoint kernel's LDS: about D + 0.53 T + 2 W <= 16000 words). */
r3d_status r3d_grad_workspace_size(const r3d_ctx *ctx, int32_t nframes, int32_t ckpt_every,
                                   size_t *bytes);

/* Forward pass. init: the state before the first frame (device, read only).
 * mean, var: device float[nframes*P], frame-major (the filter state after
 * each frame). workspace: device, at least r3d_grad_workspace_size bytes,
 * caller-owned; it holds the checkpoints until the backward call. */
r3d_status r3d_filter_forward(r3d_ctx *ctx, const r3d_frames *frames, int32_t ckpt_every,
                              const r3d_state *init, float *mean, float *var,
                              void *workspace, size_t workspace_bytes, void *stream);

/* Backward pass, after r3d_filter_forward with the same context, frames,
 * ckpt_every and workspace. grad_mean: device float[nframes*P] = dJ/dmean;
 * grad_var: the same for var, or NULL (zero). grad: device double[11 + W],
 * overwritten with dJ/dbeta, dJ/dsigma_rw2, dJ/dnu[0..8], dJ/dirf[0..W-1]
 * (the tap gradient is 0 for a zero tap; at a zero weight nu_k the nu_k
 * entry is the one-sided derivative, the component's unweighted density
 * over the prior summed against the posterior adjoint). */
r3d_status r3d_filter_backward(r3d_ctx *ctx, const r3d_frames *frames, int32_t ckpt_every,
                               const float *grad_mean, const float *grad_var,
                               void *workspace, size_t workspace_bytes, double *grad,
                               void *stream);

/* Static description of a status code. */
const char *r3d_status_string(r3d_status status);

#ifdef __cplusplus
}
#endif

#endif /* R3D_H */
