"""FP64 CPU oracle of the R3DSP per-frame hot path (Algorithm 1).

TEST INFRASTRUCTURE ONLY: imported by tests, by the entry point's smoke check
and by the benchmark's CPU-baseline leg; never by the product path. It shares
no code, tables or constants with the HIP library.

Everything is evaluated literally in float64 with numpy, vectorised over
pixels only. Conventions (readings of the paper where it is silent):

* all quantities are in bin units: a ToA y and a depth d live on the integer
  bin grid (Sec. II-D takes T = N_T, one bin per time unit);
* the IRF is a pmf ``irf[0..W-1]`` whose maximum is at tap ``c``; a surface at
  depth d gives bin t probability irf[t - d + c] (Sec. II-D: the depth is the
  position of the IRF maximum);
* the depth grid is d = d_lo, ..., d_lo + D - 1 and the correlation is
  zero-padded outside [0, T) (not circular);
* pixel p = row * cols + col; the 3x3 neighbourhood uses weights
  ``nu[(dr+1)*3 + (dc+1)]`` (a 4-neighbour cross has zero corners).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
from scipy.special import ndtr

#: clamp applied to detection probabilities before the logit in the
#: prior-presence update (its logit is undefined at 0 and 1)
LOGIT_CLAMP = 1e-6


# ---------------------------------------------------------------------------
# model
# ---------------------------------------------------------------------------
@dataclass
class Model:
    rows: int
    cols: int
    T: int
    d_lo: int
    D: int
    d_min: float
    d_max: float
    beta: float
    irf: np.ndarray
    c: int
    nu: np.ndarray
    sigma_rw2: float

    @classmethod
    def from_params(cls, p: dict) -> "Model":
        return cls(rows=int(p["rows"]), cols=int(p["cols"]), T=int(p["T"]),
                   d_lo=int(p["d_lo"]), D=int(p["D"]), d_min=float(p["d_min"]),
                   d_max=float(p["d_max"]), beta=float(p["beta"]),
                   irf=np.asarray(p["irf"], dtype=np.float64).copy(),
                   c=int(p["c"]), nu=np.asarray(p["nu"], dtype=np.float64).copy(),
                   sigma_rw2=float(p["sigma_rw2"]))

    @property
    def P(self) -> int:
        return self.rows * self.cols

    @property
    def W(self) -> int:
        return int(self.irf.shape[0])

    @property
    def grid(self) -> np.ndarray:
        return self.d_lo + np.arange(self.D, dtype=np.float64)


@dataclass
class State:
    """Filter state after a frame: the Gaussian q = N(m, v) of each pixel
    (Sec. III-A), its presence probability pi and its background level b."""
    m: np.ndarray
    v: np.ndarray
    pi: np.ndarray
    b: np.ndarray

    def copy(self) -> "State":
        return State(self.m.copy(), self.v.copy(), self.pi.copy(), self.b.copy())


def validate(model: Model) -> None:
    """Parameter domain: beta > 0 (Sec. II-B), random-walk variance > 0
    (Sec. III-A), a non-negative IRF with its peak tap inside the taps."""
    if not model.beta > 0:
        raise ValueError("beta must be > 0")
    if not model.sigma_rw2 > 0:
        raise ValueError("sigma_rw2 must be > 0")
    if model.W < 1 or not (0 <= model.c < model.W):
        raise ValueError("need W >= 1 and 0 <= c < W")
    if np.any(model.irf < 0) or not np.all(np.isfinite(model.irf)):
        raise ValueError("irf must be finite and non-negative")
    if model.D < 1 or model.T < 1 or model.rows < 1 or model.cols < 1:
        raise ValueError("empty grid")
    if model.nu.shape != (9,) or np.any(model.nu < 0) or model.nu.sum() <= 0:
        raise ValueError("nu must be 9 non-negative weights, not all zero")
    if not model.d_max > model.d_min:
        raise ValueError("need d_max > d_min")


# ---------------------------------------------------------------------------
# a1: photon-count histogram (Sec. II-A, discrete Poisson model)
# ---------------------------------------------------------------------------
def histogram(row_ptr: np.ndarray, toa: np.ndarray, T: int,
              pixels: Optional[Sequence[int]] = None) -> np.ndarray:
    """z_t = number of photons of the pixel whose ToA falls in bin t."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    toa = np.asarray(toa, dtype=np.int64)
    P = row_ptr.shape[0] - 1
    pix = np.arange(P) if pixels is None else np.asarray(pixels, dtype=np.int64)
    z = np.zeros((pix.shape[0], T), dtype=np.int64)
    for i, p in enumerate(pix):
        y = toa[row_ptr[p]:row_ptr[p + 1]]
        if y.size and (y.min() < 0 or y.max() >= T):
            raise ValueError(f"ToA outside [0, T) in pixel {p}")
        np.add.at(z[i], y, 1)
    return z


# ---------------------------------------------------------------------------
# a2 + a3: beta-divergence cost (Sec. II-B, eq. beta_div2 and the histogram
# form that follows it; Sec. II-C, eq. beta_CE)
# ---------------------------------------------------------------------------
def modified_irf(irf: np.ndarray, beta: float) -> np.ndarray:
    """The IRF raised to the power beta element-wise (Sec. II-B)."""
    return np.asarray(irf, dtype=np.float64) ** beta


def correlation(z: np.ndarray, model: Model) -> np.ndarray:
    """Cross-correlation of the histogram with the modified IRF on the depth
    grid (Sec. II-B: z^T s_d^beta): sum_j irf[j]^beta z[d-c+j], with z = 0
    outside [0, T). Returns [n, D]."""
    h = modified_irf(model.irf, model.beta)
    z = np.asarray(z, dtype=np.float64)
    d = model.d_lo + np.arange(model.D)
    corr = np.zeros((z.shape[0], model.D))
    for j in range(model.W):
        t = d - model.c + j
        ok = (t >= 0) & (t < model.T)
        corr[:, ok] += h[j] * z[:, t[ok]]
    return corr


def cost_from_histogram(z: np.ndarray, model: Model) -> np.ndarray:
    """Log pseudo-likelihood on the depth grid, histogram form:
    ell(d) = -K * CE_beta(d) = (beta+1)/beta * sum_j irf[j]^beta z[d-c+j]
    (eq. beta_CE; the correlation above times (beta+1)/beta). Returns [n, D]."""
    scale = (model.beta + 1.0) / model.beta
    return scale * correlation(z, model)


def cost_from_histogram_pirf(z: np.ndarray, model: Model, irf_pix: np.ndarray,
                             c_pix: Optional[np.ndarray] = None) -> np.ndarray:
    """The same cost with a pixel-dependent IRF (Sec. II-A: the method also
    applies when the shape of the IRF depends on the pixel): row i of
    ``irf_pix`` ([n, W]) and tap ``c_pix[i]`` (default the model's c) are the
    IRF of the pixel of row i of ``z``; ell_i(d) = (beta+1)/beta *
    sum_j irf_pix[i, j]^beta z_i[d - c_i + j]. Returns [n, D]."""
    z = np.asarray(z, dtype=np.float64)
    irf_pix = np.asarray(irf_pix, dtype=np.float64)
    n, W = irf_pix.shape
    if z.shape[0] != n:
        raise ValueError("one IRF per histogram row")
    c_pix = np.full(n, model.c) if c_pix is None else np.asarray(c_pix, dtype=np.int64)
    h = irf_pix ** model.beta
    scale = (model.beta + 1.0) / model.beta
    d = model.d_lo + np.arange(model.D)
    ell = np.zeros((n, model.D))
    for i in range(n):
        for j in range(W):
            t = d - c_pix[i] + j
            ok = (t >= 0) & (t < model.T)
            ell[i, ok] += h[i, j] * z[i, t[ok]]
    return scale * ell


def cost_from_photons(row_ptr, toa, model: Model,
                      pixels: Optional[Sequence[int]] = None) -> np.ndarray:
    """Same cost, photon form (eq. beta_div2 as printed): the sum over the
    pixel's photons k of f0(y_k | d)^beta = irf[y_k - d + c]^beta."""
    h = modified_irf(model.irf, model.beta)
    scale = (model.beta + 1.0) / model.beta
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    toa = np.asarray(toa, dtype=np.int64)
    P = row_ptr.shape[0] - 1
    pix = np.arange(P) if pixels is None else np.asarray(pixels, dtype=np.int64)
    d = model.d_lo + np.arange(model.D)
    ell = np.zeros((pix.shape[0], model.D))
    for i, p in enumerate(pix):
        for y in toa[row_ptr[p]:row_ptr[p + 1]]:
            j = y - d + model.c
            ok = (j >= 0) & (j < model.W)
            ell[i, ok] += h[j[ok]]
    return scale * ell


# ---------------------------------------------------------------------------
# a4: spatio-temporal prior (Sec. III-A, eq. predict, flat components,
# mixture weights)
# ---------------------------------------------------------------------------
def flat_component(model: Model):
    """Gaussian standing in for the uniform law on (d_min, d_max): mean
    (d_min+d_max)/2, variance (d_max-d_min)^2/12 (Sec. III-A)."""
    return 0.5 * (model.d_min + model.d_max), (model.d_max - model.d_min) ** 2 / 12.0


def prior_components(model: Model, state: State, pixels: np.ndarray):
    """Mixture components of the prior of each pixel in ``pixels``.

    For each of the 9 stencil positions (weight nu_k, zero weight = absent):
    a neighbour inside the frame whose previous presence probability exceeds
    0.5 contributes its Gaussian q = N(m, v); an undetected or out-of-frame
    neighbour contributes the flat Gaussian. The random walk then adds
    sigma_rw2 to every variance (the convolution in eq. predict).
    Returns log-weights log(nu_k) - log(2 pi V)/2, means and variances, [n, 9].
    """
    pixels = np.asarray(pixels, dtype=np.int64)
    r, col = np.divmod(pixels, model.cols)
    m_f, v_f = flat_component(model)
    n = pixels.shape[0]
    logw = np.full((n, 9), -np.inf)
    mean = np.zeros((n, 9))
    var = np.ones((n, 9))
    for k in range(9):
        dr, dc = k // 3 - 1, k % 3 - 1
        rr, cc = r + dr, col + dc
        inside = (rr >= 0) & (rr < model.rows) & (cc >= 0) & (cc < model.cols)
        q = np.where(inside, rr * model.cols + cc, 0)
        if np.any(inside & ~np.isfinite(state.pi[q])):
            raise ValueError("neighbour state needed but not available")
        det = inside & (state.pi[q] > 0.5)
        if np.any(det & ~(np.isfinite(state.m[q]) & np.isfinite(state.v[q]))):
            raise ValueError("neighbour state needed but not available")
        mk = np.where(det, state.m[q], m_f)
        vk = np.where(det, state.v[q], v_f) + model.sigma_rw2
        mean[:, k] = mk
        var[:, k] = vk
        if model.nu[k] > 0:
            logw[:, k] = math.log(model.nu[k]) - 0.5 * np.log(2.0 * math.pi * vk)
    return logw, mean, var


def log_prior(logw: np.ndarray, mean: np.ndarray, var: np.ndarray,
              grid: np.ndarray) -> np.ndarray:
    """log f(d) = log sum_k exp(logw_k - (d - m_k)^2 / (2 V_k)), [n, D]."""
    a = logw[:, :, None] - (grid[None, None, :] - mean[:, :, None]) ** 2 / (2.0 * var[:, :, None])
    amax = np.max(a, axis=1)
    return amax + np.log(np.sum(np.exp(a - amax[:, None, :]), axis=1))


# ---------------------------------------------------------------------------
# a5: pseudo-posterior and its moments (Sec. II-C, eq. approx_post, moments
# by integration over the discretised domain; Sec. III-A, eq. KL_div)
# ---------------------------------------------------------------------------
def posterior_moments(ell: np.ndarray, logf: np.ndarray, grid: np.ndarray) -> dict:
    """Pseudo-posterior on the grid, p(d) proportional to f(d) exp(ell(d)).
    Returns the first maximiser d*, the mean and (population) variance,
    computed centred on d*, and the log-margin of d* over the runner-up."""
    L = logf + ell
    n = L.shape[0]
    rows = np.arange(n)
    i_star = np.argmax(L, axis=1)
    L_star = L[rows, i_star]
    w = np.exp(L - L_star[:, None])
    Z = w.sum(axis=1)
    d_star = grid[i_star]
    dd = grid[None, :] - d_star[:, None]
    mean = d_star + (dd * w).sum(axis=1) / Z
    var = (dd * dd * w).sum(axis=1) / Z - (mean - d_star) ** 2
    if L.shape[1] > 1:
        L2 = L.copy()
        L2[rows, i_star] = -np.inf
        margin = L_star - L2.max(axis=1)
    else:
        margin = np.full(n, np.inf)
    return dict(index=i_star, d_star=d_star, mean=mean, var=var, margin=margin,
                L_star=L_star)


# ---------------------------------------------------------------------------
# a7: background and reflectivity (Sec. II-E, eq. lik_bg_poisson)
# ---------------------------------------------------------------------------
def background_intensity(z: np.ndarray, model: Model, d_star: np.ndarray,
                         detected: np.ndarray, irf_pix: Optional[np.ndarray] = None,
                         c_pix: Optional[np.ndarray] = None):
    """Undetected pixel: b = K / T and r = 0. Detected pixel: maximum
    likelihood (r, b) of z_t ~ Poisson(r s_t + b), s_t = irf[t - d* + c]
    (zero outside the taps), r, b >= 0, with d* the integer depth given (the
    filter passes its depth estimate, the posterior mean, rounded to the
    nearest bin).

    Setting both score equations to zero gives K = r S + b T (S = sum s_t),
    so the optimum lies on b(r) = (K - r S) / T, r in [0, K/S]. The
    log-likelihood restricted to that segment is concave; its derivative
    phi'(r) = sum_t z_t (s_t - S/T) / (r s_t + b(r)) is decreasing and is
    bisected to float64 resolution. r = 0 when phi'(0) <= 0. With
    ``irf_pix`` ([n, W]) and ``c_pix`` the IRF of each row's pixel is its own
    (Sec. II-A, pixel-dependent IRF)."""
    z = np.asarray(z, dtype=np.float64)
    n, T = z.shape
    K = z.sum(axis=1)
    r_hat = np.zeros(n)
    b_hat = K / T
    t = np.arange(T)
    for i in np.nonzero(np.asarray(detected) & (K > 0))[0]:
        irf_i = model.irf if irf_pix is None else np.asarray(irf_pix[i], dtype=np.float64)
        c_i = model.c if c_pix is None else int(c_pix[i])
        tap = t - int(d_star[i]) + c_i
        inwin = (tap >= 0) & (tap < irf_i.shape[0])
        s = np.zeros(T)
        s[inwin] = irf_i[tap[inwin]]
        S = s.sum()
        if S <= 0:
            continue
        nzb = np.nonzero(z[i])[0]
        cnt, s_nz = z[i, nzb], s[nzb]

        def dphi(rr):
            bb = (K[i] - rr * S) / T
            lam = rr * s_nz + bb
            with np.errstate(divide="ignore", invalid="ignore"):
                terms = cnt * (s_nz - S / T) / lam
            terms = np.where(lam > 0, terms, -np.inf)
            return terms.sum()

        hi = K[i] / S
        if dphi(0.0) <= 0:
            continue
        if dphi(hi) >= 0:
            r_hat[i], b_hat[i] = hi, 0.0
            continue
        lo = 0.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:
                break
            if dphi(mid) > 0:
                lo = mid
            else:
                hi = mid
        r_hat[i] = 0.5 * (lo + hi)
        b_hat[i] = (K[i] - r_hat[i] * S) / T
    return r_hat, b_hat


# ---------------------------------------------------------------------------
# prior presence probability for the next frame (Sec. III-B, eq. prior_detect)
# ---------------------------------------------------------------------------
def pi0_next(model: Model, pi_now: np.ndarray, pixels: np.ndarray) -> np.ndarray:
    """pi0 = sigmoid(sum_k nu_k logit(pi_k)) over the stencil; pi is clamped
    to [1e-6, 1 - 1e-6] and an out-of-frame neighbour counts as pi = 0.5."""
    pixels = np.asarray(pixels, dtype=np.int64)
    r, col = np.divmod(pixels, model.cols)
    acc = np.zeros(pixels.shape[0])
    for k in range(9):
        if model.nu[k] == 0:
            continue
        dr, dc = k // 3 - 1, k % 3 - 1
        rr, cc = r + dr, col + dc
        inside = (rr >= 0) & (rr < model.rows) & (cc >= 0) & (cc < model.cols)
        q = np.where(inside, rr * model.cols + cc, 0)
        pk = np.where(inside, np.clip(pi_now[q], LOGIT_CLAMP, 1 - LOGIT_CLAMP), 0.5)
        acc += model.nu[k] * np.log(pk / (1.0 - pk))
    return 1.0 / (1.0 + np.exp(-acc))


# ---------------------------------------------------------------------------
# Algorithm 1: one frame, and a run over frames
# ---------------------------------------------------------------------------
def init_state(model: Model) -> State:
    """Initial state (left open by the paper): every pixel flat and
    undetected (pi = 0.5), background 0."""
    m_f, v_f = flat_component(model)
    P = model.P
    return State(np.full(P, m_f), np.full(P, v_f), np.full(P, 0.5), np.zeros(P))


def step(model: Model, state: State, z: np.ndarray, pixels=None,
         pi_in: Optional[np.ndarray] = None,
         faulty: Optional[np.ndarray] = None,
         irf_pix: Optional[np.ndarray] = None,
         c_pix: Optional[np.ndarray] = None):
    """One frame of Algorithm 1 for the pixels in ``pixels`` (default all).

    ``z`` holds the histograms of exactly those pixels ([n, T]). ``pi_in``
    (length P, default all ones) is the presence probability of the current
    frame supplied by the detector; ``faulty`` (length P bool) marks pixels
    without observations: their pseudo-posterior is the prior and their
    presence probability 0.5 (Sec. III-B, last paragraph). ``irf_pix``
    ([P, W], with ``c_pix`` [P] or the model's c) gives every pixel an IRF of
    its own (Sec. II-A): the cost and the background / reflectivity estimate
    then use the pixel's IRF. Returns the new state (NaN outside ``pixels``)
    and a dict of per-pixel outputs.
    """
    validate(model)
    P = model.P
    pixels = np.arange(P) if pixels is None else np.asarray(pixels, dtype=np.int64)
    z = np.asarray(z)
    if z.shape != (pixels.shape[0], model.T):
        raise ValueError("z must be [len(pixels), T]")
    fault_full = np.zeros(P, bool) if faulty is None else np.asarray(faulty, bool)
    pi_full = np.ones(P) if pi_in is None else np.asarray(pi_in, np.float64)
    pi_now = np.where(fault_full, 0.5, pi_full)
    fault = fault_full[pixels]
    grid = model.grid

    logw, mean, var = prior_components(model, state, pixels)
    logf = log_prior(logw, mean, var, grid)
    if irf_pix is None:
        ell = cost_from_histogram(z, model)
        irf_sel = c_sel = None
    else:
        irf_sel = np.asarray(irf_pix, dtype=np.float64)[pixels]
        c_sel = None if c_pix is None else np.asarray(c_pix, dtype=np.int64)[pixels]
        ell = cost_from_histogram_pirf(z, model, irf_sel, c_sel)
    ell[fault] = 0.0
    post = posterior_moments(ell, logf, grid)
    detected = pi_now[pixels] > 0.5
    zz = np.where(fault[:, None], 0, z)
    # the depth point estimate is the pseudo-posterior mean (Sec. II-E); the
    # tabulated IRF is placed at its nearest bin (ties to even)
    d_mle = np.rint(post["mean"])
    r_hat, b_hat = background_intensity(zz, model, d_mle, detected, irf_sel, c_sel)
    b_hat = np.where(fault, state.b[pixels], b_hat)

    new = State(np.full(P, np.nan), np.full(P, np.nan), np.full(P, np.nan),
                np.full(P, np.nan))
    new.m[pixels] = post["mean"]
    new.v[pixels] = post["var"]
    new.pi[pixels] = pi_now[pixels]
    new.b[pixels] = b_hat
    out = dict(pixels=pixels, mean=post["mean"], var=post["var"],
               depth=np.where(detected, post["mean"], np.nan),
               argmax=post["d_star"].astype(np.int64), margin=post["margin"],
               d_mle=d_mle.astype(np.int64),
               intensity=r_hat, background=b_hat,
               pi0_next=pi0_next(model, pi_now, pixels))
    return new, out


def run(model: Model, frames, state: Optional[State] = None, pi_in=None,
        faulty=None):
    """Run Algorithm 1 over ``frames``: each item is a [P, T] histogram or a
    (row_ptr, toa) photon list. ``pi_in`` is None or one length-P array per
    frame. Returns (final state, list of per-frame output dicts)."""
    st = init_state(model) if state is None else state.copy()
    outs = []
    for n, fr in enumerate(frames):
        if isinstance(fr, tuple):
            z = histogram(fr[0], fr[1], model.T)
        else:
            z = np.asarray(fr)
        pin = None if pi_in is None else pi_in[n]
        st, o = step(model, st, z, pi_in=pin, faulty=faulty)
        outs.append(o)
    return st, outs


# ---------------------------------------------------------------------------
# minimum-divergence (pseudo-ML) estimates: the cost alone, no prior
# (Sec. II-B, last paragraph; Appendix, eq. div_MSL)
# ---------------------------------------------------------------------------
def argmax_with_margin(J: np.ndarray) -> dict:
    """First maximiser of each row of J, its value and its margin over the
    best other grid point (inf for a single point)."""
    J = np.asarray(J, dtype=np.float64)
    n = J.shape[0]
    rows = np.arange(n)
    i = np.argmax(J, axis=1)
    v = J[rows, i]
    if J.shape[1] > 1:
        J2 = J.copy()
        J2[rows, i] = -np.inf
        margin = v - J2.max(axis=1)
    else:
        margin = np.full(n, np.inf)
    return dict(index=i, value=v, margin=margin)


def min_divergence(z: np.ndarray, model: Model) -> dict:
    """Minimum beta-divergence depth estimate of each pixel: minimising
    eq. beta_div2 over the depth grid, i.e. maximising the histogram
    cross-correlation ell(d) of Sec. II-B with no prior. Returns the first
    maximiser (grid index and depth), ell there (natural log units, as
    cost_from_histogram) and its margin over the runner-up."""
    r = argmax_with_margin(cost_from_histogram(z, model))
    r["d_hat"] = model.d_lo + r["index"]
    return r


def msl_objective(z_bands, models) -> np.ndarray:
    """Multispectral beta-divergence (Appendix, eq. div_MSL): the divergence
    is Const - (beta+1)/beta * prod_l (1/K_l) sum_k f_l(y_lk | d)^beta, so its
    minimiser maximises prod_l c_l(d) / K_l with c_l the band's histogram
    correlation with irf_l^beta. Returns sum_l [log c_l(d) - log K_l], [n, D]
    (-inf where some band's correlation vanishes). The bands share T, the
    depth grid and beta; each has its own IRF and peak tap. A band without
    photons (K_l = 0) has no empirical distribution and is left out."""
    if len(z_bands) != len(models) or not models:
        raise ValueError("one model per band")
    m0 = models[0]
    for m in models:
        if (m.T, m.d_lo, m.D, m.beta) != (m0.T, m0.d_lo, m0.D, m0.beta):
            raise ValueError("bands must share T, the depth grid and beta")
    n = np.asarray(z_bands[0]).shape[0]
    J = np.zeros((n, m0.D))
    for zb, m in zip(z_bands, models):
        zb = np.asarray(zb, dtype=np.float64)
        K = zb.sum(axis=1)
        corr = correlation(zb, m)
        with np.errstate(divide="ignore"):
            term = np.log(corr) - np.log(np.where(K > 0, K, 1.0))[:, None]
        J += np.where((K > 0)[:, None], term, 0.0)
    return J


def msl_min_divergence(z_bands, models) -> dict:
    """Minimum multispectral beta-divergence depth of each pixel (Appendix,
    eq. div_MSL; the estimator compared there). First maximiser of
    msl_objective, its value and margin."""
    r = argmax_with_margin(msl_objective(z_bands, models))
    r["d_hat"] = models[0].d_lo + r["index"]
    return r


# ---------------------------------------------------------------------------
# continuous ToAs, Gaussian IRF: the minimum-divergence depth off the grid
# (Sec. II-B, eq. beta_div2 with the photon sum; Sec. V: the correlation may
# be continuous, and a Gaussian IRF simplifies the update rules)
# ---------------------------------------------------------------------------
def gauss_cost(y: np.ndarray, d, sigma: float, beta: float) -> np.ndarray:
    """(beta+1)/beta * sum_k f0(y_k | d)^beta for a Gaussian IRF of standard
    deviation sigma (unit integral) and continuous depth(s) d: the photon sum
    of eq. beta_div2 without the constant. With f0(y|d) = N(y; d, sigma^2),
    f0^beta = (2 pi sigma^2)^(-beta/2) exp(-beta (y - d)^2 / (2 sigma^2))."""
    y = np.asarray(y, dtype=np.float64)
    d = np.atleast_1d(np.asarray(d, dtype=np.float64))
    amp = (2.0 * math.pi * sigma * sigma) ** (-beta / 2.0)
    e = y[None, :] - d[:, None]
    return (beta + 1.0) / beta * amp * np.exp(-beta * e * e / (2.0 * sigma * sigma)).sum(axis=1)


def gauss_min_divergence(row_ptr, toa, sigma: float, beta: float, d_lo: int, D: int,
                         tol: float = 1e-12, max_iter: int = 10000) -> dict:
    """Minimum beta-divergence depth of each pixel for a Gaussian IRF,
    maximised over continuous d. The photon ToAs are the bin indices (the
    depth convention of the grid). The objective sum_k exp(-(y_k - d)^2 /
    (2 h^2)), h^2 = sigma^2 / beta, is stationary where
    d = sum_k w_k y_k / sum_k w_k, w_k = exp(-(y_k - d)^2 / (2 h^2)); this
    fixed point, iterated from the first maximiser on the depth grid
    (photon form, every photon), climbs to the local maximum of that
    maximiser's basin, held to the grid's span [d_lo, d_lo + D - 1] (the
    admissible depths). Returns the continuous depth, the cost there (natural
    log units, gauss_cost), the grid maximiser and the grid margin (best grid
    value minus the best value two or more bins away). A pixel without
    photons keeps d_lo with cost 0."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    P = len(row_ptr) - 1
    grid = d_lo + np.arange(D, dtype=np.float64)
    depth = np.full(P, float(d_lo))
    value = np.zeros(P)
    gidx = np.zeros(P, dtype=np.int64)
    margin = np.full(P, np.inf)
    h2 = sigma * sigma / beta
    for p in range(P):
        y = np.asarray(toa[row_ptr[p]:row_ptr[p + 1]], dtype=np.float64)
        if y.size == 0:
            continue
        J = gauss_cost(y, grid, sigma, beta)
        i = int(np.argmax(J))
        gidx[p] = i
        far = np.abs(np.arange(D) - i) >= 2
        if far.any():
            margin[p] = J[i] - J[far].max()
        d = grid[i]
        for _ in range(max_iter):
            w = np.exp(-(y - d) ** 2 / (2.0 * h2))
            dn = float(np.dot(w, y) / w.sum())
            if abs(dn - d) <= tol * max(1.0, abs(d)):
                d = dn
                break
            d = dn
        # the admissible depths are the grid's span: a basin whose peak lies
        # beyond it rises to the nearer end of the span
        depth[p] = d = min(max(d, grid[0]), grid[-1])
        value[p] = gauss_cost(y, d, sigma, beta)[0]
    return dict(depth=depth, value=value, grid_index=gidx, margin=margin)


# ---------------------------------------------------------------------------
# differentiable filter: loss and its finite-difference gradient
# ---------------------------------------------------------------------------
def gaussian_irf_sigma(sigma: float, W: int, c: int) -> np.ndarray:
    """Bin-integrated Gaussian IRF with standard deviation sigma, peak at
    tap c, renormalised over the W taps (Sec. II-A integral; Sec. II-D unit
    integral)."""
    j = np.arange(W, dtype=np.float64)
    pmf = ndtr((j - c + 0.5) / sigma) - ndtr((j - c - 0.5) / sigma)
    return pmf / pmf.sum()


def filter_loss(theta: np.ndarray, model: Model, frames, d_true: np.ndarray,
                pi_in=None, faulty=None) -> float:
    """Mean over pixels and frames of (posterior mean - true depth)^2 for the
    filter run with theta = (beta, irf sigma, sigma_rw2, nu[0..8]). The
    posterior mean is the soft-argmax of the log pseudo-posterior at
    temperature one bin. ``pi_in`` and ``faulty`` are passed to ``run``
    unchanged (inputs, not parameters)."""
    theta = np.asarray(theta, dtype=np.float64)
    mdl = Model(rows=model.rows, cols=model.cols, T=model.T, d_lo=model.d_lo,
                D=model.D, d_min=model.d_min, d_max=model.d_max,
                beta=float(theta[0]),
                irf=gaussian_irf_sigma(float(theta[1]), model.W, model.c),
                c=model.c, nu=theta[3:12].copy(), sigma_rw2=float(theta[2]))
    _, outs = run(mdl, frames, pi_in=pi_in, faulty=faulty)
    err = [(o["mean"] - np.asarray(d_true[n], np.float64)) ** 2 for n, o in enumerate(outs)]
    return float(np.mean(np.stack(err)))


def filter_loss_grad_fd(theta: np.ndarray, model: Model, frames, d_true,
                        rel_step: float = 1e-6, pi_in=None, faulty=None) -> np.ndarray:
    """Central finite differences of ``filter_loss`` with a relative step."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros_like(theta)
    for i in range(theta.shape[0]):
        h = rel_step * max(abs(theta[i]), 1e-2)
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        g[i] = (filter_loss(tp, model, frames, d_true, pi_in, faulty)
                - filter_loss(tm, model, frames, d_true, pi_in, faulty)) / (2 * h)
    return g
