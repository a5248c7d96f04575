"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine with a different algorithm, a closed form, an invariance, a limit, or
a hand-derived worked example stored under tests/golden/. Together they are
chosen so that a dropped term, a wrong sign or index, or a transposed
operand anywhere in the oracle fails at least one of them.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate, optimize, stats

import oracle
from oracle import Model, State

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def make_model(rows=5, cols=5, T=64, W=9, c=4, beta=0.4, sigma=1.7, nu=None,
               sigma_rw2=3.0, d_lo=0, D=None, d_min=None, d_max=None, irf=None):
    if irf is None:
        irf = oracle.gaussian_irf_sigma(sigma, W, c)
    D = T if D is None else D
    return Model(rows=rows, cols=cols, T=T, d_lo=d_lo, D=D,
                 d_min=float(d_lo if d_min is None else d_min),
                 d_max=float(d_lo + D - 1 if d_max is None else d_max),
                 beta=beta, irf=np.asarray(irf, float), c=c,
                 nu=np.array([1 / 16] * 4 + [0.5] + [1 / 16] * 4) if nu is None else np.asarray(nu, float),
                 sigma_rw2=sigma_rw2)


def random_photons(rng, P, T, lam=8):
    counts = rng.poisson(lam, P)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    toa = rng.integers(0, T, row_ptr[-1])
    return row_ptr, toa


def detected_state(model, m, v, pi=1.0):
    P = model.P
    return State(np.full(P, float(m)), np.full(P, float(v)), np.full(P, float(pi)), np.zeros(P))


# ---------------------------------------------------------------- histogram
def test_histogram_matches_bincount():
    rng = np.random.default_rng(1)
    row_ptr, toa = random_photons(rng, 30, 50)
    z = oracle.histogram(row_ptr, toa, 50)
    for p in range(30):
        y = toa[row_ptr[p]:row_ptr[p + 1]]
        np.testing.assert_array_equal(z[p], np.bincount(y, minlength=50))
        assert z[p].sum() == row_ptr[p + 1] - row_ptr[p]


def test_histogram_rejects_out_of_range_toa():
    with pytest.raises(ValueError):
        oracle.histogram(np.array([0, 2]), np.array([3, 50]), 50)
    with pytest.raises(ValueError):
        oracle.histogram(np.array([0, 1]), np.array([-1]), 50)


# ---------------------------------------------------------------- cost (a3)
def test_cost_photon_form_equals_histogram_form():
    """Two different formulas of Sec. II-B (sum over photons of f0^beta, and
    z^T s_d^beta) must agree; catches a sign or offset error in either."""
    rng = np.random.default_rng(2)
    m = make_model(T=80, W=11, c=3, beta=0.37, sigma=2.2, D=70, d_lo=5)
    row_ptr, toa = random_photons(rng, 12, 80, lam=10)
    a = oracle.cost_from_photons(row_ptr, toa, m)
    b = oracle.cost_from_histogram(oracle.histogram(row_ptr, toa, 80), m)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_cost_beta_one_is_matched_filter():
    """beta = 1: the cost is 2x the matched-filter correlation of z with the
    IRF (Sec. II-B); compared with numpy's full convolution."""
    rng = np.random.default_rng(3)
    m = make_model(T=60, W=7, c=2, beta=1.0, sigma=1.3)
    row_ptr, toa = random_photons(rng, 6, 60)
    z = oracle.histogram(row_ptr, toa, 60)
    ell = oracle.cost_from_histogram(z, m)
    for p in range(6):
        conv = np.convolve(z[p].astype(float), m.irf[::-1])
        d = np.arange(60)
        np.testing.assert_allclose(ell[p], 2.0 * conv[d - m.c + m.W - 1], rtol=1e-13, atol=1e-13)


def test_beta_to_zero_recovers_log_likelihood():
    """As beta -> 0 the beta-divergence tends to KL (Sec. II-B): cost
    differences tend to log-likelihood differences, with error O(beta)."""
    irf = np.array([0.05, 0.15, 0.3, 0.25, 0.15, 0.1])
    T, c = 40, 2
    toa = np.array([17, 18, 18, 19, 20, 21])
    row_ptr = np.array([0, len(toa)])
    d1, d2 = 18, 19  # windows of both cover every photon
    ll = lambda d: np.sum(np.log(irf[toa - d + c]))
    target = ll(d1) - ll(d2)
    errs = []
    for beta in (1e-3, 1e-4, 1e-6):
        m = make_model(rows=1, cols=1, T=T, W=6, c=c, beta=beta, irf=irf)
        ell = oracle.cost_from_photons(row_ptr, toa, m)[0]
        errs.append(abs((ell[d1] - ell[d2]) - target))
    assert errs[2] < 1e-5 * abs(target) + 1e-7
    assert errs[0] / errs[1] == pytest.approx(10.0, rel=0.05)  # linear in beta


def test_golden_worked_pixel():
    """Hand-derived cost values and posterior of a 1x1, T = 6 frame."""
    g = json.load(open(os.path.join(GOLDEN, "worked_tiny_pixel.json")))
    mpmath.mp.dps = 40
    ns = {"sqrt": mpmath.sqrt}
    for case in g["cases"]:
        m = make_model(rows=1, cols=1, T=g["T"], W=3, c=g["c"], beta=case["beta"],
                       irf=g["irf"], d_lo=g["d_lo"], D=g["D"], d_min=g["d_min"],
                       d_max=g["d_max"],
                       sigma_rw2=float(eval(g["sigma_rw2_expr"], {}, {})))
        z = oracle.histogram(np.array([0, len(g["toa"])]), np.array(g["toa"]), g["T"])
        np.testing.assert_array_equal(z[0], g["histogram"])
        ell_exp = [mpmath.mpf(eval(e, ns, {})) if e not in ("0",) else mpmath.mpf(0)
                   for e in case["ell_expr"]]
        ell = oracle.cost_from_histogram(z, m)[0]
        np.testing.assert_allclose(ell, [float(x) for x in ell_exp], rtol=1e-14, atol=1e-14)
        st, out = oracle.step(m, oracle.init_state(m), z)
        L = [ell_exp[d] + eval(g["log_prior_expr"], {}, {"d": mpmath.mpf(d)}) for d in range(g["D"])]
        Lmax = max(L)
        w = [mpmath.e ** (x - Lmax) for x in L]
        Z = sum(w)
        mean = sum(d * w[d] for d in range(g["D"])) / Z
        var = sum((d - mean) ** 2 * w[d] for d in range(g["D"])) / Z
        assert out["argmax"][0] == case["argmax"]
        assert out["mean"][0] == pytest.approx(float(mean), abs=1e-12)
        assert out["var"][0] == pytest.approx(float(var), abs=1e-12)


# --------------------------------------------------------------- prior (a4)
def test_identical_neighbours_no_photons_gives_random_walk_gaussian():
    """Zero photons and nine identical detected neighbours: the pseudo-
    posterior is the prior N(m, v + sigma_rw2) (eq. predict), whose discrete
    moments on the integer grid equal the continuous ones up to
    exp(-2 pi^2 V) (Poisson summation)."""
    m = make_model(rows=3, cols=3, T=400, sigma_rw2=2.5)
    st = detected_state(m, 201.37, 4.2)
    z = np.zeros((1, m.T), np.int64)
    _, out = oracle.step(m, st, z, pixels=[4])
    assert out["mean"][0] == pytest.approx(201.37, abs=1e-10)
    assert out["var"][0] == pytest.approx(4.2 + 2.5, abs=1e-10)


def test_mixture_moments_include_component_normalisation():
    """Distinct detected neighbours, zero photons: the prior is the mixture
    sum_k nu_k N(m_k, v_k + s2) / sum nu (each component a normalised
    density), so its moments are the mixture moments. Dropping the
    -log(2 pi V)/2 term or the random-walk variance fails this."""
    rng = np.random.default_rng(5)
    m = make_model(rows=3, cols=3, T=600, sigma_rw2=1.5,
                   nu=rng.uniform(0.2, 1.0, 9))
    st = State(rng.uniform(250, 350, 9), rng.uniform(1.0, 40.0, 9), np.ones(9), np.zeros(9))
    _, out = oracle.step(m, st, np.zeros((1, m.T), np.int64), pixels=[4])
    wts = m.nu / m.nu.sum()
    V = st.v + m.sigma_rw2
    mu = np.sum(wts * st.m)
    var = np.sum(wts * (V + st.m ** 2)) - mu ** 2
    assert out["mean"][0] == pytest.approx(mu, abs=1e-9)
    assert out["var"][0] == pytest.approx(var, abs=1e-8)


def test_random_walk_convolution_by_quadrature():
    """eq. predict: integral of the random-walk kernel against N(m, v) equals
    the oracle's component density N(d; m, v + s2), checked by quadrature."""
    m = make_model(rows=1, cols=1, T=100, sigma_rw2=2.0, nu=[0, 0, 0, 0, 1, 0, 0, 0, 0])
    st = detected_state(m, 40.3, 3.1)
    logw, mean, var = oracle.prior_components(m, st, np.array([0]))
    grid = np.array([35.0, 40.0, 41.5, 47.0])
    lf = oracle.log_prior(logw, mean, var, grid)[0]
    for d, l in zip(grid, lf):
        f = lambda x: stats.norm.pdf(d, x, math.sqrt(2.0)) * stats.norm.pdf(x, 40.3, math.sqrt(3.1))
        val, _ = integrate.quad(f, 0, 100, points=[40.3], epsabs=1e-14)
        assert math.exp(l) == pytest.approx(val, rel=1e-9)


def test_flat_prior_symmetric_grid_mean_is_centre():
    """Undetected neighbours, zero photons, grid symmetric about
    (d_min + d_max)/2: the posterior mean is the centre (symmetry)."""
    m = make_model(rows=3, cols=3, T=101)
    st = oracle.init_state(m)
    _, out = oracle.step(m, st, np.zeros((9, m.T), np.int64))
    np.testing.assert_allclose(out["mean"], 50.0, atol=1e-9)


def test_detection_threshold_is_strict():
    """pi = 0.5 counts as undetected (flat component); pi just above 0.5
    uses the neighbour's Gaussian (Algorithm 1's test pi > 0.5)."""
    m = make_model(rows=3, cols=3, T=201)
    z = np.zeros((1, m.T), np.int64)
    _, out_half = oracle.step(m, detected_state(m, 30.0, 2.0, pi=0.5), z, pixels=[4])
    _, out_det = oracle.step(m, detected_state(m, 30.0, 2.0, pi=0.5000001), z, pixels=[4])
    assert out_half["mean"][0] == pytest.approx(100.0, abs=1e-9)
    assert out_det["mean"][0] == pytest.approx(30.0, abs=1e-9)


def test_mixture_weight_scale_invariance_and_cross():
    """Scaling every nu by a constant leaves the posterior unchanged; a
    zero-cornered stencil equals dropping those components."""
    rng = np.random.default_rng(6)
    m1 = make_model(rows=4, cols=4, T=70)
    row_ptr, toa = random_photons(rng, 16, 70)
    z = oracle.histogram(row_ptr, toa, 70)
    st = State(rng.uniform(20, 50, 16), rng.uniform(1, 10, 16), rng.uniform(0.3, 1, 16), np.zeros(16))
    _, a = oracle.step(m1, st, z)
    m2 = make_model(rows=4, cols=4, T=70, nu=3.0 * m1.nu)
    _, b = oracle.step(m2, st, z)
    np.testing.assert_allclose(a["mean"], b["mean"], rtol=1e-12)
    np.testing.assert_allclose(a["var"], b["var"], rtol=1e-10)
    # cross: corners zero == an explicit 5-component evaluation
    nu = np.array([0, .1, 0, .2, .4, .1, 0, .2, 0])
    m3 = make_model(rows=4, cols=4, T=70, nu=nu)
    logw, mean, var = oracle.prior_components(m3, st, np.arange(16))
    assert np.all(np.isneginf(logw[:, [0, 2, 6, 8]]))
    keep = [1, 3, 4, 5, 7]
    lf = oracle.log_prior(logw[:, keep], mean[:, keep], var[:, keep], m3.grid)
    np.testing.assert_allclose(oracle.log_prior(logw, mean, var, m3.grid), lf, rtol=1e-13)


def test_pi0_nonlinear_averaging_invariant():
    """eq. prior_detect: equal pi everywhere and weights summing to one give
    pi0 = pi at interior pixels; out-of-frame neighbours count as 0.5."""
    m = make_model(rows=5, cols=5)
    for x in (0.2, 0.7, 0.95):
        pi = np.full(25, x)
        p0 = oracle.pi0_next(m, pi, np.arange(25))
        assert p0[12] == pytest.approx(x, rel=1e-12)
        inside = m.nu[[4, 5, 7, 8]].sum()  # corner pixel 0 sees these
        assert p0[0] == pytest.approx(1 / (1 + math.exp(-inside * math.log(x / (1 - x)))), rel=1e-12)
    p0 = oracle.pi0_next(m, np.ones(25), np.array([12]))
    assert p0[0] == pytest.approx(1 - 1e-6, rel=1e-9)


# ------------------------------------------------------------ posterior (a5)
def test_shift_equivariance():
    """Shifting every ToA and every state mean by k shifts argmax and mean by
    k and leaves the variance unchanged (away from the grid edges)."""
    rng = np.random.default_rng(7)
    m = make_model(rows=3, cols=4, T=300)
    P = 12
    depth = 120
    toa = np.concatenate([depth - m.c + rng.choice(m.W, 15, p=m.irf) for _ in range(P)])
    toa = np.concatenate([toa, rng.integers(100, 160, 4 * P)])
    pix = np.concatenate([np.repeat(np.arange(P), 15), np.repeat(np.arange(P), 4)])
    order = np.argsort(pix, kind="stable")
    toa, pix = toa[order], pix[order]
    row_ptr = np.concatenate([[0], np.cumsum(np.bincount(pix, minlength=P))])
    st = State(rng.uniform(115, 125, P), rng.uniform(1, 5, P), np.ones(P), np.zeros(P))
    _, a = oracle.step(m, st, oracle.histogram(row_ptr, toa, m.T))
    k = 37
    st2 = State(st.m + k, st.v.copy(), st.pi.copy(), st.b.copy())
    _, b = oracle.step(m, st2, oracle.histogram(row_ptr, toa + k, m.T))
    # only interior pixels: an out-of-frame neighbour brings the flat
    # component, whose mean (d_min + d_max)/2 does not move with the shift
    inner = [5, 6]
    np.testing.assert_array_equal(b["argmax"][inner], a["argmax"][inner] + k)
    np.testing.assert_allclose(b["mean"][inner], a["mean"][inner] + k, atol=1e-9)
    np.testing.assert_allclose(b["var"][inner], a["var"][inner], rtol=1e-8)


def test_noiseless_single_peak():
    """K photons in one bin t0: with a skewed IRF whose maximum is tap c and
    a flat prior the argmax is t0 (the depth is the IRF peak, Sec. II-D);
    with a symmetric IRF and a prior centred at t0 the mean is t0 too."""
    skew = np.array([0.02, 0.1, 0.4, 0.25, 0.13, 0.07, 0.03])  # max at tap 2
    m = make_model(rows=1, cols=1, T=200, W=7, c=2, irf=skew, beta=0.5)
    z = np.zeros((1, 200), np.int64)
    z[0, 77] = 40
    _, out = oracle.step(m, oracle.init_state(m), z)
    assert out["argmax"][0] == 77
    m2 = make_model(rows=3, cols=3, T=200, W=9, c=4, beta=0.5)
    z2 = np.zeros((1, 200), np.int64)
    z2[0, 77] = 25
    _, out2 = oracle.step(m2, detected_state(m2, 77.0, 3.0), z2, pixels=[4])
    assert out2["argmax"][0] == 77
    assert out2["mean"][0] == pytest.approx(77.0, abs=1e-9)


def test_faulty_pixel_posterior_is_prior():
    """A faulty pixel keeps the prior as its pseudo-posterior and pi = 0.5
    (Sec. III-B); its moments equal those of the Gaussian mixture evaluated
    with scipy's normal density."""
    rng = np.random.default_rng(8)
    m = make_model(rows=3, cols=3, T=150, sigma_rw2=2.0)
    st = State(rng.uniform(60, 90, 9), rng.uniform(2, 30, 9), np.ones(9), np.zeros(9))
    faulty = np.zeros(9, bool)
    faulty[4] = True
    z = np.zeros((1, m.T), np.int64)
    z[0, [10, 70, 71, 72]] = 5  # photons that must be ignored
    new, out = oracle.step(m, st, z, pixels=[4], faulty=faulty)
    g = m.grid
    dens = sum(m.nu[k] * stats.norm.pdf(g, st.m[k], math.sqrt(st.v[k] + 2.0)) for k in range(9))
    p = dens / dens.sum()
    mu = (g * p).sum()
    assert out["mean"][0] == pytest.approx(mu, abs=1e-9)
    assert out["var"][0] == pytest.approx(((g - mu) ** 2 * p).sum(), abs=1e-8)
    assert new.pi[4] == 0.5 and math.isnan(out["depth"][0])


def test_undetected_pixel_has_no_depth_and_background_k_over_t():
    m = make_model(rows=2, cols=2, T=50)
    rng = np.random.default_rng(9)
    row_ptr, toa = random_photons(rng, 4, 50)
    z = oracle.histogram(row_ptr, toa, 50)
    pi = np.array([0.2, 0.5, 0.9, 1.0])
    _, out = oracle.step(m, oracle.init_state(m), z, pi_in=pi)
    assert np.isnan(out["depth"][0]) and np.isnan(out["depth"][1])
    assert np.isfinite(out["depth"][2]) and np.isfinite(out["depth"][3])
    np.testing.assert_allclose(out["background"][:2], z[:2].sum(1) / 50)
    np.testing.assert_array_equal(out["intensity"][:2], 0.0)


# ----------------------------------------------------- background / intensity
def test_golden_intensity():
    g = json.load(open(os.path.join(GOLDEN, "worked_intensity.json")))
    ns = {"sqrt": math.sqrt}
    m = make_model(rows=1, cols=1, T=g["T"], W=3, c=g["c"], irf=g["irf"])
    for hist, r_e, b_e in ((g["histogram"], g["r_expr"], g["b_expr"]),
                           (g["boundary_case"]["histogram"], g["boundary_case"]["r_expr"],
                            g["boundary_case"]["b_expr"])):
        r, b = oracle.background_intensity(np.array([hist]), m, np.array([g["d_star"]]),
                                           np.array([True]))
        assert r[0] == pytest.approx(eval(r_e, ns, {}), abs=1e-12)
        assert b[0] == pytest.approx(eval(b_e, ns, {}), abs=1e-12)


def test_intensity_matches_generic_optimiser():
    """Maximum likelihood under eq. lik_bg_poisson, compared with scipy's
    bound-constrained optimiser on the full Poisson likelihood; also the
    identity K = r S + b T at the optimum."""
    rng = np.random.default_rng(10)
    m = make_model(rows=1, cols=1, T=120, W=15, c=7, sigma=2.5)
    for trial in range(6):
        d = int(rng.integers(20, 100))
        s = np.zeros(120)
        s[d - 7:d + 8] = m.irf
        z = rng.poisson(rng.uniform(5, 40) * s + rng.uniform(0.05, 1.0))
        r, b = oracle.background_intensity(z[None], m, np.array([d]), np.array([True]))
        nll = lambda x: -(z * np.log(x[0] * s + x[1])).sum() + (x[0] * s + x[1]).sum()
        res = optimize.minimize(nll, x0=[5.0, 0.5], bounds=[(0, None), (1e-12, None)],
                                method="L-BFGS-B", options=dict(ftol=1e-15, gtol=1e-11, maxiter=10000))
        assert nll([r[0], b[0]]) <= res.fun + 1e-9
        assert r[0] == pytest.approx(res.x[0], rel=1e-4, abs=1e-4)
        assert z.sum() == pytest.approx(r[0] * s.sum() + b[0] * 120, rel=1e-12)


def test_intensity_zero_when_no_excess_in_window():
    m = make_model(rows=1, cols=1, T=100, W=9, c=4)
    z = np.zeros(100, np.int64)
    z[[5, 6, 90, 95]] = 1  # nothing near d* = 50
    r, b = oracle.background_intensity(z[None], m, np.array([50]), np.array([True]))
    assert r[0] == 0.0 and b[0] == pytest.approx(4 / 100)


# ------------------------------------------------------------------ online
def test_resume_from_state_equals_uninterrupted_run():
    rng = np.random.default_rng(11)
    m = make_model(rows=4, cols=3, T=60)
    frames = [random_photons(rng, 12, 60) for _ in range(4)]
    st_full, outs_full = oracle.run(m, frames)
    st_half, _ = oracle.run(m, frames[:2])
    st_rest, outs_rest = oracle.run(m, frames[2:], state=st_half)
    np.testing.assert_array_equal(st_full.m, st_rest.m)
    np.testing.assert_array_equal(st_full.v, st_rest.v)
    np.testing.assert_array_equal(outs_full[3]["mean"], outs_rest[1]["mean"])


def test_light_cone_subset_equals_full_frame():
    """Computing a pixel subset from a state known on its 3x3 halo gives the
    same numbers as the full frame (pixels are independent in a frame)."""
    rng = np.random.default_rng(12)
    m = make_model(rows=6, cols=7, T=50)
    frames = [oracle.histogram(*random_photons(rng, 42, 50), 50) for _ in range(2)]
    st1, _ = oracle.run(m, frames[:1])
    _, full = oracle.step(m, st1, frames[1])
    pix = np.array([0, 9, 20, 41])
    _, sub = oracle.step(m, st1, frames[1][pix], pixels=pix)
    np.testing.assert_array_equal(sub["mean"], full["mean"][pix])


def test_validate_rejects_bad_parameters():
    for kw in (dict(beta=0.0), dict(sigma_rw2=-1.0), dict(c=9)):
        with pytest.raises(ValueError):
            oracle.validate(make_model(**kw))


def test_fd_gradient_of_loss_is_consistent():
    """The finite-difference gradient of the filter loss agrees with a
    one-sided directional difference (a self-check of the FD helper)."""
    import synth
    wl = synth.config5(rows=4, cols=4, frames=2)
    mdl = Model.from_params(wl.params())
    frames = [(f.row_ptr.numpy(), f.toa.numpy()) for f in wl.frames]
    truth = wl.depth_true.numpy()
    theta = np.concatenate([[0.3, 4.0, 3.0], wl.nu])
    g = oracle.filter_loss_grad_fd(theta, mdl, frames, truth)
    u = np.random.default_rng(0).normal(size=theta.shape)
    u /= np.linalg.norm(u)
    eps = 1e-5
    lp = oracle.filter_loss(theta + eps * u, mdl, frames, truth)
    lm = oracle.filter_loss(theta - eps * u, mdl, frames, truth)
    assert (lp - lm) / (2 * eps) == pytest.approx(g @ u, rel=1e-4, abs=1e-8)


def test_gaussian_irf_is_bin_integrated_pulse():
    """Sec. II-A: the discrete IRF is the pulse integrated over each bin; it
    is renormalised over its taps (Sec. II-D's unit integral) and peaks at
    tap c. Checked against quadrature of the normal density."""
    sigma, W, c = 3.7, 31, 15
    irf = oracle.gaussian_irf_sigma(sigma, W, c)
    ref = np.array([integrate.quad(stats.norm(0.0, sigma).pdf, j - c - 0.5, j - c + 0.5,
                                   epsabs=1e-15, epsrel=1e-13)[0] for j in range(W)])
    ref /= ref.sum()
    np.testing.assert_allclose(irf, ref, rtol=1e-10, atol=1e-15)
    assert int(np.argmax(irf)) == c and abs(irf.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(irf[c - 6:c], irf[c + 6:c:-1], rtol=1e-12)


def test_step_places_the_mle_at_the_rounded_mean():
    """Sec. II-E: the depth point estimate of a detected pixel is the
    pseudo-posterior mean and the reflectivity is estimated with it. A pixel
    with two equal returns (bins 20 and 44) has a two-mode posterior whose
    argmax is one return and whose mean lies between them; the step's (r, b)
    equal the Poisson maximum likelihood with the IRF placed at the mean's
    nearest bin, found by scipy's bounded optimiser."""
    m = make_model(rows=1, cols=1, T=64, W=9, c=4, beta=0.4, sigma=1.2)
    z = np.zeros((1, 64), np.int64)
    for d in (20, 44):
        z[0, d - 4:d + 5] += np.round(12 * m.irf).astype(np.int64)
    z[0, ::7] += 1
    st = oracle.init_state(m)
    _, out = oracle.step(m, st, z)
    d_mle = int(out["d_mle"][0])
    assert d_mle == int(np.rint(out["mean"][0])) and d_mle != int(out["argmax"][0])
    t = np.arange(64)
    tap = t - d_mle + m.c
    s = np.where((tap >= 0) & (tap < m.W), m.irf[np.clip(tap, 0, m.W - 1)], 0.0)

    def nll(x):
        lam = x[0] * s + x[1]
        return -(z[0] * np.log(np.maximum(lam, 1e-300)) - lam).sum()

    res = optimize.minimize(nll, x0=[5.0, 0.5], bounds=[(0, None), (1e-12, None)],
                            method="L-BFGS-B", options=dict(ftol=1e-15, gtol=1e-12))
    assert out["intensity"][0] == pytest.approx(res.x[0], rel=1e-4)
    assert out["background"][0] == pytest.approx(res.x[1], rel=1e-4)
