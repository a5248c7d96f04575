"""Pins of the oracle's later parts: the argmax margin, the filter loss, the
minimum-divergence estimators (single band and multispectral) and the
pixel-dependent IRF. As in test_oracle_pins.py, each check is against
something other than the function under test: a hand derivation in mpmath
from a different formula, a library routine, a limit or an invariance.
"""
import mpmath
import numpy as np
import pytest
from scipy import optimize

import oracle
from oracle import Model, State
from test_oracle_pins import make_model, random_photons


# ------------------------------------------------------------- argmax margin
def test_margin_of_hand_built_posterior():
    """posterior_moments reports d* (first maximiser of log f + ell) and the
    log-margin L(d*) - max_{d != d*} L(d) (Sec. II-C, eq. approx_post on the
    grid). Values built by hand, with a prior term that changes the order."""
    grid = np.arange(4, dtype=float)
    ell = np.array([[0.0, 3.0, 1.5, 3.5],     # L = [0, 2, 1.5, 3.5 - 2] -> d* = 1
                    [1.0, 2.0, 2.0, 0.0],     # tie between d = 1 and 2
                    [5.0, 1.0, 1.0, 1.0]])
    logf = np.array([[0.0, -1.0, 0.0, -2.0],
                     [0.0, 0.0, 0.0, 0.0],
                     [-0.25, 0.0, 0.0, 0.0]])
    r = oracle.posterior_moments(ell, logf, grid)
    np.testing.assert_array_equal(r["index"], [1, 1, 0])
    assert r["margin"][0] == pytest.approx(2.0 - 1.5, abs=1e-15)
    assert r["margin"][1] == 0.0
    assert r["margin"][2] == pytest.approx(4.75 - 1.0, abs=1e-15)
    one = oracle.posterior_moments(np.array([[2.0]]), np.array([[0.0]]), np.array([7.0]))
    assert one["margin"][0] == np.inf and one["d_star"][0] == 7.0


def test_argmax_with_margin_by_sorting():
    """Margin = top value minus second value, from a full sort."""
    rng = np.random.default_rng(5)
    J = rng.normal(size=(40, 17))
    J[3, 5] = J[3, 9] = J[3].max() + 1.0  # exact tie: first wins, margin 0
    r = oracle.argmax_with_margin(J)
    s = np.sort(J, axis=1)
    np.testing.assert_allclose(r["value"], s[:, -1], rtol=0, atol=0)
    np.testing.assert_allclose(r["margin"], s[:, -1] - s[:, -2], rtol=0, atol=0)
    assert r["index"][3] == 5


# ----------------------------------------------------------------- the loss
def _loss_by_hand(theta, T, W, c, frames, pi_in, d_true, d_min, d_max):
    """Loss of a 1x1 sequence computed in mpmath from first principles: the
    bin-integrated Gaussian IRF (Sec. II-A), the photon form of the cost
    (eq. beta_div2), the 3x3 mixture in which every neighbour of a 1x1 frame
    is out of frame (flat) and the centre is the pixel's own previous state
    when detected (eq. predict, flat components), posterior means on the grid
    (eq. approx_post); loss = mean over frames of (mean - truth)^2."""
    mpmath.mp.dps = 40
    beta, sigma, s2 = (mpmath.mpf(x) for x in theta[:3])
    nu = [mpmath.mpf(x) for x in theta[3:12]]
    pulse = [mpmath.ncdf((j - c + mpmath.mpf(1) / 2) / sigma) - mpmath.ncdf((j - c - mpmath.mpf(1) / 2) / sigma)
             for j in range(W)]
    tot = sum(pulse)
    irf = [p / tot for p in pulse]
    m_f = (mpmath.mpf(d_min) + d_max) / 2
    v_f = (mpmath.mpf(d_max) - d_min) ** 2 / 12
    gauss = lambda d, m, V: mpmath.e ** (-(d - m) ** 2 / (2 * V)) / mpmath.sqrt(2 * mpmath.pi * V)
    prev = None  # (mean, var) of the previous frame if detected
    err = []
    for n, toa in enumerate(frames):
        def ell(d):
            acc = mpmath.mpf(0)
            for y in toa:
                j = y - d + c
                if 0 <= j < W:
                    acc += irf[j] ** beta
            return (beta + 1) / beta * acc
        def prior(d):
            flat_w = sum(nu[k] for k in range(9) if k != 4 or prev is None)
            f = flat_w * gauss(d, m_f, v_f + s2)
            if prev is not None:
                f += nu[4] * gauss(d, prev[0], prev[1] + s2)
            return f
        L = [mpmath.log(prior(d)) + ell(d) for d in range(T)]
        Lm = max(L)
        w = [mpmath.e ** (x - Lm) for x in L]
        Z = sum(w)
        mean = sum(d * w[d] for d in range(T)) / Z
        var = sum((d - mean) ** 2 * w[d] for d in range(T)) / Z
        err.append((mean - d_true[n]) ** 2)
        prev = (mean, var) if pi_in[n] > 0.5 else None
    return float(sum(err) / len(err))


def test_filter_loss_hand_derived():
    """filter_loss against a from-scratch mpmath evaluation of a 1x1,
    two-frame sequence whose second frame is undetected (so its depth output
    is NaN: the loss must be taken on the posterior mean). A swapped
    parameter order (IRF width vs random-walk variance) must change it."""
    T, W, c = 24, 7, 3
    frames = [[10, 11, 11, 12, 20], [11, 12, 12, 13, 3]]
    pi_in = [1.0, 0.3]
    d_true = [10.5, 12.0]
    theta = np.array([0.45, 1.3, 2.2, 0.05, 0.07, 0.06, 0.08, 0.4, 0.09, 0.1, 0.06, 0.09])
    mdl = make_model(rows=1, cols=1, T=T, W=W, c=c, beta=0.45, sigma=1.3, sigma_rw2=2.2)
    fr = [(np.array([0, len(f)]), np.array(f)) for f in frames]
    truth = [np.array([d]) for d in d_true]
    pin = [np.array([p]) for p in pi_in]
    got = oracle.filter_loss(theta, mdl, fr, truth, pi_in=pin)
    ref = _loss_by_hand(theta, T, W, c, frames, pi_in, d_true, mdl.d_min, mdl.d_max)
    assert np.isfinite(got)
    assert got == pytest.approx(ref, rel=1e-11, abs=1e-13)
    swapped = theta.copy()
    swapped[1], swapped[2] = theta[2], theta[1]
    assert abs(oracle.filter_loss(swapped, mdl, fr, truth, pi_in=pin) - ref) > 1e-6 * max(1.0, ref)


# ------------------------------------------- minimum divergence, single band
def test_min_divergence_beta_one_is_matched_filter_argmax():
    """beta = 1: the estimate is the argmax of the matched filter (Sec. II-B),
    computed here with numpy's convolution."""
    rng = np.random.default_rng(11)
    m = make_model(rows=3, cols=4, T=70, W=9, c=4, beta=1.0, sigma=1.6)
    row_ptr, toa = random_photons(rng, m.P, 70, lam=12)
    z = oracle.histogram(row_ptr, toa, 70)
    r = oracle.min_divergence(z, m)
    for p in range(m.P):
        mf = np.convolve(z[p].astype(float), m.irf[::-1])[np.arange(70) - m.c + m.W - 1]
        assert r["index"][p] == int(np.argmax(mf))
        assert r["value"][p] == pytest.approx(2.0 * mf.max(), rel=1e-13)


def test_min_divergence_beta_to_zero_is_max_likelihood():
    """beta -> 0: minimum beta-divergence = maximum likelihood (Sec. II-B,
    KL limit). With an IRF window covering every photon for every depth of
    the grid, the estimate at beta = 1e-7 equals the brute-force maximiser
    of sum_k log irf[y_k - d + c]."""
    T, W, c = 60, 41, 20
    j = np.arange(W)
    irf = np.exp(-np.abs(j - c) / 2.5) + 1e-3
    irf /= irf.sum()
    rng = np.random.default_rng(4)
    for trial in range(6):
        toa = np.sort(rng.integers(26, 35, size=7))
        m = make_model(rows=1, cols=1, T=T, W=W, c=c, beta=1e-7, irf=irf, d_lo=25, D=11)
        z = oracle.histogram(np.array([0, len(toa)]), toa, T)
        r = oracle.min_divergence(z, m)
        ll = [np.sum(np.log(irf[toa - d + c])) for d in range(25, 36)]
        assert r["d_hat"][0] == 25 + int(np.argmax(ll)), trial


def test_min_divergence_shift_equivariance_and_brute_force():
    """Shifting every ToA by k shifts the estimate by k (same value); the
    value equals a pure-Python double loop over photons and taps."""
    rng = np.random.default_rng(12)
    m = make_model(rows=1, cols=1, T=90, W=11, c=5, beta=0.6, sigma=2.0, d_lo=10, D=60)
    toa = np.concatenate([rng.integers(30, 36, 6), rng.integers(0, 90, 9)])
    toa = toa[(toa >= 20) & (toa < 70)]
    z = oracle.histogram(np.array([0, len(toa)]), toa, 90)
    r = oracle.min_divergence(z, m)
    for k in (3, -4, 7):
        zk = oracle.histogram(np.array([0, len(toa)]), toa + k, 90)
        rk = oracle.min_divergence(zk, m)
        assert rk["d_hat"][0] == r["d_hat"][0] + k
        assert rk["value"][0] == pytest.approx(r["value"][0], rel=1e-13)
    best, arg = -1.0, None
    for d in range(10, 70):
        acc = 0.0
        for y in toa:
            jj = int(y) - d + 5
            if 0 <= jj < 11:
                acc += m.irf[jj] ** 0.6
        acc *= 1.6 / 0.6
        if acc > best + 1e-12:
            best, arg = acc, d
    assert r["d_hat"][0] == arg and r["value"][0] == pytest.approx(best, rel=1e-12)


# ------------------------------------------- minimum divergence, multispectral
def _bands(rng, P=5, T=50):
    ms, zs = [], []
    for (W, c, s) in ((7, 3, 1.2), (9, 2, 1.8), (5, 2, 0.9)):
        m = make_model(rows=1, cols=P, T=T, W=W, c=c, beta=0.7, sigma=s, d_lo=3, D=40)
        row_ptr, toa = random_photons(rng, P, T, lam=9)
        ms.append(m)
        zs.append(oracle.histogram(row_ptr, toa, T))
    return ms, zs


def test_msl_single_band_is_min_divergence():
    """L = 1: the multispectral objective is log(c(d)/K) (Appendix,
    eq. div_MSL), whose maximiser is the single-band estimate."""
    rng = np.random.default_rng(21)
    ms, zs = _bands(rng)
    r1 = oracle.msl_min_divergence(zs[:1], ms[:1])
    r0 = oracle.min_divergence(zs[0], ms[0])
    np.testing.assert_array_equal(r1["index"], r0["index"])


def test_msl_hand_derived_and_invariances():
    """Two-band objective against an mpmath evaluation of
    log(c_1/K_1) + log(c_2/K_2) from the photon form; invariant under
    permuting bands and under scaling one band's counts; a band without
    photons drops out."""
    rng = np.random.default_rng(22)
    ms, zs = _bands(rng)
    J = oracle.msl_objective(zs[:2], ms[:2])
    mpmath.mp.dps = 30
    for p in range(5):
        for di, d in enumerate(range(3, 43)):
            tot = mpmath.mpf(0)
            for m, z in zip(ms[:2], zs[:2]):
                corr = mpmath.mpf(0)
                for t in range(m.T):
                    jj = t - d + m.c
                    if 0 <= jj < m.W and z[p, t]:
                        corr += z[p, t] * mpmath.mpf(m.irf[jj]) ** m.beta
                K = int(z[p].sum())
                tot = tot + (mpmath.log(corr / K) if corr > 0 else -mpmath.inf)
            if tot == -mpmath.inf:
                assert J[p, di] == -np.inf
            else:
                assert J[p, di] == pytest.approx(float(tot), rel=1e-12, abs=1e-12)
    perm = oracle.msl_objective([zs[2], zs[0], zs[1]], [ms[2], ms[0], ms[1]])
    np.testing.assert_allclose(perm, oracle.msl_objective(zs, ms), rtol=1e-13, atol=1e-13)
    scaled = oracle.msl_objective([zs[0] * 3, zs[1], zs[2]], ms)
    np.testing.assert_allclose(scaled, oracle.msl_objective(zs, ms), rtol=1e-13, atol=1e-13)
    empty = [zs[0], np.zeros_like(zs[1])]
    np.testing.assert_array_equal(oracle.msl_objective(empty, ms[:2]),
                                  oracle.msl_objective(zs[:1], ms[:1]))


def test_msl_rejects_mismatched_grids():
    ms, zs = _bands(np.random.default_rng(23))
    bad = make_model(rows=1, cols=5, T=50, W=7, c=3, beta=0.5, sigma=1.2, d_lo=3, D=40)
    with pytest.raises(ValueError):
        oracle.msl_objective([zs[0], zs[1]], [ms[0], bad])


# ------------------------------------------------------ pixel-dependent IRF
def _skewed_irfs(rng, P, W, c):
    """Asymmetric per-pixel IRFs peaking at tap c (a fast rise, a slow
    exponential tail of random length, as real detector IRFs)."""
    j = np.arange(W)
    out = np.zeros((P, W))
    for p in range(P):
        rise, tail = rng.uniform(0.6, 1.4), rng.uniform(1.5, 5.0)
        x = np.where(j <= c, np.exp(-((j - c) / rise) ** 2), np.exp(-(j - c) / tail))
        out[p] = x / x.sum()
    return out


def test_pixel_irf_equal_rows_reproduce_shared_path():
    """Equal per-pixel IRFs reproduce the shared-IRF oracle exactly (cost and
    a whole Algorithm 1 step, including a7)."""
    rng = np.random.default_rng(31)
    m = make_model(rows=4, cols=5, T=70, W=9, c=4, beta=0.45, sigma=1.5)
    row_ptr, toa = random_photons(rng, m.P, 70, lam=14)
    z = oracle.histogram(row_ptr, toa, 70)
    tiled = np.tile(m.irf, (m.P, 1))
    np.testing.assert_array_equal(oracle.cost_from_histogram_pirf(z, m, tiled), oracle.cost_from_histogram(z, m))
    st = oracle.init_state(m)
    a_state, a = oracle.step(m, st, z)
    b_state, b = oracle.step(m, st, z, irf_pix=tiled, c_pix=np.full(m.P, m.c))
    for k in ("mean", "var", "argmax", "intensity", "background", "pi0_next"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(a_state.b, b_state.b)


def test_pixel_irf_photon_form_shift_and_matched_filter():
    """Per-pixel cost against (i) a double loop over each pixel's photons
    (eq. beta_div2 as printed), (ii) the same IRF stored with a leading zero
    tap and c + 1 (same pulse), (iii) numpy's convolution at beta = 1."""
    rng = np.random.default_rng(32)
    P, W, c, T = 6, 12, 3, 64
    m = make_model(rows=2, cols=3, T=T, W=W, c=c, beta=0.55, d_lo=2, D=58)
    irfs = _skewed_irfs(rng, P, W, c)
    cpix = rng.integers(2, 5, P)
    row_ptr, toa = random_photons(rng, P, T, lam=10)
    z = oracle.histogram(row_ptr, toa, T)
    ell = oracle.cost_from_histogram_pirf(z, m, irfs, cpix)
    for p in range(P):
        ref = np.zeros(m.D)
        for y in toa[row_ptr[p]:row_ptr[p + 1]]:
            for di, d in enumerate(range(2, 60)):
                jj = int(y) - d + int(cpix[p])
                if 0 <= jj < W:
                    ref[di] += irfs[p, jj] ** 0.55
        np.testing.assert_allclose(ell[p], (1.55 / 0.55) * ref, rtol=1e-12, atol=1e-12)
    padded = np.concatenate([np.zeros((P, 1)), irfs], axis=1)
    np.testing.assert_allclose(oracle.cost_from_histogram_pirf(z, m, padded, cpix + 1), ell, rtol=1e-14, atol=1e-14)
    m1 = make_model(rows=2, cols=3, T=T, W=W, c=c, beta=1.0, d_lo=0, D=T)
    ell1 = oracle.cost_from_histogram_pirf(z, m1, irfs)
    for p in range(P):
        conv = np.convolve(z[p].astype(float), irfs[p, ::-1])
        np.testing.assert_allclose(ell1[p], 2.0 * conv[np.arange(T) - c + W - 1], rtol=1e-13, atol=1e-13)


def test_pixel_irf_reflectivity_matches_generic_optimiser():
    """a7 with each pixel's own IRF: the Poisson MLE of eq. lik_bg_poisson
    at d*, checked against scipy's bounded optimiser of the full
    likelihood with that pixel's IRF, and the identity K = r S + b T."""
    rng = np.random.default_rng(33)
    P, W, c, T = 5, 15, 4, 80
    m = make_model(rows=1, cols=P, T=T, W=W, c=c, beta=0.5)
    irfs = _skewed_irfs(rng, P, W, c)
    z = np.zeros((P, T), dtype=np.int64)
    for p in range(P):
        lam = 30 * np.concatenate([np.zeros(40 - c), irfs[p], np.zeros(T - 40 + c - W)]) + 0.15
        z[p] = rng.poisson(lam)
    dstar = np.full(P, 40)
    r, b = oracle.background_intensity(z, m, dstar, np.ones(P, bool), irfs, np.full(P, c))
    for p in range(P):
        s = np.zeros(T)
        s[40 - c:40 - c + W] = irfs[p]
        nll = lambda x: -(np.sum(z[p] * np.log(x[0] * s + x[1] + 1e-300)) - x[0] * s.sum() - x[1] * T)
        res = optimize.minimize(nll, x0=[20.0, 0.2], bounds=[(0, None), (1e-9, None)], method="L-BFGS-B",
                                options=dict(ftol=1e-15, gtol=1e-12, maxiter=2000))
        assert r[p] == pytest.approx(res.x[0], rel=2e-4)
        assert z[p].sum() == pytest.approx(r[p] * s.sum() + b[p] * T, rel=1e-9)


# ------------------------------- continuous depth, Gaussian IRF (Sec. II-B, V)
def _csr(lists):
    counts = [len(x) for x in lists]
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    toa = np.concatenate([np.asarray(x, dtype=np.int64) for x in lists]) if sum(counts) else np.zeros(0, np.int64)
    return row_ptr, toa


def test_gauss_cost_is_photon_form_with_sampled_gaussian_taps():
    """On the grid, the Gaussian-IRF cost equals the photon form of the
    discrete cost (cost_from_photons) with taps irf[j] = N(j - c; 0, sigma^2)
    sampled from the density (wide enough that no photon leaves the taps)."""
    sigma, beta, c = 2.3, 0.35, 30
    W = 2 * c + 1
    j = np.arange(W) - c
    taps = np.exp(-j * j / (2 * sigma * sigma)) / np.sqrt(2 * np.pi * sigma * sigma)
    m = make_model(rows=1, cols=3, T=80, W=W, c=c, beta=beta, irf=taps, d_lo=20, D=40)
    row_ptr, toa = _csr([[31, 33, 47, 50], [45], [30, 30, 58]])
    ref = oracle.cost_from_photons(row_ptr, toa, m)
    for p in range(3):
        y = toa[row_ptr[p]:row_ptr[p + 1]]
        np.testing.assert_allclose(oracle.gauss_cost(y, m.grid, sigma, beta), ref[p], rtol=1e-13, atol=0)


def test_gauss_min_divergence_closed_forms():
    """One photon: the maximiser is the photon itself and the cost is
    (beta+1)/beta (2 pi sigma^2)^(-beta/2). Two photons closer than 2h
    (h = sigma / sqrt(beta)): the objective is unimodal and symmetric, so the
    maximiser is their midpoint. No photon: d_lo, cost 0."""
    sigma, beta = 3.0, 0.3
    h = sigma / np.sqrt(beta)
    row_ptr, toa = _csr([[40], [37, 45], [], [30, 30 + int(1.9 * h)]])
    r = oracle.gauss_min_divergence(row_ptr, toa, sigma, beta, 10, 80)
    assert r["depth"][0] == 40.0
    assert r["value"][0] == pytest.approx((beta + 1) / beta * (2 * np.pi * sigma ** 2) ** (-beta / 2), rel=1e-14)
    assert r["depth"][1] == pytest.approx(41.0, abs=1e-9)
    assert r["depth"][2] == 10.0 and r["value"][2] == 0.0
    assert r["depth"][3] == pytest.approx(30 + int(1.9 * h) / 2, abs=1e-9)


def test_gauss_min_divergence_brute_force_and_stationarity():
    """Random tiny pixels: where the grid margin is clear, the result is the
    global maximiser of the continuous objective found by a dense search
    (step 1e-4 over the grid's span, then a golden-section polish by scipy);
    at every result the objective is stationary and concave."""
    rng = np.random.default_rng(11)
    sigma, beta, d_lo, D = 1.8, 0.45, 5, 50
    lists = [list(rng.integers(0, 60, rng.integers(1, 9))) for _ in range(25)]
    row_ptr, toa = _csr(lists)
    r = oracle.gauss_min_divergence(row_ptr, toa, sigma, beta, d_lo, D)
    fine = np.arange(d_lo, d_lo + D - 1 + 1e-9, 1e-4)
    checked = 0
    for p in range(25):
        y = toa[row_ptr[p]:row_ptr[p + 1]].astype(float)
        d = r["depth"][p]
        # stationary and concave there (central differences), unless held
        # at an end of the span, where the objective rises towards the end
        e = 1e-4
        f = lambda x: oracle.gauss_cost(y, x, sigma, beta)[0]
        g1 = (f(d + e) - f(d - e)) / (2 * e)
        g2 = (f(d + e) - 2 * f(d) + f(d - e)) / (e * e)
        if d == d_lo:
            assert g1 <= 0
        elif d == d_lo + D - 1:
            assert g1 >= 0
        else:
            assert abs(g1) <= 1e-7 * max(1.0, f(d)) and g2 < 0
        if r["margin"][p] > 1e-3 * r["value"][p]:
            J = oracle.gauss_cost(y, fine, sigma, beta)
            x0 = fine[np.argmax(J)]
            res = optimize.minimize_scalar(lambda x: -f(x), method="bounded", options=dict(xatol=1e-10),
                                           bounds=(max(d_lo, x0 - 2e-4), min(d_lo + D - 1, x0 + 2e-4)))
            assert d == pytest.approx(res.x, abs=1e-5)
            assert r["value"][p] >= -res.fun - 1e-12 * abs(res.fun)
            checked += 1
    assert checked >= 15


def test_gauss_min_divergence_shift_equivariance():
    """Shifting every ToA by k bins shifts the continuous estimate by k."""
    rng = np.random.default_rng(4)
    lists = [list(rng.integers(20, 60, rng.integers(1, 12))) for _ in range(12)]
    row_ptr, toa = _csr(lists)
    a = oracle.gauss_min_divergence(row_ptr, toa, 2.5, 0.3, 0, 100)
    b = oracle.gauss_min_divergence(row_ptr, toa + 17, 2.5, 0.3, 0, 100)
    np.testing.assert_allclose(b["depth"], a["depth"] + 17, atol=1e-9)
    np.testing.assert_allclose(b["value"], a["value"], rtol=1e-12)
