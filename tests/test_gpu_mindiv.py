"""GPU parity of the minimum-divergence estimates (single band, Sec. II-B;
multispectral, Appendix eq. div_MSL) and of the frame step with per-pixel
IRFs (Sec. II-A) against the FP64 oracle, through the C ABI.

Tolerances. Single-band value: the engines' cost error (fp32 and split fp16:
relative 2e-6 of max ell; single fp16: 2^-12 relative per tap, so 2.5e-4 of
max ell). The argmax is identical wherever the oracle's margin exceeds twice
that error, and elsewhere lies in the oracle's tie set (its objective within
the same bound of the maximum). Multispectral value: each band adds the log of
a correlation computed to the relative error above, so the bound is that
error plus the fp32 rounding of log2 and of the band sum, times the number
of bands.
Per-pixel IRF step: the fp32 per-pixel path's rules (mean 1e-4 sd, variance
1e-3 relative); equal rows reproduce the shared-IRF step bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity_util import compare, frame_hist, gpu_outputs_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ENGINES = ["fp32", "fp16", "fp16x2"]


def cost_err(prec):
    return 2.5e-4 if prec == "fp16" else 2e-6


def poisson_hist(rows, cols, T, irf, c, depth, n_sig, n_bg, seed):
    """fp16 [P, T] histograms: bin t ~ Poisson(n_sig * irf[t - depth + c] +
    n_bg / T) (the observation model of Sec. II-A), depth and n_sig per
    pixel."""
    P = rows * cols
    g = torch.Generator().manual_seed(seed)
    W = len(irf)
    rate = torch.full((P, T), n_bg / T, dtype=torch.float64)
    taps = torch.arange(W)
    idx = torch.as_tensor(depth, dtype=torch.int64)[:, None] - c + taps[None, :]
    ok = (idx >= 0) & (idx < T)
    add = torch.as_tensor(n_sig, dtype=torch.float64)[:, None] * torch.as_tensor(irf)[None, :]
    rate.scatter_add_(1, idx.clamp(0, T - 1), torch.where(ok, add, 0.0))
    return torch.poisson(rate, generator=g).to(torch.float16)


def check_argmax(am_gpu, J, value_gpu, value_tol, label):
    """GPU argmax against the oracle objective J [n, D] (first maximiser,
    ties within ``value_tol``); the value at the GPU's index within
    value_tol of the oracle's maximum."""
    r = oracle.argmax_with_margin(J)
    idx = am_gpu.astype(np.int64)
    sure = r["margin"] > 2 * value_tol
    bad = np.flatnonzero(sure & (idx != r["index"]))
    assert bad.size == 0, f"{label}: argmax differs at {bad[:8]} (margins {r['margin'][bad[:8]]})"
    rows = np.arange(J.shape[0])
    assert np.all((idx >= 0) & (idx < J.shape[1])), f"{label}: argmax off the grid"
    at = J[rows, idx]
    fin = np.isfinite(r["value"])
    gap = np.where(fin, r["value"] - at, 0.0)
    tolv = np.broadcast_to(np.asarray(value_tol, dtype=np.float64), gap.shape)
    assert np.all(gap <= 2 * tolv), f"{label}: argmax outside the tie set (gap {gap.max():.3g})"
    ref_v = r["value"]
    both_inf = np.isneginf(ref_v) & np.isneginf(value_gpu)
    err = np.where(both_inf, 0.0, np.abs(value_gpu.astype(np.float64) - ref_v))
    assert np.all(err <= value_tol), (
        f"{label}: value error {np.nanmax(err / value_tol):.3g}x tolerance")
    return r


# ------------------------------------------------------------ single band ---
@pytest.mark.parametrize("prec", ENGINES)
@pytest.mark.parametrize("shape", ["c4crop", "offset_grid"])
def test_min_divergence_matches_oracle(lib, prec, shape):
    """5x8 crop of the 4096-bin histogram workload (ragged 4x4 blocks) and a
    200-bin frame whose grid starts at d_lo = 13 with D = 150 (a grid that
    ends inside a 32-depth pair)."""
    if shape == "c4crop":
        wl = synth.config4(frames=1, rows=5, cols=8)
        hist = wl.hist[0]
    else:
        wl = synth.tiny_workload(rows=3, cols=7, T=200, W=9, c=4, frames=1)
        wl.d_lo, wl.D, wl.d_min, wl.d_max = 13, 150, 13.0, 162.0
        z = frame_hist(wl.frames[0], wl.T)
        hist = torch.as_tensor(z, dtype=torch.float16)
        hist[4] = 0  # a pixel without photons: ell = 0 everywhere
    ctx = lib.Context(wl.params(), prec)
    am, val = ctx.min_divergence(hist.to(DEV).contiguous())
    assert ctx.last_device_status() == 0
    model = oracle.Model.from_params(wl.params())
    z = frame_hist(hist, wl.T)
    J = oracle.cost_from_histogram(z, model)
    tol = cost_err(prec) * np.maximum(1.0, J.max(axis=1))
    r = check_argmax(am.cpu().numpy() - wl.d_lo, J, val.cpu().numpy(), tol, f"{prec} {shape}")
    ref = oracle.min_divergence(z, model)
    np.testing.assert_array_equal(ref["index"], r["index"])
    if shape == "offset_grid":
        assert int(am[4]) == wl.d_lo and float(val[4]) == 0.0


def test_min_divergence_first_maximiser_on_ties(lib):
    """Exact ties take the first grid depth. The IRF is symmetric about its
    peak tap c (bit for bit), so two photons in adjacent bins t and t+1 give
    ell(t) = s (h[c] + h[c+1]) and ell(t+1) = s (h[c-1] + h[c]): the same two
    terms, equal in any summation order. t is placed so that the tie
    crosses a lane group (t = 3), a 16-depth tile (15), a 32-depth pair
    (31, 63) or none (100, 200); one pixel has a single photon (unique
    maximum at its bin) and one none (every depth ties at 0: d_lo)."""
    wl = synth.tiny_workload(rows=2, cols=4, T=256, W=9, c=4, frames=1)
    model = oracle.Model.from_params(wl.params())
    z = np.zeros((wl.P, wl.T), dtype=np.int64)
    for p, t in enumerate([100, 31, 15, 3, 63, 200]):
        z[p, t] = z[p, t + 1] = 1
    z[6, 50] = 1
    ref = oracle.min_divergence(z, model)
    np.testing.assert_array_equal(ref["d_hat"], [100, 31, 15, 3, 63, 200, 50, 0])
    for prec in ENGINES:
        ctx = lib.Context(wl.params(), prec)
        am, val = ctx.min_divergence(torch.as_tensor(z, dtype=torch.float16).to(DEV))
        assert ctx.last_device_status() == 0
        np.testing.assert_array_equal(am.cpu().numpy(), ref["d_hat"], err_msg=prec)


def test_min_divergence_full_size_sampled(lib):
    """The 256x256, T = 4096 histogram frame: every pixel on the GPU, 256
    sampled pixels (corners, edges, object boundaries, random) against the
    oracle, for the split fp16 engine."""
    wl = synth.config4(device=DEV, frames=1)
    ctx = lib.Context(wl.params(), "fp16x2")
    am, val = ctx.min_divergence(wl.hist[0])
    assert ctx.last_device_status() == 0
    rng = np.random.default_rng(3)
    pix = np.unique(np.concatenate([rng.choice(wl.P, 240, replace=False),
                                    [0, 255, wl.P - 256, wl.P - 1, 40 * 256 + 20,
                                     40 * 256 + 19, 180 * 256 + 168, 100 * 256 + 100]]))
    model = oracle.Model.from_params(wl.params())
    z = frame_hist(wl.hist[0], wl.T, pix)
    J = oracle.cost_from_histogram(z, model)
    tol = cost_err("fp16x2") * np.maximum(1.0, J.max(axis=1))
    check_argmax(am.cpu().numpy()[pix] - wl.d_lo, J, val.cpu().numpy()[pix], tol, "full size")


# ---------------------------------------------------------- multispectral ---
def msl_bands(rows, cols, T, nb, seed=0, d_lo=0, D=None):
    """nb bands sharing T, the grid and beta, each with its own Gaussian IRF
    (sigma, W and peak tap differ) and reflectivity: a depth ramp plus a
    step; pixel 3 has no photons in band 1, pixel 5 none in any band."""
    D = T - d_lo if D is None else D
    specs = [(3.0, 33, 16), (2.0, 17, 6), (4.5, 41, 24), (1.5, 12, 3)][:nb]
    P = rows * cols
    x = np.arange(P) % cols
    depth = (T // 4 + 3 * x + 40 * (np.arange(P) >= P // 2)).astype(np.int64)
    base = dict(rows=rows, cols=cols, T=T, d_lo=d_lo, D=D, d_min=float(d_lo),
                d_max=float(d_lo + D - 1), beta=0.4, nu=synth.default_nu(), sigma_rw2=3.0)
    params, hists = [], []
    rng = np.random.default_rng(seed)
    for l, (s, W, c) in enumerate(specs):
        p = dict(base, irf=synth.gaussian_irf(s, W, c), c=c)
        n_sig = rng.uniform(2.0, 12.0, P)
        h = poisson_hist(rows, cols, T, p["irf"], c, depth, n_sig, 20.0, seed * 10 + l)
        if l == 1:
            h[3] = 0
        h[5] = 0
        params.append(p)
        hists.append(h)
    return params, hists


@pytest.mark.parametrize("prec", ENGINES)
@pytest.mark.parametrize("nb", [1, 2, 3, 4])
def test_min_divergence_msl_matches_oracle(lib, prec, nb):
    params, hists = msl_bands(5, 9, 512, nb)
    ctxs = [lib.Context(p, prec) for p in params]
    am, val = lib.min_divergence_msl(ctxs, [h.to(DEV).contiguous() for h in hists])
    assert ctxs[0].last_device_status() == 0
    models = [oracle.Model.from_params(p) for p in params]
    zs = [frame_hist(h, 512) for h in hists]
    J = oracle.msl_objective(zs, models)
    # per band: the correlation's relative error, one ulp of log2 (|log2 c| <
    # 32) and one rounding of the running sum (|J| < 128)
    tol = nb * (2.0 * cost_err(prec) + 4e-5) + 1e-5
    r = check_argmax(am.cpu().numpy(), J, val.cpu().numpy(), tol, f"msl {prec} nb={nb}")
    ref = oracle.msl_min_divergence(zs, models)
    np.testing.assert_array_equal(ref["index"], r["index"])
    # the all-empty pixel: objective 0 at every depth -> first grid point
    assert int(am[5]) == 0 and float(val[5]) == 0.0


def test_min_divergence_msl_full_size_sampled(lib):
    """Two bands at the benchmark's size, as the benchmark times them: frames
    0 and 1 of the 256x256, T = 4096 workload, the second band with a
    sigma = 4 Gaussian IRF of the same taps. Every pixel on the GPU; 256
    sampled pixels (corners, edges, object boundaries, random) against the
    oracle's multispectral objective, split fp16 engine."""
    wl = synth.config4(device=DEV, frames=2)
    p2 = dict(wl.params(), irf=synth.gaussian_irf(4.0, wl.W, wl.c))
    ctxs = [lib.Context(wl.params(), "fp16x2"), lib.Context(p2, "fp16x2")]
    am, val = lib.min_divergence_msl(ctxs, [wl.hist[0], wl.hist[1]])
    assert all(c.last_device_status() == 0 for c in ctxs)
    rng = np.random.default_rng(4)
    pix = np.unique(np.concatenate([rng.choice(wl.P, 240, replace=False),
                                    [0, 255, wl.P - 256, wl.P - 1, 40 * 256 + 20,
                                     40 * 256 + 19, 180 * 256 + 168, 100 * 256 + 100]]))
    models = [oracle.Model.from_params(wl.params()), oracle.Model.from_params(p2)]
    zs = [frame_hist(wl.hist[0], wl.T, pix), frame_hist(wl.hist[1], wl.T, pix)]
    J = oracle.msl_objective(zs, models)
    tol = 2 * (2.0 * cost_err("fp16x2") + 4e-5) + 1e-5
    check_argmax(am.cpu().numpy()[pix] - wl.d_lo, J, val.cpu().numpy()[pix], tol, "msl full size")


def test_min_divergence_msl_one_band_equals_single(lib):
    """One band: argmax of log(c/K) is the argmax of ell (the same first
    maximiser), and value = log(ell * beta / (beta+1)) - log K."""
    params, hists = msl_bands(4, 8, 256, 1, seed=2, d_lo=5, D=200)
    for prec in ENGINES:
        ctx = lib.Context(params[0], prec)
        h = hists[0].to(DEV).contiguous()
        am1, v1 = ctx.min_divergence(h)
        am2, v2 = lib.min_divergence_msl([ctx], [h])
        assert ctx.last_device_status() == 0
        np.testing.assert_array_equal(am1.cpu().numpy(), am2.cpu().numpy(), err_msg=prec)


def test_min_divergence_msl_rejects_mismatch(lib):
    params, hists = msl_bands(4, 8, 256, 2)
    bad = dict(params[1], D=params[1]["D"] - 1, d_max=params[1]["d_max"] - 1)
    a, b = lib.Context(params[0]), lib.Context(bad)
    with pytest.raises(lib.R3DError) as e:
        lib.min_divergence_msl([a, b], [h.to(DEV) for h in hists])
    assert e.value.status == -1
    c = lib.Context(params[1], "fp16")
    with pytest.raises(lib.R3DError) as e:
        lib.min_divergence_msl([a, c], [h.to(DEV) for h in hists])
    assert e.value.status == -1


@pytest.mark.parametrize("bad", [1.5, -0.0, 2050.0, -3.0])
def test_min_divergence_count_validation(lib, bad):
    params, hists = msl_bands(4, 8, 256, 2)
    for prec in ENGINES:
        ctx = lib.Context(params[0], prec)
        h = hists[0].clone()
        h[6, 77] = bad
        ctx.min_divergence(h.to(DEV))
        assert ctx.last_device_status() == -3, (prec, bad)
        ctx2 = lib.Context(params[1], prec)
        lib.min_divergence_msl([ctx2, ctx], [hists[1].to(DEV), h.to(DEV)])
        assert ctx2.last_device_status() == -3, (prec, bad)
        assert ctx.last_device_status() == 0


# ------------------------------------------------------- per-pixel IRFs ---
def pirf_workload(frames=3, seed=0):
    """10x7 photon-list sequence (T = 120, W = 11) whose pixels each have a
    Gaussian IRF of their own width (sigma 1 to 3 bins) and peak tap."""
    wl = synth.tiny_workload(seed=seed, rows=10, cols=7, T=120, W=11, c=5, frames=frames,
                             n_sig=8.0, n_bg=5.0)
    rng = np.random.default_rng(seed + 100)
    sig = rng.uniform(1.0, 3.0, wl.P)
    c_pix = rng.integers(3, 8, wl.P).astype(np.int32)
    irf_pix = np.stack([synth.gaussian_irf(s, wl.W, int(c)) for s, c in zip(sig, c_pix)])
    c_pix = np.argmax(irf_pix, axis=1).astype(np.int32)
    return wl, irf_pix, c_pix


def _state_dev(st):
    return [torch.tensor(a, dtype=torch.float32, device=DEV) for a in (st.m, st.v, st.pi, st.b)]


@pytest.mark.parametrize("form", ["csr", "hist"])
@pytest.mark.parametrize("with_c", [True, False])
def test_step_pirf_teacher_forced(lib, form, with_c):
    """Each frame starts from the oracle's state; the oracle steps with the
    same per-pixel IRFs (and peak taps, or the context's c)."""
    wl, irf_pix, c_pix = pirf_workload()
    if not with_c:
        c_pix = None
    model = oracle.Model.from_params(wl.params())
    ctx = lib.Context(wl.params())
    st = oracle.init_state(model)
    irf_d = torch.as_tensor(irf_pix, device=DEV)
    c_d = None if c_pix is None else torch.as_tensor(c_pix, device=DEV)
    g0 = torch.Generator().manual_seed(9)
    pi_in = torch.rand(wl.P, generator=g0)
    faulty = (torch.rand(wl.P, generator=g0) < 0.1).to(torch.uint8)
    for n in range(wl.nframes):
        fr = wl.frames[n]
        z = frame_hist(fr, wl.T)
        use_pf = n == 1
        new, ref = oracle.step(model, st, z, irf_pix=irf_pix, c_pix=c_pix,
                               pi_in=pi_in.numpy().astype(np.float64) if use_pf else None,
                               faulty=faulty.numpy().astype(bool) if use_pf else None)
        prev = lib.State(*_state_dev(st))
        nxt = lib.State.empty(wl.P, DEV)
        out = lib.Outputs.empty(wl.P, DEV)
        frame = ((fr.row_ptr.to(DEV), fr.toa.to(DEV)) if form == "csr"
                 else torch.as_tensor(z, dtype=torch.float16, device=DEV))
        ctx.step_pirf(frame, irf_d, prev, nxt, out, c_pix=c_d,
                      pi_in=pi_in.to(DEV) if use_pf else None,
                      faulty=faulty.to(DEV) if use_pf else None)
        assert ctx.last_device_status() == 0
        g = gpu_outputs_np(out)
        g["mean"] = nxt.m.cpu().numpy()
        compare(g, ref, label=f"pirf {form} c={with_c} frame {n}")
        np.testing.assert_allclose(nxt.pi.cpu().numpy(), new.pi, atol=1e-5)
        st = new


def test_step_pirf_equal_rows_reproduce_shared_step(lib):
    """Every row equal to the context's IRF (and c_pix NULL): the photon-list
    step is bit-identical to r3d_step_csr, and the histogram form of the
    per-pixel step to its photon-list form."""
    wl = synth.tiny_workload(rows=6, cols=9, T=96, W=9, c=4, frames=2)
    ctx = lib.Context(wl.params())
    irf_d = torch.as_tensor(np.tile(wl.irf, (wl.P, 1)), device=DEV)
    init = lib.State.empty(wl.P, DEV)
    ctx.state_init(init)
    runs = {}
    for mode in ("csr", "pirf_csr", "pirf_hist"):
        prev = init.clone()
        res = []
        for fr in wl.frames:
            nxt = lib.State.empty(wl.P, DEV)
            out = lib.Outputs.empty(wl.P, DEV)
            rp, toa = fr.row_ptr.to(DEV), fr.toa.to(DEV)
            if mode == "csr":
                ctx.step_csr(rp, toa, prev, nxt, out)
            elif mode == "pirf_csr":
                ctx.step_pirf((rp, toa), irf_d, prev, nxt, out)
            else:
                ctx.step_pirf(ctx.histogram(rp, toa), irf_d, prev, nxt, out)
            res.append((gpu_outputs_np(out), [t.cpu().numpy() for t in (nxt.m, nxt.v, nxt.pi, nxt.b)]))
            prev = nxt
        runs[mode] = res
        assert ctx.last_device_status() == 0
    for other in ("pirf_csr", "pirf_hist"):
        for (oa, sa), (ob, sb) in zip(runs["csr"], runs[other]):
            for k in oa:
                np.testing.assert_array_equal(oa[k], ob[k], err_msg=f"{other} {k}")
            for a, b in zip(sa, sb):
                np.testing.assert_array_equal(a, b, err_msg=other)


@pytest.mark.parametrize("case", ["negative_tap", "zero_row", "nan_tap", "c_out_of_range"])
def test_step_pirf_rejects_invalid_irf(lib, case):
    wl, irf_pix, c_pix = pirf_workload(frames=1)
    irf_pix = irf_pix.copy()
    c_pix = c_pix.copy()
    if case == "negative_tap":
        irf_pix[13, 2] = -1e-3
    elif case == "zero_row":
        irf_pix[13] = 0.0
    elif case == "nan_tap":
        irf_pix[13, 4] = np.nan
    else:
        c_pix[13] = wl.W
    ctx = lib.Context(wl.params())
    init = lib.State.empty(wl.P, DEV)
    ctx.state_init(init)
    nxt = lib.State.empty(wl.P, DEV)
    out = lib.Outputs.empty(wl.P, DEV)
    fr = wl.frames[0]
    ctx.step_pirf((fr.row_ptr.to(DEV), fr.toa.to(DEV)), torch.as_tensor(irf_pix, device=DEV),
                  init, nxt, out, c_pix=torch.as_tensor(c_pix, device=DEV))
    assert ctx.last_device_status() == -1
    # the other pixels are still computed
    ok = np.ones(wl.P, bool)
    ok[13] = False
    assert np.all(np.isfinite(nxt.m.cpu().numpy()[ok]))


def test_step_pirf_argument_errors(lib):
    wl, irf_pix, c_pix = pirf_workload(frames=1)
    ctx = lib.Context(wl.params())
    st = lib.State.empty(wl.P, DEV)
    ctx.state_init(st)
    nxt = lib.State.empty(wl.P, DEV)
    out = lib.Outputs.empty(wl.P, DEV)
    fr = wl.frames[0]
    with pytest.raises(lib.R3DError) as e:
        ctx.step_pirf((fr.row_ptr.to(DEV), fr.toa.to(DEV)), None, st, nxt, out)
    assert e.value.status == -1
    with pytest.raises(lib.R3DError) as e:
        ctx.step_pirf((fr.row_ptr.to(DEV), fr.toa.to(DEV)), torch.as_tensor(irf_pix, device=DEV),
                      st, st, out)
    assert e.value.status == -1


# ------------------------------- continuous depth, Gaussian IRF (Sec. II-B, V)
def _gauss_check(wl, sigma, depth, value, gidx, label, pixels=None):
    """GPU continuous estimates against the oracle (fp64). Where the
    oracle's grid margin exceeds 1e-4 of its value the basin is unambiguous:
    depth within 1e-3 bins plus an fp32 ulp, value within 1e-5 relative,
    grid maximiser identical. Elsewhere the GPU's depth must be as good:
    the objective there within 1e-5 relative of the oracle's maximum."""
    rp = wl.frames[0].row_ptr.numpy()
    toa = wl.frames[0].toa.numpy()
    r = oracle.gauss_min_divergence(rp, toa, sigma, wl.beta, wl.d_lo, wl.D)
    P = len(rp) - 1
    pix = np.arange(P) if pixels is None else np.asarray(pixels)
    d = depth.astype(np.float64)
    sure = r["margin"] > 1e-4 * r["value"]
    n_sure = 0
    for p in pix:
        y = toa[rp[p]:rp[p + 1]]
        if sure[p]:
            n_sure += 1
            tol = 1e-3 + float(np.spacing(np.float32(abs(r["depth"][p]) + 1)))
            assert abs(d[p] - r["depth"][p]) <= tol, (label, p, d[p], r["depth"][p])
            assert value[p] == pytest.approx(r["value"][p], rel=1e-5, abs=1e-30), (label, p)
            assert gidx[p] == wl.d_lo + r["grid_index"][p], (label, p)
        else:
            at = oracle.gauss_cost(y, d[p], sigma, wl.beta)[0] if len(y) else 0.0
            assert at >= r["value"][p] * (1 - 1e-5), (label, p, at, r["value"][p])
    return n_sure


@pytest.mark.parametrize("shape", ["video_crop", "offset_grid"])
def test_min_divergence_gauss_matches_oracle(lib, shape):
    if shape == "video_crop":
        wl = synth.config2(rows=8, cols=12, frames=1)
        sigma = 3.0
    else:
        wl = synth.tiny_workload(rows=5, cols=9, T=200, W=9, c=4, frames=1, sigma=2.0, n_sig=12, n_bg=6)
        wl.d_lo, wl.D, wl.d_min, wl.d_max = 13, 150, 13.0, 162.0
        sigma = 2.0
    ctx = lib.Context(wl.params())
    f = wl.frames[0]
    depth, value, gidx = ctx.min_divergence_gauss(f.row_ptr.to(DEV), f.toa.to(DEV), sigma)
    assert ctx.last_device_status() == 0
    n = _gauss_check(wl, sigma, depth.cpu().numpy(), value.cpu().numpy(), gidx.cpu().numpy(), shape)
    assert n >= 0.8 * wl.P


def test_min_divergence_gauss_edge_cases(lib):
    """A pixel without photons gets d_lo and 0; one photon gives its bin; a
    ToA outside [0, T) is reported; sigma must be positive."""
    wl = synth.tiny_workload(rows=1, cols=4, T=64, W=9, c=4, frames=1)
    ctx = lib.Context(wl.params())
    rp = torch.tensor([0, 0, 1, 3, 5], dtype=torch.int32, device=DEV)
    toa = torch.tensor([40, 10, 20, 63, 0], dtype=torch.int16, device=DEV)
    depth, value, gidx = ctx.min_divergence_gauss(rp, toa, 1.5)
    assert ctx.last_device_status() == 0
    d = depth.cpu().numpy()
    assert d[0] == wl.d_lo and float(value[0]) == 0.0
    assert d[1] == 40.0 and int(gidx[1]) == 40
    r = oracle.gauss_min_divergence(rp.cpu().numpy(), toa.cpu().numpy(), 1.5, wl.beta, wl.d_lo, wl.D)
    np.testing.assert_allclose(d, r["depth"], atol=1e-3)
    np.testing.assert_allclose(value.cpu().numpy(), r["value"], rtol=1e-5)
    bad = torch.tensor([0, 1, 1, 1, 1], dtype=torch.int32, device=DEV)
    ctx.min_divergence_gauss(bad, torch.tensor([64], dtype=torch.int16, device=DEV), 1.5)
    assert ctx.last_device_status() == -2  # R3D_ERANGE
    with pytest.raises(lib.R3DError):
        ctx.min_divergence_gauss(rp, toa, 0.0)
    with pytest.raises(lib.R3DError):
        ctx.min_divergence_gauss(rp, toa, float("nan"))


def test_min_divergence_gauss_full_video_frame_sampled(lib):
    """The 128x128 video's first frame (T=1500, sigma=3): 300 sampled pixels
    against the oracle."""
    wl = synth.config2(frames=1)
    ctx = lib.Context(wl.params())
    f = wl.frames[0]
    depth, value, gidx = ctx.min_divergence_gauss(f.row_ptr.to(DEV), f.toa.to(DEV), 3.0)
    assert ctx.last_device_status() == 0
    rng = np.random.default_rng(3)
    pix = np.unique(np.concatenate([[0, 127, wl.P - 128, wl.P - 1], rng.choice(wl.P, 296, replace=False)]))
    sub_rp = [0]
    sub_toa = []
    rp, toa = f.row_ptr.numpy(), f.toa.numpy()
    for p in pix:
        sub_toa.append(toa[rp[p]:rp[p + 1]])
        sub_rp.append(sub_rp[-1] + rp[p + 1] - rp[p])
    r = oracle.gauss_min_divergence(np.array(sub_rp), np.concatenate(sub_toa), 3.0, wl.beta, wl.d_lo, wl.D)
    d = depth.cpu().numpy()[pix].astype(np.float64)
    v = value.cpu().numpy()[pix]
    sure = r["margin"] > 1e-4 * r["value"]
    assert sure.sum() >= 250
    np.testing.assert_allclose(d[sure], r["depth"][sure], atol=1e-3 + 2.5e-4)
    np.testing.assert_allclose(v[sure], r["value"][sure], rtol=1e-5)
    for i in np.flatnonzero(~sure):
        y = np.concatenate(sub_toa)[sub_rp[i]:sub_rp[i + 1]]
        assert oracle.gauss_cost(y, d[i], 3.0, wl.beta)[0] >= r["value"][i] * (1 - 1e-5)
