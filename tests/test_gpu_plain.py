"""GPU parity of the plain fp32 path (photon lists and fp16 histograms)
against the FP64 oracle, called through the C ABI.

Tolerances (see parity_util): argmax identical where the oracle margin
exceeds 1e-3 nats; mean within 1e-4 * max(1, posterior sd) bins; variance
within 1e-3 relative; reflectivity/background within 1e-3 relative;
histograms bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity_util import compare, frame_hist, gpu_outputs_np, light_cone_oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def to_dev(frame):
    return (frame.row_ptr.to(DEV), frame.toa.to(DEV))


def run_gpu(r3d, wl, frames, precision=0, pi_in=None, faulty=None, hist=False):
    filt = r3d.R3DFilter(wl.params(), precision, device=DEV)
    outs = []
    for n, fr in enumerate(frames):
        if hist:
            src = fr if isinstance(fr, torch.Tensor) else filt.ctx.histogram(*to_dev(fr))
        else:
            src = to_dev(fr)
        pin = None if pi_in is None else pi_in[n]
        o = filt.step(src, pi_in=pin, faulty=faulty)
        d = gpu_outputs_np(o)
        d["mean"] = filt.state.m.cpu().numpy()
        outs.append(d)
    assert filt.ctx.last_device_status() == 0
    return outs, filt


def run_oracle(wl, frames, pi_in=None, faulty=None):
    model = oracle.Model.from_params(wl.params())
    st = oracle.init_state(model)
    outs, states = [], []
    for n, fr in enumerate(frames):
        z = frame_hist(fr, wl.T)
        pin = None if pi_in is None else pi_in[n].cpu().numpy()
        fl = None if faulty is None else faulty.cpu().numpy().astype(bool)
        states.append(st)
        st, o = oracle.step(model, st, z, pi_in=pin, faulty=fl)
        outs.append(o)
    return outs, states, model


# --------------------------------------------------------------- a1
def test_histogram_bit_exact(lib):
    wl = synth.config2(frames=1)
    seqs = synth.config3(nseq=2, frames=1, res_choices=(64,), T_choices=(500, 2048))
    for w in [wl] + seqs:
        fr = w.frames[0]
        ctx = lib.Context(w.params())
        h = ctx.histogram(*to_dev(fr))
        assert ctx.last_device_status() == 0
        z = oracle.histogram(fr.row_ptr.numpy(), fr.toa.numpy(), w.T)
        got = h.float().cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(got, z)
        assert got.sum() == fr.nnz


def test_histogram_reports_bad_toa_and_overflow(lib):
    wl = synth.tiny_workload()
    ctx = lib.Context(wl.params())
    rp = torch.tensor([0, 2, 3], dtype=torch.int32, device=DEV)
    toa = torch.tensor([1, wl.T, 5], dtype=torch.int16, device=DEV)
    out = torch.empty((2, wl.T), dtype=torch.float16, device=DEV)
    p = wl.params()
    p["rows"], p["cols"] = 1, 2
    ctx2 = lib.Context(p)
    ctx2.histogram(rp, toa, out)
    assert ctx2.last_device_status() == -2
    assert ctx2.last_device_status() == 0  # cleared
    rp = torch.tensor([0, 2100, 2100], dtype=torch.int32, device=DEV)
    toa = torch.full((2100,), 7, dtype=torch.int16, device=DEV)
    ctx2.histogram(rp, toa, out)
    assert ctx2.last_device_status() == -3
    del ctx


# --------------------------------------------------------------- a3
def test_cost_plain_matches_oracle(lib):
    for w in (synth.tiny_workload(T=300, W=21, c=9), synth.config4(frames=1, rows=4, cols=5)):
        fr = w.frames[0] if w.hist is None else None
        ctx = lib.Context(w.params())
        hist = ctx.histogram(*to_dev(fr)) if fr is not None else w.hist[0].to(DEV).contiguous()
        ell = ctx.cost(hist).cpu().numpy()
        z = frame_hist(hist, w.T)
        ref = oracle.cost_from_histogram(z, oracle.Model.from_params(w.params()))
        np.testing.assert_allclose(ell, ref, rtol=2e-6, atol=2e-6 * ref.max())


# --------------------------------------------------------------- a1..a7
def test_single_frame_config1(lib):
    """Single frame 32x32, T=1024, photon lists, full size."""
    wl = synth.config1()
    g, _ = run_gpu(lib, wl, wl.frames)
    o, _, model = run_oracle(wl, wl.frames)
    rep = compare(g[0], o[0], label="config1")
    print(rep)


@pytest.mark.parametrize("case", ["plain", "faulty_pi"])
def test_video_teacher_forced(lib, case):
    """Every frame starts from the oracle's own state (cast to fp32), so each
    step is compared in isolation: 40x40 crop of the video workload; in the
    faulty_pi case with caller-supplied presence probabilities and 10 %
    faulty pixels (Sec. III-B)."""
    wl = synth.config2(frames=4, rows=40, cols=40)
    pi_in = faulty = None
    if case == "faulty_pi":
        g0 = torch.Generator().manual_seed(23)
        pi_in = torch.rand(len(wl.frames), wl.P, generator=g0)
        faulty = (torch.rand(wl.P, generator=g0) < 0.1).to(torch.uint8)
    o, states, model = run_oracle(wl, wl.frames, pi_in=pi_in, faulty=faulty)
    fl = None if faulty is None else faulty.numpy().astype(bool)
    ctx = lib.Context(wl.params())
    for n, fr in enumerate(wl.frames):
        st = states[n]
        prev = lib.State(*(torch.tensor(a, dtype=torch.float32, device=DEV)
                           for a in (st.m, st.v, st.pi, st.b)))
        nxt = lib.State.empty(wl.P, DEV)
        out = lib.Outputs.empty(wl.P, DEV)
        ctx.step_csr(*to_dev(fr), prev, nxt, out,
                     pi_in=None if pi_in is None else pi_in[n].to(DEV),
                     faulty=None if faulty is None else faulty.to(DEV))
        g = gpu_outputs_np(out)
        g["mean"] = nxt.m.cpu().numpy()
        z = frame_hist(fr, wl.T)
        rep = compare(g, o[n], model=model, state=st, z=z, pixels=np.arange(wl.P), faulty=fl,
                      label=f"{case} frame {n}")
        print(n, rep)
    assert ctx.last_device_status() == 0


def test_video_free_running(lib):
    """GPU and oracle each run their own chain over 5 frames (40x40 crop)."""
    wl = synth.config2(frames=5, rows=40, cols=40)
    g, _ = run_gpu(lib, wl, wl.frames)
    o, states, model = run_oracle(wl, wl.frames)
    for n in range(len(o)):
        rep = compare(g[n], o[n], mean_rel=1e-3, var_rel=1e-2, int_rel=1e-2,
                      label=f"free frame {n}")
        print(n, rep)


def test_hist_path_equals_csr_path(lib):
    """The fp16-histogram entry point gives bit-identical results to the
    photon-list entry point on the same data (fp32 precision)."""
    wl = synth.config2(frames=3, rows=24, cols=20)
    a, _ = run_gpu(lib, wl, wl.frames)
    b, _ = run_gpu(lib, wl, wl.frames, hist=True)
    for x, y in zip(a, b):
        for k in x:
            np.testing.assert_array_equal(x[k], y[k])


def test_faulty_pixels_and_detection_input(lib):
    wl = synth.config2(frames=3, rows=20, cols=24)
    g0 = torch.Generator().manual_seed(5)
    pi_in = [torch.rand(wl.P, generator=g0).to(DEV) for _ in wl.frames]
    faulty = (torch.rand(wl.P, generator=g0) < 0.1).to(torch.uint8).to(DEV)
    g, _ = run_gpu(lib, wl, wl.frames, pi_in=pi_in, faulty=faulty)
    o, states, model = run_oracle(wl, wl.frames, pi_in=pi_in, faulty=faulty)
    for n in range(len(o)):
        compare(g[n], o[n], mean_rel=1e-3, var_rel=1e-2, int_rel=1e-2, label=f"faulty {n}")


@pytest.mark.parametrize("case", ["one_pixel", "empty", "offset_grid", "w1", "ragged"])
def test_edge_cases(lib, case):
    kw = dict(rows=3, cols=5, T=96, frames=2, W=9, c=4)
    if case == "one_pixel":
        kw.update(rows=1, cols=1)
    if case == "ragged":
        kw.update(rows=7, cols=9)
    if case == "w1":
        kw.update(W=1, c=0)
    wl = synth.tiny_workload(**kw)
    if case == "w1":
        wl.irf = np.array([1.0])
    if case == "empty":
        wl.frames = [synth.CsrFrame(torch.zeros(wl.P + 1, dtype=torch.int32),
                                    torch.zeros(0, dtype=torch.int16)) for _ in wl.frames]
    if case == "offset_grid":
        wl.d_lo, wl.D, wl.d_min, wl.d_max = 10, 70, 10.0, 79.0
    g, _ = run_gpu(lib, wl, wl.frames)
    o, states, model = run_oracle(wl, wl.frames)
    for n in range(len(o)):
        compare(g[n], o[n], mean_rel=1e-3, var_rel=1e-2, int_rel=1e-2, label=f"{case} {n}")


def test_determinism_and_resume(lib):
    wl = synth.config2(frames=4, rows=16, cols=16)
    a, fa = run_gpu(lib, wl, wl.frames)
    b, _ = run_gpu(lib, wl, wl.frames)
    for x, y in zip(a, b):
        for k in x:
            np.testing.assert_array_equal(x[k], y[k])
    # resume: two frames, save the state, a fresh filter continues from it
    _, f2 = run_gpu(lib, wl, wl.frames[:2])
    saved = f2.state.clone()
    f3 = lib.R3DFilter(wl.params(), 0, device=DEV)
    f3.set_state(saved)
    for n in (2, 3):
        o = f3.step(to_dev(wl.frames[n]))
        np.testing.assert_array_equal(o.depth.cpu().numpy(), a[n]["depth"])


def test_full_size_video_sampled(lib):
    """Full 128x128 x 12-frame video prefix in the launch configuration used
    for timing; sampled pixels checked against the oracle's light cone."""
    wl = synth.config2(frames=12)
    g, _ = run_gpu(lib, wl, wl.frames)
    model = oracle.Model.from_params(wl.params())
    rng = np.random.default_rng(0)
    targets = np.sort(rng.choice(wl.P, 6, replace=False))
    targets = np.unique(np.concatenate([targets, [0, wl.P - 1, 20 * 128 + 10]]))
    ref = light_cone_oracle(model, wl.frames, targets, 11)
    sub = {k: v[targets] for k, v in g[11].items()}
    compare(sub, ref, mean_rel=1e-3, var_rel=1e-2, int_rel=1e-2, label="full-size sample")
