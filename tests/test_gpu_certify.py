"""Parity at full size, state-forced: the benchmark's configuration (256x256
pixels, T = 4096 fp16 histograms, 30 frames of the moving scene, the split
fp16 matrix-core engine, and the fp32 vector engine on three frames) and the
128x128 x 50-frame photon-list video (plain, with presence probabilities
and faulty pixels, and with a Gaussian IRF of its own for every pixel).

The GPU runs its own chain over all 30 frames (one step call per frame).
At frames 0, 1, 2, 10, 20, 28 and 29 the GPU's input state (fp32, cast to
float64) is handed to the oracle, which steps the sampled pixels of that
frame from exactly that state; so every sampled output is compared with the
oracle on identical inputs, at the stated tolerances: argmax identical
where the oracle's margin exceeds 1e-3 nats, else inside the oracle's tie
set (log posterior within 1e-3 of its maximum); posterior mean within
1e-4 * max(1, sd) bins plus half an fp32 ulp of the depth (the stored
output's own rounding: 1.2e-4 bins above depth 2048); variance 1e-3
relative; reflectivity and background
1e-3 relative; next prior presence 1e-5 absolute.

Sampled pixels per frame (about 290): the four corners, 8 random pixels on
each image edge, the two aligned 4x4 blocks with the most depth
discontinuities inside them (one on the square moving right, one on the
disk moving left) and 224 random pixels elsewhere."""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity_util import compare, frame_hist, gpu_outputs_np

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FRAMES = (0, 1, 2, 10, 20, 28, 29)


def boundary_blocks(depth: np.ndarray):
    """Top-left corners of the aligned 4x4 block with the most internal
    depth steps (> 50 bins between 4-neighbours) in the upper half (the
    square) and in the lower half (the disk)."""
    rows, cols = depth.shape
    step = np.zeros_like(depth, dtype=bool)
    step[:, 1:] |= np.abs(np.diff(depth, axis=1)) > 50
    step[1:, :] |= np.abs(np.diff(depth, axis=0)) > 50
    cnt = step.reshape(rows // 4, 4, cols // 4, 4).sum(axis=(1, 3))
    half = rows // 8
    out = []
    for lo, hi in ((0, half), (half, rows // 4)):
        sub = cnt[lo:hi]
        br, bc = np.unravel_index(np.argmax(sub), sub.shape)
        assert sub[br, bc] > 0
        out.append((4 * (br + lo), 4 * bc))
    return out


def sample_pixels(wl, n, rng):
    rows, cols = wl.rows, wl.cols
    depth = wl.depth_true[n].reshape(rows, cols).cpu().numpy().astype(np.int64)
    pix = [0, cols - 1, (rows - 1) * cols, rows * cols - 1]
    pix += list(rng.choice(cols, 8, replace=False))                        # top row
    pix += list((rows - 1) * cols + rng.choice(cols, 8, replace=False))    # bottom row
    pix += list(rng.choice(rows, 8, replace=False) * cols)                 # left column
    pix += list(rng.choice(rows, 8, replace=False) * cols + cols - 1)      # right column
    for r0, c0 in boundary_blocks(depth):
        pix += [(r0 + i) * cols + c0 + j for i in range(4) for j in range(4)]
    pix = set(int(p) for p in pix)
    while len(pix) < 290:
        pix.add(int(rng.integers(wl.P)))
    return np.array(sorted(pix))


def gpu_chain(lib, wl, prec, keep):
    """Run all frames on the GPU; return, for each frame in ``keep``, the
    input state (float64 oracle State), the outputs and the next state's
    mean (numpy)."""
    ctx = lib.Context(wl.params(), prec)
    st = [lib.State.empty(wl.P, DEV), lib.State.empty(wl.P, DEV)]
    ctx.state_init(st[0])
    out = lib.Outputs.empty(wl.P, DEV)
    saved = {}
    for n in range(wl.nframes):
        prev, nxt = st[n % 2], st[(n + 1) % 2]
        if n in keep:
            s_in = oracle.State(*(t.double().cpu().numpy() for t in (prev.m, prev.v, prev.pi, prev.b)))
        ctx.step_hist(wl.hist[n], prev, nxt, out)
        if n in keep:
            g = gpu_outputs_np(out)
            g["mean"] = nxt.m.cpu().numpy()
            saved[n] = (s_in, g)
    assert ctx.last_device_status() == 0
    return saved


@pytest.fixture(scope="module")
def workload():
    return synth.config4(device=DEV, frames=30)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,frames", [("fp16x2", FRAMES), ("fp32", (1, 10, 29))])
def test_full_size_state_forced(lib, workload, prec, frames):
    wl = workload
    model = oracle.Model.from_params(wl.params())
    saved = gpu_chain(lib, wl, prec, set(frames))
    rng = np.random.default_rng(2024)
    for n in frames:
        s_in, g = saved[n]
        pix = sample_pixels(wl, n, rng)
        z = frame_hist(wl.hist[n], wl.T, pix)
        _, ref = oracle.step(model, s_in, z, pixels=pix)
        sub = {k: v[pix] for k, v in g.items()}
        rep = compare(sub, ref, model=model, state=s_in, z=z, pixels=pix, mean_rel=1e-4,
                      var_rel=1e-3, int_rel=1e-3, label=f"{prec} frame {n}")
        print(prec, n, len(pix), rep, flush=True)


# ------------------------------------------- the photon-list video, full size
VIDEO_FRAMES = (0, 1, 2, 25, 49)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case,frames", [("plain", VIDEO_FRAMES), ("faulty_pi", (1, 25, 49))])
def test_full_size_video_state_forced(lib, case, frames):
    """The 128x128 x 50-frame photon-list video (T = 1500, CSR int16, fp32
    per-pixel step) at full size, state-forced as above: the GPU runs its own
    chain over all 50 frames; at the listed frames about 290 sampled pixels
    (corners, edges, the two 4x4 blocks with the most depth steps, random)
    are stepped by the oracle from the GPU's input state. In the faulty_pi
    case every frame has caller-supplied presence probabilities (uniform on
    [0, 1]: about half the pixels undetected) and 5 % of the pixels are
    faulty (their posterior is the prior alone, Sec. III-B)."""
    wl = synth.config2()
    model = oracle.Model.from_params(wl.params())
    keep = set(frames)
    pi_in = faulty = None
    if case == "faulty_pi":
        g0 = torch.Generator().manual_seed(31)
        pi_in = [torch.rand(wl.P, generator=g0) for _ in range(wl.nframes)]
        faulty = torch.rand(wl.P, generator=g0) < 0.05
    ctx = lib.Context(wl.params())
    st = [lib.State.empty(wl.P, DEV), lib.State.empty(wl.P, DEV)]
    ctx.state_init(st[0])
    out = lib.Outputs.empty(wl.P, DEV)
    fdev = None if faulty is None else faulty.to(torch.uint8).to(DEV)
    saved = {}
    for n, f in enumerate(wl.frames):
        prev, nxt = st[n % 2], st[(n + 1) % 2]
        if n in keep:
            s_in = oracle.State(*(t.double().cpu().numpy() for t in (prev.m, prev.v, prev.pi, prev.b)))
        ctx.step_csr(f.row_ptr.to(DEV), f.toa.to(DEV), prev, nxt, out,
                     pi_in=None if pi_in is None else pi_in[n].to(DEV), faulty=fdev)
        if n in keep:
            g = gpu_outputs_np(out)
            g["mean"] = nxt.m.cpu().numpy()
            saved[n] = (s_in, g)
    assert ctx.last_device_status() == 0
    rng = np.random.default_rng(77)
    fl = None if faulty is None else faulty.numpy()
    for n in frames:
        s_in, g = saved[n]
        pix = sample_pixels(wl, n, rng)
        z = frame_hist(wl.frames[n], wl.T, pix)
        _, ref = oracle.step(model, s_in, z, pixels=pix,
                             pi_in=None if pi_in is None else pi_in[n].double().numpy(), faulty=fl)
        sub = {k: v[pix] for k, v in g.items()}
        rep = compare(sub, ref, model=model, state=s_in, z=z, pixels=pix, mean_rel=1e-4,
                      var_rel=1e-3, int_rel=1e-3, faulty=fl, label=f"video {case} frame {n}")
        print("video", case, n, len(pix), rep, flush=True)


@pytest.mark.timeout(900)
def test_full_size_video_pirf_state_forced(lib):
    """The same video with every pixel its own Gaussian IRF (sigma uniform on
    [2.5, 3.5] bins, 31 taps; Sec. II-A), as the per-pixel-IRF entry point is
    timed: the GPU runs its chain over all 50 frames; at frames 1, 25 and 49
    the sampled pixels are stepped by the oracle from the GPU's input state
    with the same IRFs. Near ties (oracle margin <= 1e-3) may take another
    grid depth; everything else at the stated tolerances."""
    wl = synth.config2()
    model = oracle.Model.from_params(wl.params())
    rng = np.random.default_rng(5)
    irf_pix = np.stack([synth.gaussian_irf(s, wl.W, wl.c) for s in rng.uniform(2.5, 3.5, wl.P)])
    frames = (1, 25, 49)
    ctx = lib.Context(wl.params())
    st = [lib.State.empty(wl.P, DEV), lib.State.empty(wl.P, DEV)]
    ctx.state_init(st[0])
    out = lib.Outputs.empty(wl.P, DEV)
    irf_d = torch.as_tensor(irf_pix, device=DEV)
    saved = {}
    for n, f in enumerate(wl.frames):
        prev, nxt = st[n % 2], st[(n + 1) % 2]
        if n in frames:
            s_in = oracle.State(*(t.double().cpu().numpy() for t in (prev.m, prev.v, prev.pi, prev.b)))
        ctx.step_pirf((f.row_ptr.to(DEV), f.toa.to(DEV)), irf_d, prev, nxt, out)
        if n in frames:
            g = gpu_outputs_np(out)
            g["mean"] = nxt.m.cpu().numpy()
            saved[n] = (s_in, g)
    assert ctx.last_device_status() == 0
    rng = np.random.default_rng(78)
    for n in frames:
        s_in, g = saved[n]
        pix = sample_pixels(wl, n, rng)
        z = frame_hist(wl.frames[n], wl.T, pix)
        _, ref = oracle.step(model, s_in, z, pixels=pix, irf_pix=irf_pix)
        sub = {k: v[pix] for k, v in g.items()}
        rep = compare(sub, ref, mean_rel=1e-4, var_rel=1e-3, int_rel=1e-3, label=f"video pirf frame {n}")
        print("video pirf", n, len(pix), rep, flush=True)
