#!/usr/bin/env python
"""Throughput of the R3DSP hot path on one MI355X.

Workload (the metric's configuration): 256x256 pixels x 30 frames, T = 4096
timing bins, fp16 photon-count histograms (signal Poisson(50) spread by a
sigma = 6 bin IRF with 64 taps, background Poisson(400) uniform), beta = 0.5,
3x3 spatio-temporal fusion. One step = one pass of the whole per-frame path
(a1..a7: cost, prior, argmax/moments, state update, background/reflectivity,
prior presence) over the 30 frames, starting from the initial state, through
the sequence entry point r3d_run_hist (one launch of the tile kernel per
frame).
Inputs are drawn on the device before timing (15 GiB resident in HBM).

Prints one JSON line with the matrix-core form's pixel-frames/s, the plain
fp32 form's rate on the same workload, entry point, steps and warm-up (with
its FLOP rate against the fp32 vector peak), the roofline of the tile kernel
(HBM-bound: algorithmic bytes per launch over the average launch time,
measured with events on the launch stream), the accuracy of the timed run's
last frame against the FP64 CPU oracle stepped from the GPU's own input
state, and the oracle's rate on a bounded sample (64x64 x 3 frames of the
same recipe, on single-threaded worker processes forked before the GPU is
used).

``--traffic-probe`` runs 4 frames of the sequence call, then a 512 MiB
device copy, and exits: the driver of the rocprofv3 counter runs whose
results are recorded under profiles/.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pixel-frames/sec (cost+argmax+fusion) at 256×256×4096 bins; MFMA/batched vs plain"
HBM_PEAK_GBS = 8000.0
# fp32 FMAs without packing: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6


def algorithmic_bytes_per_pixel_frame(T: int) -> int:
    """fp16 histogram row + previous state (m, v, pi, b) + next state +
    six per-pixel outputs, each read or written once."""
    return 2 * T + 16 + 16 + 24


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_tile_step_fp16x2_hist256x256x4096.json")
KERNEL_SRCS = ["paper_2004_09211_amd/csrc/k_tile.hip", "paper_2004_09211_amd/csrc/r3d_device.hpp",
               "paper_2004_09211_amd/csrc/r3d_tile.hpp", "paper_2004_09211_amd/build.py"]


def measured_traffic(precision: str, frames: int):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    record, if it was taken on the kernel sources as they are now (else None)."""
    import hashlib
    if precision != "fp16x2" or not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    sha = hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read() for s in KERNEL_SRCS))
    if sha.hexdigest()[:16] != rec["kernel_src_sha"]:
        return None
    # one launch per frame: frame 0 (flat initial prior), frame 1 (the prior
    # left by frame 0), then F - 2 steady launches
    if frames < 3:
        return None
    total = (rec["frame0_launch_bytes"] + rec["frame1_launch_bytes"]
             + (frames - 2) * rec["steady_launch_bytes"])
    return round(total / frames)


def traffic_probe():
    """Counter driver: 4 frames of the sequence call on the benchmark's
    workload, then a 512 MiB device-to-device copy (an elementwise kernel
    reading and writing 512 MiB) that calibrates FETCH_SIZE / WRITE_SIZE."""
    import torch
    import synth
    from paper_2004_09211_amd import r3d
    r3d.load()
    dev = torch.device("cuda:0")
    wl = synth.config4(seed=0, device=dev, frames=4)
    ctx = r3d.Context(wl.params(), "fp16x2")
    st = [r3d.State.empty(wl.P, dev), r3d.State.empty(wl.P, dev)]
    out = r3d.Outputs.empty(4 * wl.P, dev)
    ctx.state_init(st[0])
    ctx.run_hist([wl.hist[n] for n in range(4)], st, out)
    torch.cuda.synchronize()
    src = torch.ones(512 * 2**20 // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    if ctx.last_device_status() != 0:
        raise RuntimeError("device status")
    print("traffic probe done", flush=True)


def run_gpu(args):
    import torch
    import synth
    from paper_2004_09211_amd import r3d

    if not os.path.exists(r3d.LIB_PATH):
        from paper_2004_09211_amd import build
        build.build()
    r3d.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = synth.config4(seed=0, device=dev, frames=args.frames)
    torch.cuda.synchronize()
    P, F, T = wl.P, wl.nframes, wl.T
    params = wl.params()

    def make(precision):
        ctx = r3d.Context(params, precision)
        st = [r3d.State.empty(P, dev), r3d.State.empty(P, dev)]
        out = r3d.Outputs.empty(P, dev)
        return ctx, st, out

    hists = [wl.hist[n] for n in range(F)]

    def sequence(ctx, st, out, ev=None, per_frame=False):
        ctx.state_init(st[0])
        if ev is not None:
            ev[0].record()
        if per_frame:
            # one r3d_step_hist per frame
            for n in range(F):
                ctx.step_hist(hists[n], st[n % 2], st[(n + 1) % 2], out)
        else:
            ctx.run_hist(hists, st, out)
        if ev is not None:
            ev[1].record()

    def timed(precision, steps, warmup, per_frame=False):
        ctx = r3d.Context(params, precision)
        st = [r3d.State.empty(P, dev), r3d.State.empty(P, dev)]
        out = r3d.Outputs.empty((1 if per_frame else F) * P, dev)
        for _ in range(warmup):
            sequence(ctx, st, out, per_frame=per_frame)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            sequence(ctx, st, out, evs[s], per_frame=per_frame)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        status = ctx.last_device_status()
        if status != 0:
            raise RuntimeError(f"device status {status}")
        # launches of the tile kernel per step: one per frame
        launches = F
        launch_ms = sum(a.elapsed_time(b) for a, b in evs) / (steps * launches)
        return wall, launch_ms, (ctx, st, out)

    prec = r3d.PRECISIONS[args.precision]
    wall, launch_ms, last = timed(prec, args.steps, args.warmup)
    ms_per_step = 1e3 * wall / args.steps
    value = P * F * args.steps / wall
    plain = None
    if args.plain_steps > 0 and prec != r3d.R3D_FP32:
        # the plain form (fp32 vector FMAs, no matrix cores) through the same
        # sequence call, steps and warm-up
        pw, pl, _ = timed(r3d.R3D_FP32, args.steps, args.warmup)
        flop = 2.0 * P * wl.D * wl.W  # the full correlation: one FMA per pixel, depth and tap
        tf = flop / (pl * 1e-3) / 1e12
        plain = dict(value=P * F * args.steps / pw, ms_per_step=1e3 * pw / args.steps,
                     launch_ms=pl, precision="fp32", entry="r3d_run_hist (one launch per frame)",
                     tflops=tf, valu_frac=tf / FP32_VALU_PEAK_TFLOPS)
    # algorithmic bytes of one frame per launch
    bytes_launch = algorithmic_bytes_per_pixel_frame(T) * P
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_traffic(args.precision, F),
                kernel=f"k_tile_step (one launch per frame, {F}-frame sequence call)",
                launch_ms=round(launch_ms, 5), bytes_per_launch=round(bytes_launch))
    # what the accuracy check of the timed run needs: frame F-1's histograms,
    # its input state (the sequence call leaves it in the second buffer) and
    # its outputs
    ctx, st, out = last
    tail = dict(hist=wl.hist[F - 1], state_in=st[(F - 1) % 2], state_out=st[F % 2], out=out,
                frame=F - 1)
    res = dict(value=value, ms_per_step=ms_per_step, plain=plain, roofline=roof, P=P, F=F, T=T,
               params=params, tail=tail)
    return res


def run_batched(args):
    """Uneven batch: 64 sequences x 10 frames (resolutions 32..256 squared,
    500..4000 bins, log-normal photon counts) through one persistent launch
    replayed from a captured graph, launch shape from the autotuner (tuned
    before timing); compared with the per-frame entry point launched once per
    sequence and frame on the same inputs."""
    import torch
    import synth
    from paper_2004_09211_amd import r3d, tune

    dev = torch.device("cuda:0")
    wls = synth.config3(seed=0, device=dev)
    torch.cuda.synchronize()
    seqs = [r3d.Sequence.allocate(r3d.Context(w.params()), [(f.row_ptr, f.toa) for f in w.frames],
                                  dev) for w in wls]

    def reset():
        for q in seqs:
            q.init_state()

    cfg = tune.tune(seqs, reset, reps=1, cache=args.tune_cache or None)
    batch = r3d.Batch(seqs, blocks=cfg["blocks"])
    times = []
    for i in range(args.batched_reps + 1):
        reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        batch.launch()
        e1.record()
        status = batch.status()
        if status != 0:
            raise RuntimeError(f"batch status {status}")
        if i > 0:
            times.append(e0.elapsed_time(e1))
    batch.close()
    pf = sum(w.P * len(w.frames) for w in wls)
    ms = sorted(times)[len(times) // 2]
    # per-frame launches of the same step on the same inputs
    st = [(r3d.State.empty(q.ctx.P, dev), r3d.State.empty(q.ctx.P, dev)) for q in seqs]
    outs = [r3d.Outputs.empty(q.ctx.P, dev) for q in seqs]
    pms = []
    for i in range(2):
        for q, s2 in zip(seqs, st):
            q.ctx.state_init(s2[0])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for n in range(max(len(w.frames) for w in wls)):
            for q, w, s2, o in zip(seqs, wls, st, outs):
                if n < len(w.frames):
                    q.ctx.step_csr(*q.frames[n], s2[n % 2], s2[(n + 1) % 2], o)
        e1.record()
        torch.cuda.synchronize()
        if i > 0:
            pms.append(e0.elapsed_time(e1))
    for q in seqs:
        if q.ctx.last_device_status() != 0:
            raise RuntimeError("per-frame path reported a device error")
    photons = sum(int(f.row_ptr[-1]) for w in wls for f in w.frames)
    return dict(value=round(pf / (ms * 1e-3), 1), unit="pixel-frames/s", ms_per_pass=round(ms, 3),
                pixel_frames=pf, photons=photons,
                per_frame_launches=dict(value=round(pf / (pms[0] * 1e-3), 1),
                                        ms_per_pass=round(pms[0], 3)),
                speedup_vs_per_frame=round(pms[0] / ms, 3),
                tuned={k: cfg[k] for k in ("item_px", "balanced", "blocks")},
                workload="64 uneven sequences x 10 frames (32..256 squared, T 500..4000, "
                         "log-normal photon counts, fp32 photon lists)")


def run_grad(args):
    """Differentiable filter on 128x128 x 20 frames (T=1024, moving plane):
    forward with a checkpoint every 5 frames, then the adjoint of
    loss = mean (posterior mean - true depth)^2, timed separately (median of
    the repetitions) with events on the launch stream."""
    import torch
    import synth
    from paper_2004_09211_amd import r3d

    dev = torch.device("cuda:0")
    wl = synth.config5(seed=0, device=dev)
    frames = r3d.Frames([(f.row_ptr, f.toa) for f in wl.frames])
    ctx = r3d.Context(wl.params())
    N, P, E = len(wl.frames), wl.P, 5
    init = r3d.State.empty(P, dev)
    ctx.state_init(init)
    ws = torch.empty(ctx.grad_workspace_size(N, E), dtype=torch.uint8, device=dev)
    mean = torch.empty(N * P, device=dev)
    var = torch.empty(N * P, device=dev)
    grad = torch.empty(11 + wl.W, dtype=torch.float64, device=dev)
    truth = wl.depth_true.reshape(-1).float()
    fw, bw = [], []
    for i in range(args.grad_reps + 1):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        ctx.filter_forward(frames, E, init, mean, var, ws)
        e[1].record()
        gm = (2.0 / (N * P)) * (mean - truth)
        ctx.filter_backward(frames, E, gm, None, ws, grad)
        e[2].record()
        torch.cuda.synchronize()
        if i > 0:
            fw.append(e[0].elapsed_time(e[1]))
            bw.append(e[1].elapsed_time(e[2]))
    if ctx.last_device_status() != 0:
        raise RuntimeError("gradient pass reported a device error")
    fms, bms = sorted(fw)[len(fw) // 2], sorted(bw)[len(bw) // 2]
    return dict(value=round(N * P / ((fms + bms) * 1e-3), 1), unit="pixel-frames/s",
                forward_ms=round(fms, 3), backward_ms=round(bms, 3),
                backward_over_forward=round(bms / fms, 2), ckpt_every=E,
                workload="128x128 x 20 frames, T=1024, photon lists; gradient w.r.t. beta, "
                         "IRF taps, sigma_rw2, nu[9]")


# ---------------------------------------------------------------------------
# the oracle leg: the FP64 CPU oracle timed on a bounded sample of the
# workload (cpu_baseline), and the accuracy of the timed GPU run's last frame
# against it
# ---------------------------------------------------------------------------
def _oracle_task(task):
    """One worker task: oracle.step for a chunk of pixels from a given full
    state. Returns the chunk's outputs and new state."""
    import oracle
    params, state, z, pix = task
    model = oracle.Model.from_params(params)
    new, out = oracle.step(model, oracle.State(*state), z, pixels=pix)
    return pix, tuple(a[pix] for a in (new.m, new.v, new.pi, new.b)), out


class OracleLeg:
    """A pool of CPU workers forked before the GPU is touched (each runs the
    oracle single-threaded on chunks of pixels of one frame; a frame's
    chunks all start from the same full previous state, so the chunked run
    equals the whole-frame run)."""

    def __init__(self, workers: int):
        import multiprocessing as mp
        self.workers = workers
        self.pool = mp.get_context("fork").Pool(workers)

    def close(self):
        self.pool.close()
        self.pool.join()

    def step(self, params, state, z, pix, chunk):
        import numpy as np
        tasks = [(params, state, z[i:i + chunk], pix[i:i + chunk]) for i in range(0, len(pix), chunk)]
        res = self.pool.map(_oracle_task, tasks)
        P = params["rows"] * params["cols"]
        new = [np.full(P, np.nan) for _ in range(4)]
        outs = {}
        for p, st, o in res:
            for a, b in zip(new, st):
                a[p] = b
            for k, v in o.items():
                if isinstance(v, np.ndarray) and v.shape[:1] == p.shape:
                    outs.setdefault(k, []).append(v)
        return tuple(new), {k: np.concatenate(v) for k, v in outs.items()}

    def baseline(self, rows: int, frames: int):
        """The oracle on a rows x rows crop of the workload's recipe (drawn on
        the host) for ``frames`` frames from the initial state."""
        import numpy as np
        import oracle
        import synth
        wl = synth.config4(seed=1, device="cpu", frames=frames, rows=rows, cols=rows)
        params = wl.params()
        model = oracle.Model.from_params(params)
        s0 = oracle.init_state(model)
        state = (s0.m, s0.v, s0.pi, s0.b)
        pix = np.arange(wl.P)
        zs = [wl.hist[n].float().numpy().astype(np.int64) for n in range(frames)]
        t0 = time.perf_counter()
        for n in range(frames):
            state, _ = self.step(params, state, zs[n], pix, chunk=max(1, wl.P // (4 * self.workers)))
        dt = time.perf_counter() - t0
        n = wl.P * frames
        return dict(value=round(n / dt, 2), unit="pixel-frames/s", cores=self.workers,
                    kind="oracle",
                    sample=f"{rows}x{rows} crop x {frames} frames of the same workload recipe "
                           f"(T=4096, drawn on the host; {n} pixel-frames, {dt:.1f} s on "
                           f"{self.workers} single-threaded worker processes)")

    def accuracy(self, params, tail, npix: int):
        """The timed run's last frame on ``npix`` sampled pixels (corners and
        seeded random pixels), stepped by the oracle from the GPU's own input
        state of that frame: argmax disagreements beyond the 1e-3 nat margin,
        and the largest posterior-mean and variance errors over their
        tolerances (1e-4 * max(1, sd) bins plus half an fp32 ulp of the
        depth, the stored output's own rounding; 1e-3 relative)."""
        import numpy as np
        import oracle
        P = params["rows"] * params["cols"]
        rng = np.random.default_rng(7)
        pix = np.unique(np.concatenate([[0, params["cols"] - 1, P - params["cols"], P - 1],
                                        rng.choice(P, npix - 4, replace=False)]))
        idx = __import__("torch").as_tensor(pix, device=tail["hist"].device)
        z = tail["hist"].index_select(0, idx).float().cpu().numpy().astype(np.int64)
        s_in = tuple(getattr(tail["state_in"], k).double().cpu().numpy() for k in ("m", "v", "pi", "b"))
        _, ref = self.step(params, s_in, z, pix, chunk=max(1, len(pix) // self.workers))
        f = tail["frame"]
        o = tail["out"]
        off = f * P
        am = o.argmax[off:off + P].cpu().numpy()[pix].astype(np.int64)
        mean = tail["state_out"].m.cpu().numpy()[pix].astype(np.float64)
        var = o.var[off:off + P].cpu().numpy()[pix].astype(np.float64)
        sure = ref["margin"] > 1e-3
        sd = np.sqrt(np.maximum(ref["var"], 0.0))
        same = am == ref["argmax"]
        model = oracle.Model.from_params(params)
        st = oracle.State(*s_in)
        near = (~sure) & ~same
        outside = 0
        if near.any():
            logw, mu, vv = oracle.prior_components(model, st, pix[near])
            L = oracle.log_prior(logw, mu, vv, model.grid) + oracle.cost_from_histogram(z[near], model)
            gap = L.max(axis=1) - L[np.arange(L.shape[0]), am[near] - model.d_lo]
            outside = int(np.sum(gap > 1e-3))
        return dict(frame=int(f), pixels=int(len(pix)),
                    argmax_mismatch_beyond_margin=int(np.sum(sure & ~same)),
                    argmax_outside_tie_set=outside,
                    max_mean_err_over_tol=round(float(np.max(np.abs(mean - ref["mean"]) / (
                        1e-4 * np.maximum(1.0, sd)
                        + 0.5 * np.spacing(np.abs(ref["mean"]).astype(np.float32)).astype(np.float64)))), 4),
                    max_var_err_over_tol=round(float(np.max(np.abs(var - ref["var"]) / (1e-3 * np.maximum(1.0, ref["var"])))), 4),
                    rule="oracle stepped from the GPU's input state of the frame; pass = 0, 0, <= 1, <= 1")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp16x2", choices=["fp32", "fp16", "fp16x2"])
    ap.add_argument("--frames", type=int, default=30)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=64)
    ap.add_argument("--cpu-frames", type=int, default=3)
    ap.add_argument("--cpu-workers", type=int, default=16)
    ap.add_argument("--accuracy-pixels", type=int, default=256)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-reps", type=int, default=5)
    ap.add_argument("--tune-cache", default="")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--grad-reps", type=int, default=5)
    ap.add_argument("--traffic-probe", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path is measured on a single MI355X "
              "(multi-GPU sharding is a design note, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    # the oracle's workers are single-threaded processes
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    if args.traffic_probe:
        traffic_probe()
        return
    leg = cpu = accuracy = None
    if not args.no_cpu_baseline:
        # forked before anything touches the GPU; timed before the GPU legs
        workers = max(1, min(args.cpu_workers, len(os.sched_getaffinity(0))))
        leg = OracleLeg(workers)
        cpu = leg.baseline(args.cpu_rows, args.cpu_frames)
    res = run_gpu(args)
    if leg is not None:
        accuracy = leg.accuracy(res["params"], res["tail"], args.accuracy_pixels)
        leg.close()
    res.pop("tail")
    batched = None if args.no_batched else run_batched(args)
    gradient = None if args.no_grad else run_grad(args)
    line = dict(
        metric=METRIC, value=round(res["value"], 1), unit="pixel-frames/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=round(res["ms_per_step"], 4),
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype={"fp32": "f32", "fp16": "fp16 mfma, f32 acc", "fp16x2": "fp16x2 mfma, f32 acc"}[args.precision],
        data="synthetic",
        config=dict(workload=f"hist {res['P'] // 256}x256 x {res['F']} frames, T={res['T']}, fp16 "
                             f"histograms, W=64, beta=0.5, 3x3 fusion",
                    pixels=res["P"], frames=res["F"], T=res["T"], precision=args.precision,
                    parallelism="single GPU"),
        plain_fp32=(None if res["plain"] is None else
                    dict(value=round(res["plain"]["value"], 1),
                         ms_per_step=round(res["plain"]["ms_per_step"], 3),
                         launch_ms=round(res["plain"]["launch_ms"], 4),
                         entry=res["plain"]["entry"],
                         tflops=round(res["plain"]["tflops"], 2),
                         valu_frac=round(res["plain"]["valu_frac"], 4),
                         speedup=round(res["value"] / res["plain"]["value"], 3))),
        roofline=res["roofline"], accuracy=accuracy, cpu_baseline=cpu, batched=batched,
        gradient=gradient)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
