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
    if precision != "fp16x2" or not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    if sources_sha(KERNEL_SRCS) != rec["kernel_src_sha"]:
        return None
    # one launch per frame: frame 0 (flat initial prior), frame 1 (the prior
    # left by frame 0), then F - 2 steady launches
    if frames < 3:
        return None
    total = (rec["frame0_launch_bytes"] + rec["frame1_launch_bytes"]
             + (frames - 2) * rec["steady_launch_bytes"])
    return round(total / frames)


COUNTER_FILE = os.path.join(ROOT, "profiles", "counters_valu_lds.json")
COUNTER_SRCS = ["paper_2004_09211_amd/csrc/k_tile.hip", "paper_2004_09211_amd/csrc/k_plain.hip",
                "paper_2004_09211_amd/csrc/k_batch.hip", "paper_2004_09211_amd/csrc/k_adjoint.hip",
                "paper_2004_09211_amd/csrc/r3d_device.hpp", "paper_2004_09211_amd/csrc/r3d_pixel.hpp",
                "paper_2004_09211_amd/csrc/r3d_tile.hpp", "paper_2004_09211_amd/build.py"]


def sources_sha(srcs) -> str:
    import hashlib
    return hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read() for s in srcs)).hexdigest()[:16]


def recorded_counters(kernel: str):
    """The committed rocprofv3 counter record of ``kernel`` (VALU issue
    fraction and LDS figures per launch), if it was taken on the kernel
    sources as they are now (else None)."""
    if not os.path.exists(COUNTER_FILE):
        return None
    rec = json.load(open(COUNTER_FILE))
    if rec.get("kernel_src_sha") != sources_sha(COUNTER_SRCS):
        return None
    return rec["kernels"].get(kernel)


def counter_probe():
    """Counter driver: a few launches of every measured kernel on its
    workload (split-fp16 tile step, 3 frames of the 256x256x4096 histograms;
    the fp32 vector form, 1 frame; the photon-list video, 5 frames; one pass
    of the uneven batch with a fixed launch shape; one gradient pass)."""
    import torch
    import synth
    from paper_2004_09211_amd import r3d
    r3d.load()
    dev = torch.device("cuda:0")
    wl = synth.config4(seed=0, device=dev, frames=3)
    for prec, nf in (("fp16x2", 3), ("fp32", 1)):
        ctx = r3d.Context(wl.params(), prec)
        st = [r3d.State.empty(wl.P, dev), r3d.State.empty(wl.P, dev)]
        out = r3d.Outputs.empty(nf * wl.P, dev)
        ctx.state_init(st[0])
        ctx.run_hist([wl.hist[n] for n in range(nf)], st, out)
        torch.cuda.synchronize()
        assert ctx.last_device_status() == 0
    del wl
    wv = synth.config2(seed=0, device=dev, frames=5)
    ctx = r3d.Context(wv.params())
    st = [r3d.State.empty(wv.P, dev), r3d.State.empty(wv.P, dev)]
    out = r3d.Outputs.empty(wv.P, dev)
    ctx.state_init(st[0])
    for n, f in enumerate(wv.frames):
        ctx.step_csr(f.row_ptr, f.toa, st[n % 2], st[(n + 1) % 2], out)
    torch.cuda.synchronize()
    assert ctx.last_device_status() == 0
    wls = synth.config3(seed=0, device=dev)
    seqs = [r3d.Sequence.allocate(r3d.Context(w.params()), [(f.row_ptr, f.toa) for f in w.frames], dev)
            for w in wls]
    for q in seqs:
        q.init_state()
    batch = r3d.Batch(seqs, blocks=0)
    batch.launch()
    assert batch.status() == 0
    batch.close()
    wg = synth.config5(seed=0, device=dev)
    frames = r3d.Frames([(f.row_ptr, f.toa) for f in wg.frames])
    ctx = r3d.Context(wg.params())
    N, P, E = len(wg.frames), wg.P, 5
    init = r3d.State.empty(P, dev)
    ctx.state_init(init)
    ws = torch.empty(ctx.grad_workspace_size(N, E), dtype=torch.uint8, device=dev)
    mean = torch.empty(N * P, device=dev)
    var = torch.empty(N * P, device=dev)
    grad = torch.empty(11 + wg.W, dtype=torch.float64, device=dev)
    ctx.filter_forward(frames, E, init, mean, var, ws)
    gm = (2.0 / (N * P)) * (mean - wg.depth_true.reshape(-1).float())
    ctx.filter_backward(frames, E, gm, None, ws, grad)
    torch.cuda.synchronize()
    assert ctx.last_device_status() == 0
    print("counter probe done", flush=True)


def sequence_probe(frames: int = 20):
    """Counter driver for the steady frames: one sequence call of the
    split-fp16 tile step over the first ``frames`` frames of the
    256x256x4096 histograms (one launch per frame, each counted on its own)."""
    import torch
    import synth
    from paper_2004_09211_amd import r3d
    r3d.load()
    dev = torch.device("cuda:0")
    wl = synth.config4(seed=0, device=dev, frames=frames)
    ctx = r3d.Context(wl.params(), "fp16x2")
    st = [r3d.State.empty(wl.P, dev), r3d.State.empty(wl.P, dev)]
    out = r3d.Outputs.empty(frames * wl.P, dev)
    ctx.state_init(st[0])
    ctx.run_hist([wl.hist[n] for n in range(frames)], st, out)
    torch.cuda.synchronize()
    assert ctx.last_device_status() == 0
    print("sequence probe done", flush=True)


COUNTER_KERNELS = {"k_tile_step<2,3>": "r3d::k_tile_step<2, 3>", "k_tile_step<0,3>": "r3d::k_tile_step<0, 3>",
                   "k_step_plain": "r3d::k_step_plain<false>", "k_batch": "r3d::k_batch(",
                   "k_adjoint": "k_adjoint(r3d::DevModel"}


def record_counters(pmc_dirs, command: str, out_path: str = ""):
    """Write profiles/counters_valu_lds.json from rocprofv3 --pmc runs (each
    with --kernel-trace) of ``--counter-probe``, one directory per counter
    pass: per kernel, the mean per launch of each counter and of the traced
    duration. ``valu_busy_frac`` is rocprofv3's VALUBusy (the share of the
    GPU's active cycles in which the compute units' vector ALUs execute)."""
    import csv
    import glob
    out = {}
    for pmc_dir in pmc_dirs:
        cc = glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)
        kt = glob.glob(os.path.join(pmc_dir, "**", "*kernel_trace.csv"), recursive=True)
        if not cc or not kt:
            raise SystemExit(f"no counter_collection / kernel_trace CSV under {pmc_dir}")
        dur = {}
        for r in csv.DictReader(open(kt[0])):
            dur[r["Correlation_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        per = {}
        for r in csv.DictReader(open(cc[0])):
            key = next((k for k, v in COUNTER_KERNELS.items() if v in r["Kernel_Name"]), None)
            if key is None:
                continue
            d = per.setdefault(key, {"launches": {}, "counters": {}})
            d["launches"][r["Correlation_Id"]] = dur.get(r["Correlation_Id"])
            d["counters"].setdefault(r["Counter_Name"], {})
            d["counters"][r["Counter_Name"]][r["Correlation_Id"]] = (
                d["counters"][r["Counter_Name"]].get(r["Correlation_Id"], 0.0) + float(r["Counter_Value"]))
        for key, d in per.items():
            ids = [i for i, t in d["launches"].items() if t is not None]
            if not ids:
                continue
            rec = out.setdefault(key, {})
            rec.setdefault("launches", len(ids))
            rec.setdefault("duration_us", round(sum(d["launches"][i] for i in ids) / len(ids), 2))
            for name, vals in sorted(d["counters"].items()):
                rec[name] = round(sum(vals.get(i, 0.0) for i in ids) / len(ids), 4)
            if "VALUBusy" in rec:
                rec["valu_busy_frac"] = round(rec["VALUBusy"] / 100.0, 4)
    rec = {"kernel_src_sha": sources_sha(COUNTER_SRCS), "command": command, "kernels": out}
    json.dump(rec, open(out_path or COUNTER_FILE, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def record_traffic(fetch_dir: str, write_dir: str, command: str, out_path: str = ""):
    """Write the HBM traffic record of the split-fp16 tile step from two
    rocprofv3 --pmc runs of --traffic-probe (FETCH_SIZE, then WRITE_SIZE):
    each counter is scaled by what it reads for the probe's elementwise
    kernel over 512 MiB (which reads and writes 524288 KiB)."""
    import csv
    import glob

    def per_dispatch(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit(f"no counter_collection CSV under {d}")
        tile, calib = {}, {}
        for r in csv.DictReader(open(f[0])):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if "r3d::k_tile_step<2, 3>" in r["Kernel_Name"]:
                tile[int(r["Correlation_Id"])] = tile.get(int(r["Correlation_Id"]), 0.0) + v
            elif "neg" in r["Kernel_Name"]:  # torch.neg over 512 MiB
                calib[int(r["Correlation_Id"])] = calib.get(int(r["Correlation_Id"]), 0.0) + v
        if len(tile) != 4 or len(calib) != 1:
            raise SystemExit(f"{counter}: {len(tile)} tile launches, {len(calib)} calibration kernels")
        return [tile[k] for k in sorted(tile)], next(iter(calib.values()))

    fetch, fcal = per_dispatch(fetch_dir, "FETCH_SIZE")
    write, wcal = per_dispatch(write_dir, "WRITE_SIZE")
    fs, ws = 524288.0 / fcal, 524288.0 / wcal
    byts = [1024.0 * (f * fs + w * ws) for f, w in zip(fetch, write)]
    steady = (byts[2] + byts[3]) / 2
    rec = {"kernel": "k_tile_step<2,3> (split fp16 matrix cores, W=64)",
           "workload": "hist 256x256 T=4096 fp16, sequence call, one launch per frame",
           "kernel_src_sha": sources_sha(KERNEL_SRCS), "command": command,
           "fetch_kib": [round(x, 1) for x in fetch], "write_kib": [round(x, 1) for x in write],
           "fetch_calibration_kib": round(fcal, 1), "write_calibration_kib": round(wcal, 1),
           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
           "frame0_launch_bytes": round(byts[0]), "frame1_launch_bytes": round(byts[1]),
           "steady_launch_bytes": round(steady),
           "avg_bytes_per_launch_30": round((byts[0] + byts[1] + 28 * steady) / 30)}
    json.dump(rec, open(out_path or TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def summarize_trace(path: str, steps: int, warmup: int, frames: int = 30):
    """Per-launch figures of the split-fp16 tile step from a rocprofv3
    kernel-trace CSV of the default command: the first ``warmup`` sequences
    of ``frames`` launches are warm-up, the next ``steps`` are the timed
    ones. Prints the mean kernel duration, the mean launch-to-launch period
    inside the timed sequences and a per-frame table."""
    import csv
    rows = [r for r in csv.DictReader(open(path)) if r["Kernel_Name"].startswith("void r3d::k_tile_step<2, 3>")]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    t = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows]
    timed = t[warmup * frames:(warmup + steps) * frames]
    if len(timed) != steps * frames:
        raise SystemExit(f"{len(t)} launches in the trace, expected at least {(warmup + steps) * frames}")
    dur = [(e - b) / 1e3 for b, e in timed]
    per = []
    for s in range(steps):
        seq = timed[s * frames:(s + 1) * frames]
        per += [(seq[i + 1][0] - seq[i][0]) / 1e3 for i in range(frames - 1)]
    bytes_launch = algorithmic_bytes_per_pixel_frame(4096) * 65536
    md = sum(dur) / len(dur)
    mp = sum(per) / len(per)
    print(f"launches in trace {len(t)}; timed {len(timed)} ({steps} sequences of {frames})")
    print(f"mean kernel duration {md:.2f} us -> {bytes_launch / md / 1e3:.1f} GB/s, "
          f"frac {bytes_launch / md / 1e3 / HBM_PEAK_GBS:.4f}")
    print(f"mean launch-to-launch period {mp:.2f} us -> {bytes_launch / mp / 1e3:.1f} GB/s, "
          f"frac {bytes_launch / mp / 1e3 / HBM_PEAK_GBS:.4f}")
    print("frame | duration mean / min / max (us)")
    for f in range(frames):
        d = [dur[s * frames + f] for s in range(steps)]
        print(f"{f:5d} | {sum(d) / len(d):7.1f} {min(d):7.1f} {max(d):7.1f}")


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
                     tflops=tf, valu_frac=tf / FP32_VALU_PEAK_TFLOPS,
                     counters=recorded_counters("k_tile_step<0,3>"))
    # algorithmic bytes of one frame per launch
    bytes_launch = algorithmic_bytes_per_pixel_frame(T) * P
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_traffic(args.precision, F),
                kernel=f"k_tile_step (one launch per frame, {F}-frame sequence call)",
                counters=recorded_counters("k_tile_step<2,3>"),
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


def run_video(args):
    """Photon-list video: 128x128 x 50 frames, T=1500, CSR int16 ToAs
    (signal Poisson(3), background Poisson(30)), fp32 per-pixel step
    (r3d_step_csr, one launch per frame), inputs resident on the device;
    median over the repetitions of one pass over the 50 frames."""
    import torch
    import synth
    from paper_2004_09211_amd import r3d

    dev = torch.device("cuda:0")
    wl = synth.config2(seed=0, device=dev)
    ctx = r3d.Context(wl.params())
    st = [r3d.State.empty(wl.P, dev), r3d.State.empty(wl.P, dev)]
    out = r3d.Outputs.empty(wl.P, dev)
    frames = [(f.row_ptr, f.toa) for f in wl.frames]
    N = len(frames)
    times = []
    for i in range(args.video_reps + 1):
        ctx.state_init(st[0])
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for n in range(N):
            ctx.step_csr(*frames[n], st[n % 2], st[(n + 1) % 2], out)
        e1.record()
        torch.cuda.synchronize()
        if i > 0:
            times.append(e0.elapsed_time(e1))
    if ctx.last_device_status() != 0:
        raise RuntimeError("video pass reported a device error")
    ms = sorted(times)[len(times) // 2]
    photons = sum(int(f.row_ptr[-1]) for f in wl.frames)
    return dict(value=round(wl.P * N / (ms * 1e-3), 1), unit="pixel-frames/s", ms_per_pass=round(ms, 3),
                ms_per_frame=round(ms / N, 4), photons_per_frame=round(photons / N),
                valu=recorded_counters("k_step_plain"),
                workload="128x128 x 50 frames, T=1500, photon lists (CSR int16), fp32 per-pixel step")


def run_rows(args):
    """The minimum-divergence and per-pixel-IRF rows, each timed on a
    workload shaped like the paper's (events on the launch stream, median
    over repetitions, inputs resident on the device):
    * min_divergence: the prior-free argmax of the split-fp16 cost on the
      256x256 x 4096-bin histograms (frames 0-3 in turn), HBM-bound;
    * min_divergence_msl: two bands of that size (the second band with a
      sigma=4 Gaussian IRF of the same 64 taps, its counts those of the next
      frame);
    * min_divergence_gauss: the continuous Gaussian-IRF maximiser on the
      128x128 photon-list video (sigma=3 bins), one launch per frame;
    * step_pirf: the 128x128 x 50-frame photon-list video with a per-pixel
      Gaussian IRF (sigma uniform in [2.5, 3.5] bins, 31 taps), one step per
      frame."""
    import numpy as np
    import torch
    import synth
    from paper_2004_09211_amd import r3d

    dev = torch.device("cuda:0")
    reps = 5

    def timed(fn, n):
        times = []
        for i in range(reps + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for k in range(n):
                fn(k)
            e1.record()
            torch.cuda.synchronize()
            if i > 0:
                times.append(e0.elapsed_time(e1) / n)
        return sorted(times)[len(times) // 2]

    out = {}
    wl = synth.config4(seed=0, device=dev, frames=4)
    P, T = wl.P, wl.T
    ctx = r3d.Context(wl.params(), "fp16x2")
    am = torch.empty(P, dtype=torch.int32, device=dev)
    val = torch.empty(P, dtype=torch.float32, device=dev)
    ms = timed(lambda k: ctx.min_divergence(wl.hist[k % 4], am, val), 8)
    bts = P * (2 * T + 8)
    out["min_divergence"] = dict(
        ms_per_launch=round(ms, 4), value=round(P / (ms * 1e-3), 1), unit="pixels/s",
        bytes_per_launch=bts, achieved_gbs=round(bts / (ms * 1e-3) / 1e9, 1),
        frac_hbm=round(bts / (ms * 1e-3) / 8e12, 4),
        workload="256x256 pixels, T=4096 fp16 histograms, W=64, beta=0.5, split fp16")
    p2 = dict(wl.params(), irf=synth.gaussian_irf(4.0, wl.W, wl.c))
    bands = [ctx, r3d.Context(p2, "fp16x2")]
    ms = timed(lambda k: r3d.min_divergence_msl(bands, [wl.hist[k % 4], wl.hist[(k + 1) % 4]], am, val), 8)
    bts = P * (2 * 2 * T + 8)
    out["min_divergence_msl"] = dict(
        ms_per_launch=round(ms, 4), value=round(P / (ms * 1e-3), 1), unit="pixels/s",
        bytes_per_launch=bts, achieved_gbs=round(bts / (ms * 1e-3) / 1e9, 1),
        frac_hbm=round(bts / (ms * 1e-3) / 8e12, 4),
        workload="2 bands of 256x256 pixels, T=4096 fp16 histograms, 64-tap IRFs (sigma 6 and 4)")
    if ctx.last_device_status() != 0 or bands[1].last_device_status() != 0:
        raise RuntimeError("minimum-divergence leg reported a device error")
    del wl, ctx, bands
    wv = synth.config2(seed=0, device=dev)
    cv = r3d.Context(wv.params())
    frames = [(f.row_ptr, f.toa) for f in wv.frames]
    N = len(frames)
    dep = torch.empty(wv.P, dtype=torch.float32, device=dev)
    vv = torch.empty(wv.P, dtype=torch.float32, device=dev)
    ga = torch.empty(wv.P, dtype=torch.int32, device=dev)
    ms = timed(lambda k: cv.min_divergence_gauss(*frames[k % N], 3.0, dep, vv, ga), N)
    out["min_divergence_gauss"] = dict(
        ms_per_launch=round(ms, 4), value=round(wv.P / (ms * 1e-3), 1), unit="pixels/s",
        workload="128x128 photon lists (CSR int16), T=1500, Gaussian IRF sigma=3 bins, continuous depth")
    rng = np.random.default_rng(5)
    sig = rng.uniform(2.5, 3.5, wv.P)
    irf_pix = torch.as_tensor(np.stack([synth.gaussian_irf(x, wv.W, wv.c) for x in sig]), device=dev)
    st = [r3d.State.empty(wv.P, dev), r3d.State.empty(wv.P, dev)]
    o = r3d.Outputs.empty(wv.P, dev)
    cv.state_init(st[0])
    ms = timed(lambda k: cv.step_pirf(frames[k % N], irf_pix, st[k % 2], st[(k + 1) % 2], o), N)
    out["step_pirf"] = dict(
        ms_per_frame=round(ms, 4), value=round(wv.P / (ms * 1e-3), 1), unit="pixel-frames/s",
        workload="128x128 x 50 frames, T=1500, photon lists, per-pixel Gaussian IRFs (sigma 2.5..3.5, 31 taps)")
    if cv.last_device_status() != 0:
        raise RuntimeError("per-pixel-IRF leg reported a device error")
    return out


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
                valu=recorded_counters("k_batch"),
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
                valu=recorded_counters("k_adjoint"),
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
                    kind="oracle", host_cpus=os.cpu_count(),
                    host_cpus_usable=len(os.sched_getaffinity(0)),
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
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
    ap.add_argument("--counter-probe", action="store_true")
    ap.add_argument("--sequence-probe", action="store_true",
                    help="20 frames of the tile step's sequence call, for per-launch counters")
    ap.add_argument("--summarize-trace", default="",
                    help="kernel-trace CSV of a rocprofv3 run of this script: print the tile "
                         "step's per-launch figures over the timed sequences and exit")
    ap.add_argument("--record-counters", nargs="*", default=None,
                    help="output directory of a rocprofv3 --pmc --kernel-trace run of "
                         "--counter-probe: write the counter record under profiles/ and exit")
    ap.add_argument("--record-command", default="")
    ap.add_argument("--record-out", default="", help="where the record goes (default: under profiles/)")
    ap.add_argument("--record-traffic", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="output directories of the two rocprofv3 --pmc runs of --traffic-probe "
                         "(FETCH_SIZE, WRITE_SIZE): write the traffic record and exit")
    ap.add_argument("--no-video", action="store_true")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the minimum-divergence and per-pixel-IRF legs")
    ap.add_argument("--video-reps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path is measured on a single MI355X "
              "(multi-GPU sharding is a design note, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    # the oracle's workers are single-threaded processes
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    if args.record_traffic:
        record_traffic(*args.record_traffic, args.record_command, args.record_out)
        return
    if args.record_counters is not None:
        record_counters(args.record_counters, args.record_command, args.record_out)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.steps, args.warmup, args.frames)
        return
    if args.traffic_probe:
        traffic_probe()
        return
    if args.counter_probe:
        counter_probe()
        return
    if args.sequence_probe:
        sequence_probe()
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
    video = None if args.no_video else run_video(args)
    batched = None if args.no_batched else run_batched(args)
    gradient = None if args.no_grad else run_grad(args)
    rows = None if args.no_rows else run_rows(args)
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
                         counters=res["plain"]["counters"],
                         speedup=round(res["value"] / res["plain"]["value"], 3))),
        roofline=res["roofline"], accuracy=accuracy, cpu_baseline=cpu, video=video,
        batched=batched, gradient=gradient, rows=rows)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
