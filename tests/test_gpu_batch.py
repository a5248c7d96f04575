"""GPU tests of the persistent batched launch (r3d_batch_*): many uneven
sequences of photon-list frames in one graph-captured kernel.

* The batch gives bit-identical outputs and states to running every
  sequence frame by frame through r3d_step_csr (both evaluate one pixel per
  wavefront with the same arithmetic), for several row-band sizes.
* Against the FP64 oracle: free-running chains, under the rules of
  parity_util (argmax identical where the oracle margin exceeds 1e-3 nats,
  mean 1e-3 * max(1, sd), variance 1e-2, reflectivity 1e-2 relative).
* Graph replays with eager work between them reproduce the first replay.
* A one-poll spin limit is reported as R3D_ETIMEDOUT and every wavefront
  still exits; the error word is cleared by the status read.
* The full 64-sequence x 10-frame uneven workload in the configuration that
  is timed: bit-identical to the per-frame path, and sampled pixels of
  two sequences against the oracle's light cone.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity_util import compare, frame_hist, gpu_outputs_np, light_cone_oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KEYS = ("depth", "var", "intensity", "background", "pi0_next", "argmax")


def dev_frames(wl):
    return [(f.row_ptr.to(DEV), f.toa.to(DEV)) for f in wl.frames]


def small_batch():
    """Uneven sequences: resolutions, bins, IRF widths, beta and frame
    counts all differ."""
    seqs = synth.config3(nseq=4, frames=4, res_choices=(8, 16, 23), T_choices=(300, 700, 1500),
                         max_count=400)
    seqs[1].frames = seqs[1].frames[:2]
    seqs.append(synth.tiny_workload(seed=3, rows=7, cols=9, T=128, frames=5, W=9, c=4, beta=0.8))
    seqs.append(synth.tiny_workload(seed=4, rows=1, cols=1, T=64, frames=3, W=1, c=0))
    seqs[-1].irf = np.array([1.0])
    return seqs


def make_sequences(lib, wls, chunk_rows=0, extras=None):
    out = []
    for i, wl in enumerate(wls):
        ctx = lib.Context(wl.params())
        kw = (extras or {}).get(i, {})
        q = lib.Sequence.allocate(ctx, dev_frames(wl), DEV, chunk_rows=chunk_rows, **kw)
        q.init_state()
        out.append(q)
    return out


def batch_outputs(q, n):
    P = q.ctx.P
    return {k: getattr(q.out, k)[n * P:(n + 1) * P].cpu().numpy() for k in KEYS}


def sequential(lib, wl, pi_in=None, faulty=None):
    filt = lib.R3DFilter(wl.params(), 0, device=DEV)
    outs = []
    for n, fr in enumerate(dev_frames(wl)):
        pin = None if pi_in is None else pi_in[n * wl.P:(n + 1) * wl.P]
        outs.append(gpu_outputs_np(filt.step(fr, pi_in=pin, faulty=faulty)))
    assert filt.ctx.last_device_status() == 0
    return outs, filt.state


def assert_same(a: dict, b: dict, label):
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), f"{label}: {k} differs"


def assert_state_same(s, t, label):
    for k in ("m", "v", "pi", "b"):
        assert np.array_equal(getattr(s, k).cpu().numpy(), getattr(t, k).cpu().numpy(),
                              equal_nan=True), f"{label}: state {k} differs"


@pytest.mark.parametrize("chunk_rows", [0, 1, 3])
def test_batch_equals_per_frame_path(lib, chunk_rows):
    wls = small_batch()
    g0 = torch.Generator().manual_seed(11)
    P0 = wls[0].P
    pi_in = torch.rand(len(wls[0].frames) * P0, generator=g0).to(DEV)
    faulty = (torch.rand(P0, generator=g0) < 0.15).to(torch.uint8).to(DEV)
    seqs = make_sequences(lib, wls, chunk_rows, extras={0: dict(pi_in=pi_in, faulty=faulty)})
    batch = lib.Batch(seqs)
    batch.launch()
    assert batch.status() == 0
    for i, (wl, q) in enumerate(zip(wls, seqs)):
        ref, st = sequential(lib, wl, *((pi_in, faulty) if i == 0 else (None, None)))
        for n in range(len(wl.frames)):
            assert_same(batch_outputs(q, n), ref[n], f"seq {i} frame {n}")
        assert_state_same(q.final_state, st, f"seq {i}")


def test_batch_matches_oracle(lib):
    wls = small_batch()
    seqs = make_sequences(lib, wls)
    batch = lib.Batch(seqs)
    batch.launch()
    assert batch.status() == 0
    for i, (wl, q) in enumerate(zip(wls, seqs)):
        model = oracle.Model.from_params(wl.params())
        st = oracle.init_state(model)
        for n, fr in enumerate(wl.frames):
            st, o = oracle.step(model, st, frame_hist(fr, wl.T))
            g = batch_outputs(q, n)
            g["mean"] = g["depth"]  # no detection input: every pixel is detected
            compare(g, o, mean_rel=1e-3, var_rel=1e-2, int_rel=1e-2, label=f"seq {i} frame {n}")


def test_graph_replays_reproduce(lib):
    wls = small_batch()[:4]
    seqs = make_sequences(lib, wls, chunk_rows=2)
    batch = lib.Batch(seqs)
    batch.launch()
    assert batch.status() == 0
    first = [[batch_outputs(q, n) for n in range(len(q.frames))] for q in seqs]
    for rep in range(3):
        for q in seqs:  # eager work between the replays
            for t in (q.out.depth, q.out.var, q.out.argmax):
                t.zero_()
            q.init_state()
        torch.cuda.synchronize()
        batch.launch()
        assert batch.status() == 0
        for i, q in enumerate(seqs):
            for n in range(len(q.frames)):
                assert_same(batch_outputs(q, n), first[i][n], f"replay {rep} seq {i} frame {n}")


def test_spin_limit_reports_timeout(lib):
    """Frame-1 items are handed out while frame 0 is still being computed, so
    a one-poll limit is exhausted; the kernel still drains and the error word
    is cleared by the read."""
    wl = synth.config3(nseq=1, frames=3, res_choices=(64,), T_choices=(2048,), max_count=200)[0]
    seqs = make_sequences(lib, [wl], chunk_rows=4)
    batch = lib.Batch(seqs, spin_limit=1)
    batch.launch()
    assert batch.status() == lib.STATUS_CODES["R3D_ETIMEDOUT"]
    assert batch.status() == 0
    ok = lib.Batch(make_sequences(lib, [wl], chunk_rows=4))
    ok.launch()
    assert ok.status() == 0


def test_batch_rejects_unsupported(lib):
    wl = synth.tiny_workload()
    ctx16 = lib.Context(wl.params(), "fp16")
    q = lib.Sequence.allocate(ctx16, dev_frames(wl), DEV)
    with pytest.raises(lib.R3DError) as e:
        lib.Batch([q])
    assert e.value.status == lib.STATUS_CODES["R3D_EUNSUPPORTED"]
    ctx = lib.Context(wl.params())
    q = lib.Sequence.allocate(ctx, dev_frames(wl), DEV)
    q.states = (q.states[0], q.states[0])
    with pytest.raises(lib.R3DError) as e:
        lib.Batch([q])
    assert e.value.status == lib.STATUS_CODES["R3D_EINVAL"]


def test_full_uneven_workload(lib):
    """64 uneven sequences x 10 frames (resolutions 32..256, 500..4000 bins,
    log-normal photon counts), the configuration that is timed."""
    wls = synth.config3(device=DEV)
    seqs = make_sequences(lib, wls)
    batch = lib.Batch(seqs)
    batch.launch()
    assert batch.status() == 0
    for i in range(0, len(wls), 7):
        ref, st = sequential(lib, wls[i])
        for n in (0, len(wls[i].frames) - 1):
            assert_same(batch_outputs(seqs[i], n), ref[n], f"seq {i} frame {n}")
        assert_state_same(seqs[i].final_state, st, f"seq {i}")
    rng = np.random.default_rng(1)
    for i in (2, 41):
        wl = wls[i]
        model = oracle.Model.from_params(wl.params())
        targets = np.unique(np.concatenate([rng.choice(wl.P, 3, replace=False), [0, wl.P - 1]]))
        last = len(wl.frames) - 1
        ref = light_cone_oracle(model, wl.frames, targets, last)
        sub = {k: v[targets] for k, v in batch_outputs(seqs[i], last).items()}
        sub["mean"] = sub["depth"]  # no detection input: every pixel is detected
        compare(sub, ref, mean_rel=1e-3, var_rel=1e-2, int_rel=1e-2, label=f"seq {i} sample")


def test_autotuner_picks_a_shape_and_caches_it(lib, tmp_path):
    """Every candidate shape gives the same bits; the tuned one is reused
    from the cache by a second call."""
    from paper_2004_09211_amd import tune
    wls = small_batch()
    seqs = make_sequences(lib, wls)

    def reset():
        for q in seqs:
            q.init_state()

    cache = str(tmp_path / "tune.json")
    cfg = tune.tune(seqs, reset, reps=1, cache=cache)
    assert not cfg["cached"] and len(cfg["timings"]) == len(tune.candidates(1))
    again = tune.tune(seqs, reset, reps=1, cache=cache)
    assert again["cached"] and again["item_px"] == cfg["item_px"]
    reset()
    batch = lib.Batch(seqs, blocks=cfg["blocks"])
    batch.launch()
    assert batch.status() == 0
    for i, (wl, q) in enumerate(zip(wls, seqs)):
        ref, _ = sequential(lib, wl)
        for n in range(len(wl.frames)):
            assert_same(batch_outputs(q, n), ref[n], f"tuned seq {i} frame {n}")
