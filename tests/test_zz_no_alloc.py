"""GPU test of the allocation-free batch entry point (r3d_batch_run_noalloc)
against the allocating one (r3d_batch_create + r3d_batch_launch): two calls
in a row, the second on a smaller batch, each bit-identical to a fresh
batch object over the same inputs; oversized tables are rejected with
R3D_ETOOBIG before anything runs; device errors land in the first
sequence's context."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KEYS = ("depth", "var", "intensity", "background", "pi0_next", "argmax")


def dev_frames(wl):
    return [(f.row_ptr.to(DEV), f.toa.to(DEV)) for f in wl.frames]


def workloads(big: bool):
    """Uneven sequences (resolutions, bins, IRFs, beta and frame counts
    differ); the small batch has fewer, smaller sequences."""
    if big:
        seqs = synth.config3(nseq=4, frames=4, res_choices=(8, 16, 23),
                             T_choices=(300, 700, 1500), max_count=400)
        seqs[1].frames = seqs[1].frames[:2]
        seqs.append(synth.tiny_workload(seed=3, rows=7, cols=9, T=128, frames=5, W=9, c=4,
                                        beta=0.8))
        return seqs
    return [synth.tiny_workload(seed=5, rows=3, cols=5, T=96, frames=2, W=7, c=3),
            synth.tiny_workload(seed=6, rows=2, cols=2, T=64, frames=3, W=5, c=2)]


def sequences(lib, wls, contexts=None):
    out = []
    for i, wl in enumerate(wls):
        ctx = contexts[i] if contexts else lib.Context(wl.params())
        q = lib.Sequence.allocate(ctx, dev_frames(wl), DEV)
        q.init_state()
        out.append(q)
    return out


def snapshot(q):
    d = {k: getattr(q.out, k).cpu().numpy().copy() for k in KEYS}
    st = q.final_state
    d.update({f"state_{k}": getattr(st, k).cpu().numpy().copy() for k in ("m", "v", "pi", "b")})
    return d


def test_noalloc_matches_batch_object_twice(lib):
    for big in (True, False):
        wls = workloads(big)
        ctxs = [lib.Context(wl.params()) for wl in wls]
        ref = sequences(lib, wls, ctxs)
        b = lib.Batch(ref)
        b.launch()
        assert b.status() == 0
        b.close()
        got = sequences(lib, wls, ctxs)
        lib.batch_run_noalloc(got)
        torch.cuda.synchronize()
        assert ctxs[0].last_device_status() == 0
        for i, (r, g) in enumerate(zip(ref, got)):
            a, c = snapshot(r), snapshot(g)
            for k in a:
                assert np.array_equal(a[k], c[k], equal_nan=True), f"big={big} seq {i}: {k}"


def test_noalloc_errors_reach_first_context(lib):
    """Frame-1 items are handed out while frame 0 is still being computed, so
    a one-poll spin limit is exhausted: R3D_ETIMEDOUT in the first
    sequence's context; every wavefront still exits and the read clears it."""
    wl = synth.config3(nseq=1, frames=3, res_choices=(64,), T_choices=(2048,), max_count=200)[0]
    ctx = lib.Context(wl.params())
    q = lib.Sequence.allocate(ctx, dev_frames(wl), DEV, chunk_rows=4)
    q.init_state()
    lib.batch_run_noalloc([q], spin_limit=1)
    assert ctx.last_device_status() == -7
    assert ctx.last_device_status() == 0


def test_noalloc_rejects_oversized_tables(lib):
    """Frame pointer table beyond the 4 MiB scratch array: 2 x 270000 frame
    pointers of one 2x2 sequence (all frames the same photon list)."""
    wl = synth.tiny_workload(seed=7, rows=2, cols=2, T=64, frames=1, W=5, c=2)
    ctx = lib.Context(wl.params())
    fr = dev_frames(wl)[0]
    n = 270000
    st = (lib.State.empty(wl.P, DEV), lib.State.empty(wl.P, DEV))
    out = lib.Outputs.empty(wl.P, DEV)  # never written: the call is rejected first
    q = lib.Sequence(ctx, [fr] * n, st, out)
    with pytest.raises(lib.R3DError) as e:
        lib.batch_run_noalloc([q])
    assert e.value.status == -8
    # a valid call afterwards still works
    wls = workloads(False)
    seqs = sequences(lib, wls)
    lib.batch_run_noalloc(seqs)
    assert seqs[0].ctx.last_device_status() == 0
