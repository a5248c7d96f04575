"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare them under the stated rules.

Comparison rules (see the test docstrings for where each applies):
* argmax: identical wherever the oracle's log-margin of d* over the
  runner-up exceeds ``margin``; elsewhere the GPU index must lie within
  ``margin`` of the oracle's maximum in the oracle's log pseudo-posterior;
* posterior mean: |gpu - oracle| <= mean_rel * max(1, oracle posterior sd)
  + half an fp32 ulp of the oracle's mean (the output is stored in fp32);
* variance: |gpu - oracle| <= var_rel * max(1, oracle variance);
* reflectivity / background (where the posterior means round to the same
  bin, the depth at which both sides place the IRF for the MLE):
  |gpu - oracle| <= int_rel * max(1, |oracle|);
* prior presence probability: absolute 1e-5.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle


def fp32_half_ulp(x) -> np.ndarray:
    """Half the fp32 spacing at |x|: the rounding of a result delivered in
    fp32 (1.2e-4 bins for depths in [2048, 4096))."""
    return 0.5 * np.spacing(np.abs(np.asarray(x, np.float64)).astype(np.float32)).astype(np.float64)


def frame_hist(frame, T, pixels=None):
    """Oracle-side histogram of a frame (CSR pair or fp16 [P, T] tensor)."""
    if isinstance(frame, torch.Tensor):
        if pixels is not None:
            idx = torch.as_tensor(np.asarray(pixels), dtype=torch.int64, device=frame.device)
            frame = frame.index_select(0, idx)
        return frame.float().cpu().numpy().astype(np.int64)
    if hasattr(frame, "row_ptr"):
        rp, toa = frame.row_ptr, frame.toa
    else:
        rp, toa = frame
    return oracle.histogram(rp.cpu().numpy(), toa.cpu().numpy(), T, pixels)


def gpu_outputs_np(out) -> dict:
    d = {}
    for k in ("depth", "var", "intensity", "background", "pi0_next", "argmax"):
        t = getattr(out, k)
        if t is not None:
            d[k] = t.cpu().numpy()
    return d


def oracle_log_posterior(model, state, z, pixels, faulty=None):
    """The oracle's log pseudo-posterior on the grid; a faulty pixel has no
    observation, so its posterior is the prior alone (Sec. III-B)."""
    logw, mean, var = oracle.prior_components(model, state, np.asarray(pixels))
    logf = oracle.log_prior(logw, mean, var, model.grid)
    ell = oracle.cost_from_histogram(z, model)
    if faulty is not None:
        ell[np.asarray(faulty, bool)[np.asarray(pixels)]] = 0.0
    return logf + ell


def compare(gpu: dict, ref: dict, *, model=None, state=None, z=None, pixels=None,
            margin=1e-3, mean_rel=1e-4, var_rel=1e-3, int_rel=1e-3, check_aux=True,
            gpu_mean=None, faulty=None, label=""):
    """Assert GPU outputs (numpy dict, indexed like ``ref``) match the oracle.
    Returns a small report dict."""
    am_g = np.asarray(gpu["argmax"]).astype(np.int64)
    am_o = np.asarray(ref["argmax"]).astype(np.int64)
    sure = ref["margin"] > margin
    n_bad = int(np.sum(am_g[sure] != am_o[sure]))
    assert n_bad == 0, f"{label}: {n_bad} argmax mismatches with margin > {margin}"
    near = (~sure) & (am_g != am_o)
    if np.any(near) and model is not None:
        L = oracle_log_posterior(model, state, z[near], np.asarray(pixels)[near], faulty)
        idx = am_g[near] - model.d_lo
        gap = L.max(axis=1) - L[np.arange(L.shape[0]), idx]
        assert np.all(gap <= margin), f"{label}: near-tie argmax outside the tie set"
    sd = np.sqrt(np.maximum(ref["var"], 0.0))
    mean = gpu_mean if gpu_mean is not None else gpu["mean"]
    err_m = np.abs(np.asarray(mean, np.float64) - ref["mean"])
    tol_m = mean_rel * np.maximum(1.0, sd) + fp32_half_ulp(ref["mean"])
    assert np.all(err_m <= tol_m), (
        f"{label}: mean error {np.max(err_m / tol_m):.3g}x tolerance "
        f"(worst pixel {int(np.argmax(err_m / tol_m))})")
    err_v = np.abs(np.asarray(gpu["var"], np.float64) - ref["var"])
    tol_v = var_rel * np.maximum(1.0, ref["var"])
    assert np.all(err_v <= tol_v), f"{label}: var error {np.max(err_v / tol_v):.3g}x tolerance"
    dg, do = np.asarray(gpu["depth"]), ref["depth"]
    assert np.array_equal(np.isnan(dg), np.isnan(do)), f"{label}: detection pattern differs"
    if check_aux:
        same = np.rint(np.asarray(mean, np.float64)) == ref["d_mle"]
        for k in ("intensity", "background"):
            e = np.abs(np.asarray(gpu[k], np.float64) - ref[k])[same]
            t = int_rel * np.maximum(1.0, np.abs(ref[k]))[same]
            assert np.all(e <= t), f"{label}: {k} error {np.max(e / t):.3g}x tolerance"
        e = np.abs(np.asarray(gpu["pi0_next"], np.float64) - ref["pi0_next"])
        assert np.all(e <= 1e-5), f"{label}: pi0_next error {e.max():.3g}"
    return dict(near_ties=int(np.sum(~sure)), argmax_differs=int(np.sum(am_g != am_o)),
                max_mean_err=float(err_m.max()), max_mean_ratio=float(np.max(err_m / tol_m)),
                max_var_ratio=float(np.max(err_v / tol_v)))


def light_cone_oracle(model, frames, targets, n_last, pi_in=None, faulty=None):
    """Oracle outputs for pixels ``targets`` at frame ``n_last`` (0-based),
    computing at frame k only the pixels within Chebyshev distance
    n_last - k of a target (the 3x3 prior needs one more ring per frame)."""
    targets = np.asarray(targets)
    tr, tc = np.divmod(targets, model.cols)
    rr, cc = np.divmod(np.arange(model.P), model.cols)
    st = oracle.init_state(model)
    out = None
    for k in range(n_last + 1):
        rad = n_last - k
        dist = np.min(np.maximum(np.abs(rr[:, None] - tr[None, :]),
                                 np.abs(cc[:, None] - tc[None, :])), axis=1)
        pix = np.nonzero(dist <= rad)[0]
        z = frame_hist(frames[k], model.T, pix)
        pin = None if pi_in is None else pi_in[k]
        new, o = oracle.step(model, st, z, pixels=pix, pi_in=pin, faulty=faulty)
        st = new
        out = o
    sel = np.searchsorted(out["pixels"], targets)
    return {k: (v[sel] if isinstance(v, np.ndarray) and v.shape[:1] == out["pixels"].shape else v)
            for k, v in out.items()}
