"""Synthetic scenes shaped like the paper's workloads (Sec. II-D, IV).

Every draw is seeded (``torch.Generator``) and happens on the device the
caller names, so that the large histogram workloads can be drawn directly in
GPU memory. Conventions shared with the consumers:

* pixel index p = row * cols + col (row-major);
* a photon time of arrival (ToA) is an integer bin in [0, T);
* the IRF is a pmf over W taps and a surface at depth d puts tap j into bin
  t = d - c + j (c = index of the IRF maximum, Sec. II-D);
* signal photons that fall outside [0, T) are dropped (outside the gate).

Photon lists are stored per pixel and frame as CSR: ``row_ptr`` int32[P+1]
and ``toa`` int16[nnz]. ToAs are *not* sorted inside a pixel.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclass
class CsrFrame:
    row_ptr: torch.Tensor  # int32 [P+1]
    toa: torch.Tensor      # int16 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.toa.numel())


@dataclass
class Workload:
    name: str
    rows: int
    cols: int
    T: int
    irf: np.ndarray          # float64 [W], sums to 1
    c: int                   # tap of the IRF maximum
    beta: float
    sigma_rw2: float
    nu: np.ndarray           # float64 [9], 3x3 row-major, centre nu[4]
    d_lo: int
    D: int
    d_min: float
    d_max: float
    frames: List[CsrFrame] = field(default_factory=list)   # photon lists
    hist: Optional[torch.Tensor] = None                     # fp16 [N, P, T]
    depth_true: Optional[torch.Tensor] = None               # int32 [N, P]
    irf_sigma: Optional[float] = None

    @property
    def P(self) -> int:
        return self.rows * self.cols

    @property
    def W(self) -> int:
        return int(self.irf.shape[0])

    @property
    def nframes(self) -> int:
        if self.hist is not None:
            return int(self.hist.shape[0])
        return len(self.frames)

    def params(self) -> dict:
        """Model parameters as plain Python values (shared by both sides)."""
        return dict(rows=self.rows, cols=self.cols, T=self.T, d_lo=self.d_lo,
                    D=self.D, d_min=self.d_min, d_max=self.d_max,
                    beta=self.beta, irf=self.irf.copy(), c=self.c,
                    nu=self.nu.copy(), sigma_rw2=self.sigma_rw2)


# --------------------------------------------------------------------------
# instrument response
# --------------------------------------------------------------------------
def gaussian_irf(sigma: float, W: int, c: int) -> np.ndarray:
    """Bin-integrated Gaussian pulse (Sec. II-A, the integral below the
    discrete Poisson model), peak at tap c, renormalised to sum 1 over the W
    taps (Sec. II-D uses IRFs with unit integral)."""
    j = np.arange(W, dtype=np.float64)
    hi = np.array([math.erf((x - c + 0.5) / (sigma * math.sqrt(2.0))) for x in j])
    lo = np.array([math.erf((x - c - 0.5) / (sigma * math.sqrt(2.0))) for x in j])
    pmf = 0.5 * (hi - lo)
    return pmf / pmf.sum()


def default_nu() -> np.ndarray:
    """3x3 mixture weights: centre 0.5, the 8 others share the rest
    (Sec. III-A weights with M = 9 and nu0 = 0.5)."""
    nu = np.full(9, 0.5 / 8.0)
    nu[4] = 0.5
    return nu


def cross_nu(nu0: float = 0.5) -> np.ndarray:
    """4-neighbour cross (M = 5) written as a 3x3 stencil with zero corners,
    as used in the paper's experiments (Sec. IV)."""
    nu = np.zeros(9)
    nu[[1, 3, 5, 7]] = (1.0 - nu0) / 4.0
    nu[4] = nu0
    return nu


# --------------------------------------------------------------------------
# photon lists
# --------------------------------------------------------------------------
def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def csr_frame_from_counts(n_sig: torch.Tensor, n_bg: torch.Tensor,
                          depth: torch.Tensor, irf: np.ndarray, c: int, T: int,
                          g: torch.Generator) -> CsrFrame:
    """Draw one frame of photon ToAs given per-pixel signal / background
    counts. Signal ToA = depth - c + j with j ~ irf; background ToA uniform on
    {0..T-1}; signal ToAs outside [0, T) are dropped."""
    device = n_sig.device
    P = n_sig.numel()
    n = (n_sig + n_bg).to(torch.int64)
    start = torch.zeros(P + 1, dtype=torch.int64, device=device)
    start[1:] = torch.cumsum(n, 0)
    N = int(start[-1].item())
    if N == 0:
        return CsrFrame(torch.zeros(P + 1, dtype=torch.int32, device=device),
                        torch.zeros(0, dtype=torch.int16, device=device))
    pix = torch.repeat_interleave(torch.arange(P, device=device), n)
    within = torch.arange(N, device=device) - start[pix]
    is_sig = within < n_sig.to(torch.int64)[pix]
    cdf = torch.as_tensor(np.cumsum(irf), dtype=torch.float64, device=device)
    u = torch.rand(N, generator=g, device=device, dtype=torch.float64)
    taps = torch.searchsorted(cdf, u * cdf[-1]).clamp_(max=len(irf) - 1)
    bg = torch.randint(0, T, (N,), generator=g, device=device)
    t = torch.where(is_sig, depth.to(torch.int64)[pix] - c + taps, bg)
    keep = (t >= 0) & (t < T)
    pix = pix[keep]
    t = t[keep]
    counts = torch.bincount(pix, minlength=P)
    row_ptr = torch.zeros(P + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return CsrFrame(row_ptr.to(torch.int32), t.to(torch.int16))


def random_csr(P: int, T: int, mean_count: float, seed: int, device="cpu",
               empty_frac: float = 0.0) -> CsrFrame:
    """Uniform-background-only photon lists (for tests of histogramming)."""
    g = _gen(seed, device)
    n = torch.poisson(torch.full((P,), float(mean_count), device=device), generator=g)
    if empty_frac > 0:
        n = torch.where(torch.rand(P, generator=g, device=device) < empty_frac,
                        torch.zeros_like(n), n)
    z = torch.zeros(P, device=device)
    return csr_frame_from_counts(z, n, torch.zeros(P, device=device),
                                 np.ones(1), 0, T, g)


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
def _base(name, rows, cols, T, sigma, W, c, beta, nu=None, sigma_rw2=3.0):
    irf = gaussian_irf(sigma, W, c)
    return Workload(name=name, rows=rows, cols=cols, T=T, irf=irf, c=c,
                    beta=beta, sigma_rw2=sigma_rw2,
                    nu=default_nu() if nu is None else nu,
                    d_lo=0, D=T, d_min=0.0, d_max=float(T - 1), irf_sigma=sigma)


def config1(seed: int = 0, device="cpu") -> Workload:
    """Single frame, 32x32, T=1024, Gaussian IRF sigma=4 bins (W=41, c=20).
    Three fronto-parallel planes at depth bins 200/500/800 in column bands
    [0,11) / [11,22) / [22,32); reflectivity U(0.2,1); signal
    Poisson(5*refl), background Poisson(20) uniform; beta=0.2."""
    wl = _base("single-frame 32x32 T=1024", 32, 32, 1024, 4.0, 41, 20, 0.2)
    g = _gen(seed, device)
    P = wl.P
    col = torch.arange(P, device=device) % wl.cols
    depth = torch.where(col < 11, 200, torch.where(col < 22, 500, 800)).to(torch.int32)
    refl = 0.2 + 0.8 * torch.rand(P, generator=g, device=device, dtype=torch.float64)
    n_sig = torch.poisson((5.0 * refl).float(), generator=g)
    n_bg = torch.poisson(torch.full((P,), 20.0, device=device), generator=g)
    wl.frames = [csr_frame_from_counts(n_sig, n_bg, depth, wl.irf, wl.c, wl.T, g)]
    wl.depth_true = depth[None].clone()
    return wl


def _moving_scene_depth(rows, cols, n, scale=1):
    """Planar background + a square moving right + a disk moving left; the
    nearer surface wins. Sizes and depths scale with ``scale``."""
    r = torch.arange(rows)[:, None].expand(rows, cols)
    cc = torch.arange(cols)[None, :].expand(rows, cols)
    depth = torch.full((rows, cols), 1200 * scale, dtype=torch.int32)
    # object A: 24x24 square, top-left (20, 10), +1 col/frame, depth 300+2n
    a0r, a0c, asz = 20 * scale, 10 * scale + n * scale, 24 * scale
    in_a = (r >= a0r) & (r < a0r + asz) & (cc >= a0c) & (cc < a0c + asz)
    da = (300 + 2 * n) * scale
    # object B: disk radius 16 centred (90, 100), -1 col/frame, depth 800-2n
    bc_r, bc_c, rad = 90 * scale, 100 * scale - n * scale, 16 * scale
    in_b = (r - bc_r) ** 2 + (cc - bc_c) ** 2 <= rad * rad
    db = (800 - 2 * n) * scale
    depth = torch.where(in_b, torch.minimum(depth, torch.tensor(db, dtype=torch.int32)), depth)
    depth = torch.where(in_a, torch.minimum(depth, torch.tensor(da, dtype=torch.int32)), depth)
    return depth.reshape(-1)


def config2(seed: int = 0, device="cpu", frames: int = 50, rows: int = 128,
            cols: int = 128) -> Workload:
    """Video, 128x128 x 50 frames, T=1500, IRF sigma=3 (W=31, c=15): planar
    background at 1200, a 24x24 square (depth 300+2n, +1 col/frame) and a
    radius-16 disk (depth 800-2n, -1 col/frame). Signal Poisson(3),
    background Poisson(30) (SBR 0.1), CSR int16 ToAs, beta=0.3."""
    wl = _base(f"video {rows}x{cols}x{frames} T=1500 CSR", rows, cols, 1500,
               3.0, 31, 15, 0.3)
    g = _gen(seed, device)
    P = wl.P
    out, truth = [], []
    for n in range(frames):
        depth = _moving_scene_depth(128, 128, n)[: 128 * 128].reshape(128, 128)
        depth = depth[:rows, :cols].reshape(-1).to(device)
        n_sig = torch.poisson(torch.full((P,), 3.0, device=device), generator=g)
        n_bg = torch.poisson(torch.full((P,), 30.0, device=device), generator=g)
        out.append(csr_frame_from_counts(n_sig, n_bg, depth, wl.irf, wl.c, wl.T, g))
        truth.append(depth)
    wl.frames = out
    wl.depth_true = torch.stack(truth)
    return wl


def config3(seed: int = 0, device="cpu", nseq: int = 64, frames: int = 10,
            res_choices=(32, 64, 128, 256), T_choices=(500, 1024, 2048, 4000),
            max_count: int = 2000) -> List[Workload]:
    """Batched uneven workload: ``nseq`` independent sequences of ``frames``
    frames, resolution and T drawn uniformly from the given sets. Per-pixel
    photon count min(max_count, round(LogNormal(ln 20, 1.49))), zero with
    probability 0.05; each photon is signal with probability 0.1, at a plane
    depth U(0.2T, 0.8T) or, inside a square of side res/4 moving 1 px/frame,
    at the plane depth - 0.1T. IRF sigma=4 (W=41, c=20), beta=0.4."""
    g = _gen(seed, device)
    gc = _gen(seed + 7919, "cpu")
    seqs = []
    for s in range(nseq):
        res = int(res_choices[int(torch.randint(len(res_choices), (1,), generator=gc))])
        T = int(T_choices[int(torch.randint(len(T_choices), (1,), generator=gc))])
        plane = int(0.2 * T + 0.6 * T * float(torch.rand(1, generator=gc)))
        wl = _base(f"seq{s} {res}x{res} T={T}", res, res, T, 4.0, 41, 20, 0.4)
        P = wl.P
        r = torch.arange(P, device=device) // res
        cc = torch.arange(P, device=device) % res
        side = max(1, res // 4)
        frames_out, truth = [], []
        for n in range(frames):
            c0 = res // 8 + n
            in_sq = (r >= res // 4) & (r < res // 4 + side) & (cc >= c0) & (cc < c0 + side)
            depth = torch.where(in_sq, plane - int(0.1 * T), plane).to(torch.int32)
            k = torch.exp(math.log(20.0) + 1.49 * torch.randn(P, generator=g, device=device))
            k = torch.clamp(torch.round(k), max=max_count)
            k = torch.where(torch.rand(P, generator=g, device=device) < 0.05,
                            torch.zeros_like(k), k)
            n_sig = torch.binomial(k, torch.full_like(k, 0.1), generator=g)
            frames_out.append(csr_frame_from_counts(n_sig, k - n_sig, depth, wl.irf,
                                                    wl.c, T, g))
            truth.append(depth)
        wl.frames = frames_out
        wl.depth_true = torch.stack(truth)
        seqs.append(wl)
    return seqs


def config4(seed: int = 0, device="cpu", frames: int = 30, rows: int = 256,
            cols: int = 256, T: int = 4096) -> Workload:
    """Histogram / matrix-core precision path: 256x256 x 30 frames, T=4096,
    per-pixel histograms in fp16 drawn bin by bin from the Poisson background
    model (Sec. II-A): z_t ~ Poisson(50 * irf[t-d+c] + 400/T), IRF sigma=6
    with W=64 taps (c=32), beta=0.5. Scene: the video layout scaled x2
    (plane 2400, square 600+4n, disk 1600-4n, moving 2 px/frame)."""
    wl = _base(f"hist {rows}x{cols}x{frames} T={T} fp16", rows, cols, T, 6.0, 64, 32, 0.5)
    g = _gen(seed, device)
    P = wl.P
    irf_t = torch.as_tensor(wl.irf, dtype=torch.float32, device=device)
    taps = torch.arange(wl.W, device=device)
    hist = torch.empty((frames, P, T), dtype=torch.float16, device=device)
    truth = []
    for n in range(frames):
        depth = _moving_scene_depth(256, 256, n, scale=2)
        depth = depth.reshape(256, 256)[:rows, :cols].reshape(-1).to(device)
        depth = torch.clamp(depth, 0, T - 1).to(torch.int32)
        rate = torch.full((P, T), 400.0 / T, device=device)
        idx = depth.to(torch.int64)[:, None] - wl.c + taps[None, :]
        ok = (idx >= 0) & (idx < T)
        rate.scatter_add_(1, idx.clamp(0, T - 1), torch.where(ok, 50.0 * irf_t[None, :], 0.0))
        hist[n] = torch.poisson(rate, generator=g).to(torch.float16)
        del rate
        truth.append(depth)
    wl.hist = hist
    wl.depth_true = torch.stack(truth)
    return wl


def config5(seed: int = 0, device="cpu", frames: int = 20, rows: int = 128,
            cols: int = 128) -> Workload:
    """Differentiable filter: moving plane d(x, y, n) = 400 + x + 2n on a
    128x128 x 20 sequence, T=1024, IRF sigma=4 (W=41, c=20); signal
    Poisson(10), background Poisson(30); beta=0.3, sigma_rw2=3, 3x3 weights
    centre 0.5, others 1/16."""
    wl = _base(f"adjoint {rows}x{cols}x{frames} T=1024", rows, cols, 1024, 4.0,
               41, 20, 0.3)
    g = _gen(seed, device)
    P = wl.P
    x = (torch.arange(P, device=device) % cols)
    out, truth = [], []
    for n in range(frames):
        depth = (400 + x + 2 * n).to(torch.int32)
        n_sig = torch.poisson(torch.full((P,), 10.0, device=device), generator=g)
        n_bg = torch.poisson(torch.full((P,), 30.0, device=device), generator=g)
        out.append(csr_frame_from_counts(n_sig, n_bg, depth, wl.irf, wl.c, wl.T, g))
        truth.append(depth)
    wl.frames = out
    wl.depth_true = torch.stack(truth)
    return wl


def tiny_workload(seed: int = 0, rows: int = 4, cols: int = 5, T: int = 64,
                  frames: int = 3, sigma: float = 2.0, W: int = 9, c: int = 4,
                  beta: float = 0.4, n_sig: float = 6.0, n_bg: float = 4.0,
                  device="cpu") -> Workload:
    """Small moving-plane sequence for fast tests (several tiles of work but
    seconds of oracle time)."""
    wl = _base(f"tiny {rows}x{cols}x{frames} T={T}", rows, cols, T, sigma, W, c, beta)
    g = _gen(seed, device)
    P = wl.P
    x = torch.arange(P, device=device) % cols
    out, truth = [], []
    for n in range(frames):
        depth = (T // 3 + x + n).to(torch.int32)
        s = torch.poisson(torch.full((P,), float(n_sig), device=device), generator=g)
        b = torch.poisson(torch.full((P,), float(n_bg), device=device), generator=g)
        out.append(csr_frame_from_counts(s, b, depth, wl.irf, wl.c, wl.T, g))
        truth.append(depth)
    wl.frames = out
    wl.depth_true = torch.stack(truth)
    return wl
