"""ctypes binding of libr3d (include/r3d.h): argument marshalling only.

Every computation happens in the HIP library; this module converts torch
tensors to device pointers and the current torch stream to a hipStream_t.
If the library is not built, ``load()`` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_void_p, c_char_p
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libr3d.so")

R3D_FP32, R3D_FP16_MFMA, R3D_FP16X2_MFMA = 0, 1, 2
PRECISIONS = {"fp32": R3D_FP32, "fp16": R3D_FP16_MFMA, "fp16x2": R3D_FP16X2_MFMA}

STATUS = {0: "R3D_OK", -1: "R3D_EINVAL", -2: "R3D_ERANGE", -3: "R3D_EOVERFLOW",
          -4: "R3D_ENOMEM", -5: "R3D_EHIP", -6: "R3D_EUNSUPPORTED", -7: "R3D_ETIMEDOUT",
          -8: "R3D_ETOOBIG"}

STATUS_CODES = {v: k for k, v in STATUS.items()}


class Params(ctypes.Structure):
    _fields_ = [("rows", c_int32), ("cols", c_int32), ("T", c_int32),
                ("d_lo", c_int32), ("D", c_int32), ("d_min", c_double),
                ("d_max", c_double), ("beta", c_double), ("W", c_int32),
                ("c", c_int32), ("irf", POINTER(c_double)), ("nu", c_double * 9),
                ("sigma_rw2", c_double), ("precision", c_int32)]


class CState(ctypes.Structure):
    _fields_ = [("m", c_void_p), ("v", c_void_p), ("pi", c_void_p), ("b", c_void_p)]


class COut(ctypes.Structure):
    _fields_ = [("depth", c_void_p), ("var", c_void_p), ("intensity", c_void_p),
                ("background", c_void_p), ("pi0_next", c_void_p), ("argmax", c_void_p)]


class CSequence(ctypes.Structure):
    _fields_ = [("ctx", c_void_p), ("nframes", c_int32), ("row_ptr", POINTER(c_void_p)),
                ("toa", POINTER(c_void_p)), ("state", CState * 2), ("out", COut),
                ("pi_in", c_void_p), ("faulty", c_void_p), ("chunk_rows", c_int32)]


class CFrames(ctypes.Structure):
    _fields_ = [("nframes", c_int32), ("row_ptr", POINTER(c_void_p)), ("toa", POINTER(c_void_p)),
                ("pi_in", c_void_p), ("faulty", c_void_p)]


class CBatchOptions(ctypes.Structure):
    _fields_ = [("spin_limit", ctypes.c_uint32), ("blocks", c_int32)]


#: every symbol the header declares, with (restype, argtypes)
SIGNATURES = {
    "r3d_create": (c_int32, [POINTER(Params), POINTER(c_void_p)]),
    "r3d_destroy": (None, [c_void_p]),
    "r3d_state_init": (c_int32, [c_void_p, POINTER(CState), c_void_p]),
    "r3d_histogram": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "r3d_cost": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "r3d_step_csr": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               POINTER(CState), POINTER(CState), POINTER(COut), c_void_p]),
    "r3d_step_hist": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p,
                                POINTER(CState), POINTER(CState), POINTER(COut), c_void_p]),
    "r3d_run_hist": (c_int32, [c_void_p, POINTER(c_void_p), c_int32, c_void_p, c_void_p,
                               POINTER(CState), POINTER(COut), c_void_p]),
    "r3d_last_device_status": (c_int32, [c_void_p, c_void_p]),
    "r3d_batch_create": (c_int32, [POINTER(CSequence), c_int32, POINTER(CBatchOptions),
                                   POINTER(c_void_p)]),
    "r3d_batch_launch": (c_int32, [c_void_p, c_void_p]),
    "r3d_batch_status": (c_int32, [c_void_p, c_void_p]),
    "r3d_batch_destroy": (None, [c_void_p]),
    "r3d_batch_run_noalloc": (c_int32, [POINTER(CSequence), c_int32, POINTER(CBatchOptions),
                                        c_void_p]),
    "r3d_grad_workspace_size": (c_int32, [c_void_p, c_int32, c_int32, POINTER(ctypes.c_size_t)]),
    "r3d_filter_forward": (c_int32, [c_void_p, POINTER(CFrames), c_int32, POINTER(CState),
                                     c_void_p, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
    "r3d_filter_backward": (c_int32, [c_void_p, POINTER(CFrames), c_int32, c_void_p, c_void_p,
                                      c_void_p, ctypes.c_size_t, c_void_p, c_void_p]),
    "r3d_min_divergence": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "r3d_min_divergence_gauss": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p,
                                           c_void_p, c_void_p]),
    "r3d_min_divergence_msl": (c_int32, [POINTER(c_void_p), c_int32, POINTER(c_void_p), c_void_p,
                                         c_void_p, c_void_p]),
    "r3d_step_pirf": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p, POINTER(CState), POINTER(CState),
                                POINTER(COut), c_void_p]),
    "r3d_status_string": (c_char_p, [c_int32]),
}

_lib = None


class R3DError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = STATUS.get(status, str(status))
        if _lib is not None:
            msg += ": " + _lib.r3d_status_string(status).decode()
        super().__init__(f"{what}: {msg}" if what else msg)


def load(path: Optional[str] = None):
    """Load libr3d.so (built in-tree by ``build.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libr3d.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        raise R3DError(status, what)


def _ptr(t: Optional[torch.Tensor], dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return c_void_p(t.data_ptr())


def _stream(stream) -> c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


@dataclass
class State:
    m: torch.Tensor
    v: torch.Tensor
    pi: torch.Tensor
    b: torch.Tensor

    @classmethod
    def empty(cls, P: int, device="cuda"):
        return cls(*(torch.empty(P, dtype=torch.float32, device=device) for _ in range(4)))

    def c(self) -> CState:
        return CState(*(_ptr(t, torch.float32) for t in (self.m, self.v, self.pi, self.b)))

    def clone(self) -> "State":
        return State(self.m.clone(), self.v.clone(), self.pi.clone(), self.b.clone())


@dataclass
class Outputs:
    depth: Optional[torch.Tensor] = None
    var: Optional[torch.Tensor] = None
    intensity: Optional[torch.Tensor] = None
    background: Optional[torch.Tensor] = None
    pi0_next: Optional[torch.Tensor] = None
    argmax: Optional[torch.Tensor] = None

    @classmethod
    def empty(cls, P: int, device="cuda"):
        f = lambda: torch.empty(P, dtype=torch.float32, device=device)
        return cls(f(), f(), f(), f(), f(), torch.empty(P, dtype=torch.int32, device=device))

    def c(self) -> COut:
        return COut(_ptr(self.depth, torch.float32), _ptr(self.var, torch.float32),
                    _ptr(self.intensity, torch.float32), _ptr(self.background, torch.float32),
                    _ptr(self.pi0_next, torch.float32), _ptr(self.argmax, torch.int32))


def make_params(p: dict, precision=R3D_FP32):
    """Build the C parameter struct from a parameter dict; returns the struct
    and the host IRF array it points to (keep both alive during the call)."""
    irf = np.ascontiguousarray(np.asarray(p["irf"], dtype=np.float64))
    prm = Params()
    prm.rows, prm.cols, prm.T = int(p["rows"]), int(p["cols"]), int(p["T"])
    prm.d_lo, prm.D = int(p["d_lo"]), int(p["D"])
    prm.d_min, prm.d_max = float(p["d_min"]), float(p["d_max"])
    prm.beta = float(p["beta"])
    prm.W, prm.c = int(irf.shape[0]), int(p["c"])
    prm.irf = irf.ctypes.data_as(POINTER(c_double))
    for k in range(9):
        prm.nu[k] = float(p["nu"][k])
    prm.sigma_rw2 = float(p["sigma_rw2"])
    prm.precision = int(PRECISIONS.get(precision, precision))
    return prm, irf


class Context:
    """An r3d_ctx: model parameters uploaded to the current device."""

    def __init__(self, params: dict, precision=R3D_FP32):
        lib = load()
        prm, self._irf = make_params(params, precision)
        h = c_void_p()
        _check(lib.r3d_create(byref(prm), byref(h)), "r3d_create")
        self._h = h
        self.rows, self.cols = prm.rows, prm.cols
        self.P = prm.rows * prm.cols
        self.T, self.D = prm.T, prm.D
        self.precision = prm.precision

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.r3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state_init(self, st: State, stream=None):
        cs = st.c()
        _check(_lib.r3d_state_init(self._h, byref(cs), _stream(stream)), "r3d_state_init")

    def histogram(self, row_ptr, toa, out: Optional[torch.Tensor] = None, stream=None):
        if out is None:
            out = torch.empty((self.P, self.T), dtype=torch.float16, device=row_ptr.device)
        _check(_lib.r3d_histogram(self._h, _ptr(row_ptr, torch.int32), _ptr(toa, torch.int16),
                                  _ptr(out, torch.float16), _stream(stream)), "r3d_histogram")
        return out

    def cost(self, hist: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        npix = hist.shape[0]
        if out is None:
            out = torch.empty((npix, self.D), dtype=torch.float32, device=hist.device)
        _check(_lib.r3d_cost(self._h, _ptr(hist, torch.float16), npix, _ptr(out, torch.float32),
                             _stream(stream)), "r3d_cost")
        return out

    def step_csr(self, row_ptr, toa, prev: State, nxt: State, out: Outputs,
                 pi_in=None, faulty=None, stream=None):
        cp, cn, co = prev.c(), nxt.c(), out.c()
        _check(_lib.r3d_step_csr(self._h, _ptr(row_ptr, torch.int32), _ptr(toa, torch.int16),
                                 _ptr(pi_in, torch.float32), _ptr(faulty, torch.uint8),
                                 byref(cp), byref(cn), byref(co), _stream(stream)), "r3d_step_csr")

    def step_hist(self, hist, prev: State, nxt: State, out: Outputs, pi_in=None, faulty=None,
                  stream=None):
        cp, cn, co = prev.c(), nxt.c(), out.c()
        _check(_lib.r3d_step_hist(self._h, _ptr(hist, torch.float16),
                                  _ptr(pi_in, torch.float32), _ptr(faulty, torch.uint8),
                                  byref(cp), byref(cn), byref(co), _stream(stream)), "r3d_step_hist")

    def run_hist(self, hists, states, out: Outputs, pi_in=None, faulty=None, stream=None):
        """Frames ``hists`` (fp16 [P, T] device tensors) through the filter:
        frame n reads ``states[n % 2]`` and writes ``states[(n + 1) % 2]``;
        ``out`` holds ``len(hists) * P`` elements per output, frame-major."""
        n = len(hists)
        hp = (c_void_p * n)(*[_ptr(h, torch.float16) for h in hists])
        cs = (CState * 2)(states[0].c(), states[1].c())
        co = out.c()
        _check(_lib.r3d_run_hist(self._h, ctypes.cast(hp, POINTER(c_void_p)), n,
                                 _ptr(pi_in, torch.float32), _ptr(faulty, torch.uint8),
                                 cs, byref(co), _stream(stream)), "r3d_run_hist")

    def last_device_status(self, stream=None) -> int:
        return int(_lib.r3d_last_device_status(self._h, _stream(stream)))

    def min_divergence(self, hist: torch.Tensor, argmax=None, value=None, stream=None):
        """Minimum beta-divergence depth (no prior) of each pixel of the fp16
        histograms [P, T]; returns (argmax int32 [P], value float [P])."""
        if argmax is None:
            argmax = torch.empty(self.P, dtype=torch.int32, device=hist.device)
        if value is None:
            value = torch.empty(self.P, dtype=torch.float32, device=hist.device)
        _check(_lib.r3d_min_divergence(self._h, _ptr(hist, torch.float16), _ptr(argmax, torch.int32),
                                       _ptr(value, torch.float32), _stream(stream)),
               "r3d_min_divergence")
        return argmax, value

    def min_divergence_gauss(self, row_ptr, toa, sigma: float, depth=None, value=None,
                             grid_argmax=None, stream=None):
        """Continuous minimum-divergence depth of each pixel for a Gaussian
        IRF of standard deviation ``sigma`` bins, from CSR photon lists;
        returns (depth float [P], value float [P], grid_argmax int32 [P])."""
        dev = row_ptr.device
        if depth is None:
            depth = torch.empty(self.P, dtype=torch.float32, device=dev)
        if value is None:
            value = torch.empty(self.P, dtype=torch.float32, device=dev)
        if grid_argmax is None:
            grid_argmax = torch.empty(self.P, dtype=torch.int32, device=dev)
        _check(_lib.r3d_min_divergence_gauss(self._h, _ptr(row_ptr, torch.int32), _ptr(toa, torch.int16),
                                             float(sigma), _ptr(depth, torch.float32),
                                             _ptr(value, torch.float32), _ptr(grid_argmax, torch.int32),
                                             _stream(stream)),
               "r3d_min_divergence_gauss")
        return depth, value, grid_argmax

    def step_pirf(self, frame, irf_pix, prev: State, nxt: State, out: Outputs, c_pix=None,
                  pi_in=None, faulty=None, stream=None):
        """One frame with a per-pixel IRF: ``frame`` is an fp16 [P, T] histogram
        tensor or a (row_ptr, toa) photon list; ``irf_pix`` float64 [P, W]."""
        if isinstance(frame, torch.Tensor):
            rp, toa, hist = None, None, _ptr(frame, torch.float16)
        else:
            rp, toa, hist = _ptr(frame[0], torch.int32), _ptr(frame[1], torch.int16), None
        cp, cn, co = prev.c(), nxt.c(), out.c()
        _check(_lib.r3d_step_pirf(self._h, rp, toa, hist, _ptr(irf_pix, torch.float64),
                                  _ptr(c_pix, torch.int32), _ptr(pi_in, torch.float32),
                                  _ptr(faulty, torch.uint8), byref(cp), byref(cn), byref(co),
                                  _stream(stream)), "r3d_step_pirf")

    def grad_workspace_size(self, nframes: int, ckpt_every: int) -> int:
        n = ctypes.c_size_t()
        _check(_lib.r3d_grad_workspace_size(self._h, int(nframes), int(ckpt_every), byref(n)),
               "r3d_grad_workspace_size")
        return int(n.value)

    def filter_forward(self, frames: "Frames", ckpt_every: int, init: State, mean, var,
                       workspace, stream=None):
        ci = init.c()
        _check(_lib.r3d_filter_forward(self._h, byref(frames.c), int(ckpt_every), byref(ci),
                                       _ptr(mean, torch.float32), _ptr(var, torch.float32),
                                       _ptr(workspace, torch.uint8), workspace.numel(),
                                       _stream(stream)), "r3d_filter_forward")

    def filter_backward(self, frames: "Frames", ckpt_every: int, grad_mean, grad_var, workspace,
                        grad, stream=None):
        _check(_lib.r3d_filter_backward(self._h, byref(frames.c), int(ckpt_every),
                                        _ptr(grad_mean, torch.float32),
                                        _ptr(grad_var, torch.float32),
                                        _ptr(workspace, torch.uint8), workspace.numel(),
                                        _ptr(grad, torch.float64), _stream(stream)),
               "r3d_filter_backward")


def min_divergence_msl(bands, hists, argmax=None, value=None, stream=None):
    """Minimum multispectral beta-divergence depth: ``bands`` one Context per
    band (its own IRF), ``hists`` one fp16 [P, T] tensor per band; returns
    (argmax int32 [P], value float [P])."""
    n = len(bands)
    P = bands[0].P
    dev = hists[0].device
    if argmax is None:
        argmax = torch.empty(P, dtype=torch.int32, device=dev)
    if value is None:
        value = torch.empty(P, dtype=torch.float32, device=dev)
    bp = (c_void_p * n)(*[b._h for b in bands])
    hp = (c_void_p * n)(*[_ptr(h, torch.float16) for h in hists])
    _check(_lib.r3d_min_divergence_msl(ctypes.cast(bp, POINTER(c_void_p)), n,
                                       ctypes.cast(hp, POINTER(c_void_p)), _ptr(argmax, torch.int32),
                                       _ptr(value, torch.float32), _stream(stream)),
           "r3d_min_divergence_msl")
    return argmax, value


class Frames:
    """A sequence of photon-list frames (device (row_ptr, toa) pairs) with
    optional presence probabilities [nframes * P] and faulty mask [P]."""

    def __init__(self, frames, pi_in: Optional[torch.Tensor] = None,
                 faulty: Optional[torch.Tensor] = None):
        self.frames = list(frames)
        n = len(self.frames)
        self._rp = (c_void_p * n)(*[_ptr(f[0], torch.int32) for f in self.frames])
        self._toa = (c_void_p * n)(*[_ptr(f[1], torch.int16) for f in self.frames])
        self.pi_in, self.faulty = pi_in, faulty
        self.c = CFrames(n, ctypes.cast(self._rp, POINTER(c_void_p)),
                         ctypes.cast(self._toa, POINTER(c_void_p)),
                         _ptr(pi_in, torch.float32), _ptr(faulty, torch.uint8))

    def __len__(self):
        return len(self.frames)


class R3DFilter:
    """Online filter over frames (Algorithm 1) on one device: owns the two
    ping-pong states; ``step`` returns the frame's outputs."""

    def __init__(self, params: dict, precision=R3D_FP32, device="cuda"):
        self.ctx = Context(params, precision)
        self.P = self.ctx.P
        self.device = device
        self.prev = State.empty(self.P, device)
        self.next = State.empty(self.P, device)
        self.ctx.state_init(self.prev)

    @property
    def state(self) -> State:
        return self.prev

    def set_state(self, st: State):
        for a, b in zip((self.prev.m, self.prev.v, self.prev.pi, self.prev.b),
                        (st.m, st.v, st.pi, st.b)):
            a.copy_(b)

    def step(self, frame, pi_in=None, faulty=None, out: Optional[Outputs] = None) -> Outputs:
        """``frame`` is a (row_ptr, toa) pair of device tensors or an fp16
        histogram [P, T]."""
        out = Outputs.empty(self.P, self.device) if out is None else out
        if isinstance(frame, torch.Tensor):
            self.ctx.step_hist(frame, self.prev, self.next, out, pi_in, faulty)
        else:
            row_ptr, toa = frame
            self.ctx.step_csr(row_ptr, toa, self.prev, self.next, out, pi_in, faulty)
        self.prev, self.next = self.next, self.prev
        return out


@dataclass
class Sequence:
    """One sequence of a batch: its context, its photon-list frames (device
    (row_ptr, toa) pairs), two state buffers (frame n reads ``states[n % 2]``)
    and frame-major outputs of ``nframes * P`` elements."""
    ctx: Context
    frames: list
    states: tuple
    out: Outputs
    pi_in: Optional[torch.Tensor] = None
    faulty: Optional[torch.Tensor] = None
    chunk_rows: int = 0

    @classmethod
    def allocate(cls, ctx: Context, frames, device="cuda", **kw) -> "Sequence":
        P = ctx.P
        st = (State.empty(P, device), State.empty(P, device))
        out = Outputs.empty(len(frames) * P, device)
        return cls(ctx, list(frames), st, out, **kw)

    @property
    def final_state(self) -> State:
        return self.states[len(self.frames) % 2]

    def init_state(self, stream=None):
        self.ctx.state_init(self.states[0], stream)


def _c_sequences(seqs):
    """The r3d_sequence array of a list of Sequence objects, and the host
    pointer arrays it refers to (keep them alive during the call)."""
    arr = (CSequence * len(seqs))()
    keep = []
    for i, q in enumerate(seqs):
        n = len(q.frames)
        rp = (c_void_p * n)(*[_ptr(f[0], torch.int32) for f in q.frames])
        ta = (c_void_p * n)(*[_ptr(f[1], torch.int16) for f in q.frames])
        keep += [rp, ta]
        a = arr[i]
        a.ctx = q.ctx._h
        a.nframes = n
        a.row_ptr = ctypes.cast(rp, POINTER(c_void_p))
        a.toa = ctypes.cast(ta, POINTER(c_void_p))
        a.state[0] = q.states[0].c()
        a.state[1] = q.states[1].c()
        a.out = q.out.c()
        a.pi_in = _ptr(q.pi_in, torch.float32)
        a.faulty = _ptr(q.faulty, torch.uint8)
        a.chunk_rows = int(q.chunk_rows)
    return arr, keep


def batch_run_noalloc(seqs, spin_limit: int = 0, blocks: int = 0, stream=None):
    """Run a batch once with no device allocation (r3d_batch_run_noalloc):
    the tables live in the library's static per-GPU scratch array. Device
    errors go to the first sequence's context (``last_device_status``)."""
    lib = load()
    seqs = list(seqs)
    arr, keep = _c_sequences(seqs)
    opt = CBatchOptions(int(spin_limit), int(blocks))
    _check(lib.r3d_batch_run_noalloc(arr, len(seqs), byref(opt), _stream(stream)),
           "r3d_batch_run_noalloc")
    del keep


class Batch:
    """An r3d_batch: many sequences in one persistent launch, captured once
    into a graph and replayed by ``launch``."""

    def __init__(self, seqs, spin_limit: int = 0, blocks: int = 0):
        lib = load()
        self.seqs = list(seqs)
        arr, self._keep = _c_sequences(self.seqs)
        opt = CBatchOptions(int(spin_limit), int(blocks))
        h = c_void_p()
        _check(lib.r3d_batch_create(arr, len(self.seqs), byref(opt), byref(h)),
               "r3d_batch_create")
        self._h = h

    def launch(self, stream=None):
        _check(_lib.r3d_batch_launch(self._h, _stream(stream)), "r3d_batch_launch")

    def status(self, stream=None) -> int:
        return int(_lib.r3d_batch_status(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.r3d_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
