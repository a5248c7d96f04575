"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/r3d.h declares, the ctypes structs match the C layout
and parameter validation rejects bad input before touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "r3d.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(r3d_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def r3d():
    from paper_2004_09211_amd import r3d as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_2004_09211_amd import build
        build.build()
    mod.load()
    return mod


def test_every_declared_symbol_is_exported_and_bound(r3d):
    names = declared_functions()
    assert len(names) >= 9
    lib = ctypes.CDLL(r3d.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared but not exported"
    assert set(names) == set(r3d.SIGNATURES), "binding and header disagree"


def test_struct_layout_matches_c(tmp_path, r3d):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "r3d.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(r3d_params),
         offsetof(r3d_params, d_min), offsetof(r3d_params, W), offsetof(r3d_params, irf),
         offsetof(r3d_params, nu), offsetof(r3d_params, sigma_rw2),
         offsetof(r3d_params, precision), sizeof(r3d_out));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P = r3d.Params
    want = [ctypes.sizeof(P), P.d_min.offset, P.W.offset, P.irf.offset, P.nu.offset,
            P.sigma_rw2.offset, P.precision.offset, ctypes.sizeof(r3d.COut)]
    assert got == want


def test_status_strings(r3d):
    lib = r3d.load()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = lib.r3d_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.r3d_status_string(42).decode() == "unknown status"


def base_params():
    import synth
    wl = synth.tiny_workload()
    return wl.params()


@pytest.mark.parametrize("field,value", [
    ("beta", 0.0), ("beta", -1.0), ("beta", float("nan")), ("sigma_rw2", 0.0), ("c", 99),
    ("c", -1), ("T", 0), ("T", 40000), ("D", 0), ("rows", 0), ("d_max", -5.0),
])
def test_create_rejects_bad_parameters(r3d, field, value):
    p = base_params()
    p[field] = value
    prm, _irf = r3d.make_params(p)
    h = ctypes.c_void_p()
    assert r3d.load().r3d_create(ctypes.byref(prm), ctypes.byref(h)) == -1
    assert not h.value


def test_create_rejects_bad_irf_nu_precision(r3d):
    lib = r3d.load()
    for mutate in (lambda p: p.__setitem__("irf", -np.abs(p["irf"])),
                   lambda p: p.__setitem__("irf", np.zeros_like(p["irf"])),
                   lambda p: p.__setitem__("nu", np.zeros(9)),
                   lambda p: p.__setitem__("irf", np.ones(300) / 300)):
        p = base_params()
        mutate(p)
        prm, _irf = r3d.make_params(p)
        h = ctypes.c_void_p()
        assert lib.r3d_create(ctypes.byref(prm), ctypes.byref(h)) == -1
    p = base_params()
    prm, _irf = r3d.make_params(p)
    prm.precision = 7
    assert lib.r3d_create(ctypes.byref(prm), ctypes.byref(ctypes.c_void_p())) == -1
    assert lib.r3d_create(ctypes.byref(prm), None) == -1


def test_null_context_and_pointers_rejected(r3d):
    lib = r3d.load()
    st = r3d.CState()
    out = r3d.COut()
    assert lib.r3d_step_csr(None, None, None, None, None, ctypes.byref(st), ctypes.byref(st),
                            ctypes.byref(out), None) == -1
    assert lib.r3d_step_hist(None, None, None, None, ctypes.byref(st), ctypes.byref(st),
                             ctypes.byref(out), None) == -1
    assert lib.r3d_state_init(None, ctypes.byref(st), None) == -1
    assert lib.r3d_histogram(None, None, None, None, None) == -1
    assert lib.r3d_cost(None, None, 0, None, None) == -1
    assert lib.r3d_last_device_status(None, None) == -1
    lib.r3d_destroy(None)


def test_batch_entry_points_reject_bad_arguments(r3d):
    lib = r3d.load()
    h = ctypes.c_void_p()
    assert lib.r3d_batch_create(None, 1, None, ctypes.byref(h)) == -1
    seqs = (r3d.CSequence * 1)()
    assert lib.r3d_batch_create(seqs, 0, None, ctypes.byref(h)) == -1
    assert lib.r3d_batch_create(seqs, 1, None, ctypes.byref(h)) == -1  # NULL context
    assert lib.r3d_batch_create(seqs, 1, None, None) == -1
    bad = r3d.CBatchOptions(0, -3)
    assert lib.r3d_batch_create(seqs, 1, ctypes.byref(bad), ctypes.byref(h)) == -1
    assert not h.value
    assert lib.r3d_batch_launch(None, None) == -1
    assert lib.r3d_batch_status(None, None) == -1
    lib.r3d_batch_destroy(None)
    # the allocation-free run checks its arguments before any HIP call
    assert lib.r3d_batch_run_noalloc(None, 1, None, None) == -1
    assert lib.r3d_batch_run_noalloc(seqs, 0, None, None) == -1
    assert lib.r3d_batch_run_noalloc(seqs, 1, None, None) == -1  # NULL context
    assert lib.r3d_batch_run_noalloc(seqs, 1, ctypes.byref(bad), None) == -1


def test_filter_entry_points_reject_bad_arguments(r3d):
    lib = r3d.load()
    n = ctypes.c_size_t()
    assert lib.r3d_grad_workspace_size(None, 5, 5, ctypes.byref(n)) == -1
    fr = r3d.CFrames()
    st = r3d.CState()
    assert lib.r3d_filter_forward(None, ctypes.byref(fr), 5, ctypes.byref(st), None, None, None,
                                  0, None) == -1
    assert lib.r3d_filter_backward(None, ctypes.byref(fr), 5, None, None, None, 0, None,
                                   None) == -1


def test_frames_layout_matches_c(tmp_path, r3d):
    src = tmp_path / "fr.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "r3d.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(r3d_frames), offsetof(r3d_frames, row_ptr),
         offsetof(r3d_frames, toa), offsetof(r3d_frames, pi_in), offsetof(r3d_frames, faulty));
  return 0;
}
""")
    exe = tmp_path / "fr"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    F = r3d.CFrames
    assert got == [ctypes.sizeof(F), F.row_ptr.offset, F.toa.offset, F.pi_in.offset,
                   F.faulty.offset]


def test_sequence_layout_matches_c(tmp_path, r3d):
    src = tmp_path / "seq.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "r3d.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(r3d_sequence),
         offsetof(r3d_sequence, nframes), offsetof(r3d_sequence, row_ptr),
         offsetof(r3d_sequence, toa), offsetof(r3d_sequence, state),
         offsetof(r3d_sequence, out), offsetof(r3d_sequence, pi_in),
         offsetof(r3d_sequence, faulty), offsetof(r3d_sequence, chunk_rows));
  return 0;
}
""")
    exe = tmp_path / "seq"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    S = r3d.CSequence
    want = [ctypes.sizeof(S)] + [getattr(S, f).offset for f in
                                 ("nframes", "row_ptr", "toa", "state", "out", "pi_in", "faulty",
                                  "chunk_rows")]
    assert got == want


def test_binding_refuses_missing_library(tmp_path):
    from paper_2004_09211_amd import r3d as mod
    saved = mod._lib
    mod._lib = None
    try:
        with pytest.raises(RuntimeError):
            mod.load(str(tmp_path / "nope.so"))
    finally:
        mod._lib = saved


def test_product_path_does_not_import_oracle():
    """The HIP path's Python binding and sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2004_09211_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", text), f"{f} references the oracle"
