"""CPU checks of the C-ABI: the library loads, exports every function the
header declares, and the ctypes structures match the C layout."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thccp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    names = _declared_functions()
    for required in ("cpd_init", "cpd_sweep", "cpd_fit", "cpd_destroy", "cpd_workspace_size"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2502_17683_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libthccp.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(_declared_functions()) <= set(_lib.EXPORTS)


def test_ctypes_layout_matches_c():
    from paper_2502_17683_amd import _lib
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "thccp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(cpd_desc), offsetof(cpd_desc, X),
         offsetof(cpd_desc, tol), offsetof(cpd_desc, fit_every), offsetof(cpd_desc, autotune),
         offsetof(cpd_desc, solve_panel), offsetof(cpd_desc, stream), offsetof(cpd_desc, workspace_bytes),
         sizeof(cpd_stats_t), offsetof(cpd_stats_t, cond_est), offsetof(cpd_stats_t, fp64_path));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    D, S = _lib.CpdDesc, _lib.CpdStats
    want = [ctypes.sizeof(D), D.X.offset, D.tol.offset, D.fit_every.offset, D.autotune.offset,
            D.solve_panel.offset, D.stream.offset, D.workspace_bytes.offset, ctypes.sizeof(S),
            S.cond_est.offset, S.fp64_path.offset]
    assert got == want


def test_workspace_size_validates_arguments():
    from paper_2502_17683_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libthccp.so not built")
    lib = _lib.load()
    d = _lib.CpdDesc()
    assert lib.cpd_workspace_size(ctypes.byref(d)) == 0  # null pointers, zero sizes
    for m in range(4):
        d.n[m] = 20
        d.X[m] = 0x1000
        d.init[m] = 0x2000
    d.Z = 0x3000
    d.r_thc, d.r_cp = 80, 60
    d.tol = 1e-4
    size = lib.cpd_workspace_size(ctypes.byref(d))
    assert size > 0
    d.precision = 7
    assert lib.cpd_workspace_size(ctypes.byref(d)) == 0
    d.precision = 0
    d.r_cp = -1
    assert lib.cpd_workspace_size(ctypes.byref(d)) == 0
    # cpd_init rejects a missing workspace before launching anything
    d.r_cp = 60
    plan = ctypes.c_void_p()
    assert lib.cpd_init(ctypes.byref(d), ctypes.byref(plan)) == _lib.CPD_ERR_WORKSPACE
    assert lib.cpd_init(None, ctypes.byref(plan)) == _lib.CPD_ERR_INVALID_ARG
    assert lib.cpd_status_string(_lib.CPD_ERR_NOT_SPD).decode().startswith("normal matrix")


def test_lt_exchange_rejects_bad_arguments_before_any_launch():
    # validation happens on the host before any HIP call, so it runs without a GPU
    from paper_2502_17683_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libthccp.so not built")
    lib = _lib.load()
    t = (ctypes.c_double * 65)(*([0.5] * 65))
    w = (ctypes.c_double * 65)(*([1.0] * 65))
    fake = ctypes.c_void_p(256)  # never dereferenced: every case fails validation first

    def call(n_points, o=4, v=8, r_thc=16, r_cp=8, ws=None, ws_bytes=0, tt=t, E=None):
        return lib.cpd_lt_exchange(o, v, r_thc, r_cp, n_points, fake, fake, fake, fake, fake,
                                   ctypes.cast(tt, ctypes.c_void_p), ctypes.cast(w, ctypes.c_void_p),
                                   fake, fake, fake, fake, None, E, None, fake, fake, fake, ws, ws_bytes, None)

    assert call(0) == _lib.CPD_ERR_INVALID_ARG
    assert call(65) == _lib.CPD_ERR_INVALID_ARG
    assert call(4, o=0) == _lib.CPD_ERR_INVALID_ARG
    assert call(4, r_cp=-1) == _lib.CPD_ERR_INVALID_ARG
    need = lib.cpd_lt_exchange_workspace(4, 8, 16, 8, 4, 0)
    assert need >= 8 * (2 * 4 + 2 * 8 + 5 * 16 + 3 * 8) * 4 * 8
    need_pp = lib.cpd_lt_exchange_workspace(4, 8, 16, 8, 4, 1)
    assert need_pp >= need + 8 * (2 * 4 + 2 * 8 + 8 + 1) * 4 * 8
    # per-point CPDs with a NULL factor pointer, then a workspace sized for the default
    E_bad = (ctypes.c_void_p * 16)(*([256] * 15 + [0]))
    assert call(4, ws=fake, ws_bytes=need_pp, E=ctypes.cast(E_bad, ctypes.c_void_p)) == _lib.CPD_ERR_INVALID_ARG
    E_ok = (ctypes.c_void_p * 16)(*([256] * 16))
    assert call(4, ws=fake, ws_bytes=need, E=ctypes.cast(E_ok, ctypes.c_void_p)) == _lib.CPD_ERR_WORKSPACE
    assert call(4) == _lib.CPD_ERR_WORKSPACE
    assert call(4, ws=fake, ws_bytes=need - 1) == _lib.CPD_ERR_WORKSPACE
    bad_t = (ctypes.c_double * 4)(0.5, float("nan"), 0.5, 0.5)
    assert call(4, ws=fake, ws_bytes=need, tt=bad_t) == _lib.CPD_ERR_INVALID_ARG
    assert lib.cpd_lt_exchange_workspace(4, 8, 16, 8, 0, 0) == 0
    assert lib.cpd_lt_exchange_workspace(4, 8, 16, 8, 65, 0) == 0
