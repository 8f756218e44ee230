"""The allocation-free entry point cpd_ws_features_noalloc (static device
scratch inside the library) against cpd_ws_features (caller workspace),
through the C-ABI: two calls in a row, the second with a smaller input, each
bitwise equal to the workspace entry point's result (same kernels, same
order); sizes above its limit are rejected before any launch."""
import ctypes

import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, torch
from synth import make_thc

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _call_both(lib, X, Z):
    from paper_2502_17683_amd import _lib
    n0, r_thc = X.shape
    Xd, Zd = to_dev(X), to_dev(Z)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = []
    for noalloc in (False, True):
        feat = torch.full((r_thc, 8), float("nan"), dtype=torch.float32, device="cuda")
        heur = torch.full((r_thc,), float("nan"), dtype=torch.float64, device="cuda")
        if noalloc:
            rc = lib.cpd_ws_features_noalloc(n0, r_thc, Xd.data_ptr(), Zd.data_ptr(), feat.data_ptr(),
                                             heur.data_ptr(), stream)
        else:
            need = lib.cpd_ws_workspace_size(n0, r_thc, 1)
            ws = torch.empty(need, dtype=torch.uint8, device="cuda")
            rc = lib.cpd_ws_features(n0, r_thc, Xd.data_ptr(), Zd.data_ptr(), feat.data_ptr(), heur.data_ptr(),
                                     ws.data_ptr(), need, stream)
        assert rc == _lib.CPD_OK
        torch.cuda.synchronize()
        out.append((feat.cpu().numpy(), heur.cpu().numpy()))
    return out


def test_noalloc_features_equal_workspace_entry_point_twice():
    from paper_2502_17683_amd import _lib
    from oracle import warmstart as ows
    lib = _lib.load()
    for n0, r_thc, seed in ((100, 2000, 20001), (60, 300, 20002)):
        say(f"noalloc features n0={n0} r_thc={r_thc}")
        X, Z = make_thc(n0, r_thc, seed)
        (f_ws, h_ws), (f_na, h_na) = _call_both(lib, X, Z)
        assert np.all(np.isfinite(f_na)) and np.all(np.isfinite(h_na))
        assert np.array_equal(f_na, f_ws) and np.array_equal(h_na, h_ws)
        # and both against the oracle (the bar of the feature tests)
        np.testing.assert_allclose(f_na, ows.features(X, Z), rtol=0, atol=2e-6)


def test_noalloc_rejects_sizes_above_its_limit():
    from paper_2502_17683_amd import _lib
    lib = _lib.load()
    X, Z = make_thc(4, 16, 1)
    Xd, Zd = to_dev(X), to_dev(Z)
    feat = torch.empty((4096, 8), dtype=torch.float32, device="cuda")
    rc = lib.cpd_ws_features_noalloc(4, 2049, Xd.data_ptr(), Zd.data_ptr(), feat.data_ptr(), None, None)
    assert rc == _lib.CPD_ERR_INVALID_ARG
    rc = lib.cpd_ws_features_noalloc(4, 16, None, Zd.data_ptr(), feat.data_ptr(), None, None)
    assert rc == _lib.CPD_ERR_INVALID_ARG
