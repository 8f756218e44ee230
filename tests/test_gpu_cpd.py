"""Whole-method parity on the GPU through the C-ABI: matrix-free MTTKRP,
FP64 trajectories against the CPU oracle (O1 dense, O2 matrix-free),
FP32 and split-BF16 error reports, stopping rule, checkpoint resume,
determinism, graph replay and failure handling."""
import ctypes

import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, rel_err, torch
from oracle import dense, matfree
from synth import make_thc, init_factors

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _norm_cols(F):
    nrm = np.linalg.norm(F, axis=0)
    return F / np.where(nrm > 0, nrm, 1.0)


def _general(seed, dims=(13, 21, 9, 30), r_thc=70, r_cp=50):
    rng = np.random.default_rng(seed)
    X = [rng.standard_normal((d, r_thc)) / np.sqrt(d) for d in dims]
    Z = rng.standard_normal((r_thc, r_thc)) / np.sqrt(r_thc)
    init = [rng.standard_normal((d, r_cp)) for d in dims]
    return X, Z, init


def _plan(X, Z, init, r_cp, **kw):
    from paper_2502_17683_amd import CPD
    return CPD([to_dev(x) for x in X] if isinstance(X, list) else to_dev(X), to_dev(Z), r_cp,
               [to_dev(f) for f in init], **kw)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 3e-5), ("mixed", 1e-4)])
def test_mttkrp_general_modes(precision, tol):
    """Distinct X_m, non-symmetric Z, ragged sizes: every mode's MTTKRP
    against the oracle (P1 on the GPU)."""
    X, Z, init = _general(1)
    say(f"mttkrp general {precision}")
    cpd = _plan(X, Z, init, 50, precision=precision)
    F = [_norm_cols(f) for f in init]
    for n in range(4):
        ref = matfree.mttkrp(X, Z, F, n)
        got = cpd.mttkrp(n).cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say(f"  mode {n}: rel err {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("code", [100000, 120000, 140000])
def test_mttkrp_split_direct_load_shapes(code):
    """Split-BF16 MTTKRP of every mode with the direct-load 256 x 256 tiles
    forced for all three products (split-K slices on the back-projection for
    codes above 100000), distinct X_m and a non-symmetric Z, ragged sizes
    that leave partial tiles: element by element against the oracle, within
    the split bound of the products' contraction lengths times the oracle's
    MTTKRP of absolute values."""
    from paper_2502_17683_amd import test_split_force
    dims, r_thc, r_cp = (300, 281, 260, 290), 600, 520
    X, Z, init = _general(4, dims, r_thc, r_cp)
    F = [_norm_cols(f) for f in init]
    u = lambda K: 3 * 2.0 ** -16 + K * 2.0 ** -24
    k = 1.001 * (3 * u(max(dims)) + 2 * u(r_thc) + 6 * 2.0 ** -24)
    prev = test_split_force(code)
    try:
        cpd = _plan(X, Z, init, r_cp, precision="mixed")
        log = cpd.autotune_log()
        for n in range(4):
            ref = matfree.mttkrp(X, Z, F, n)
            A = matfree.mttkrp([np.abs(x) for x in X], np.abs(Z), [np.abs(f) for f in F], n)
            got = cpd.mttkrp(n).cpu().numpy()
            ratio = float(np.max(np.abs(got - ref) / (A + 1e-300)))
            say(f"  forced {code} mode {n}: max |err| / |.|-MTTKRP {ratio:.2e} (bound {k:.2e})")
            assert np.all(np.abs(got - ref) <= k * A)
        cpd.close()
    finally:
        test_split_force(prev)
    say(f"  autotune log: {log!r}")


def test_mttkrp_matches_dense_bruteforce():
    """Small molecule-like input: GPU MTTKRP == G_(n) KR(others) of the
    explicitly formed tensor."""
    X, Z = make_thc(20, 80, 0)
    init = init_factors([20] * 4, 60, 1000)
    cpd = _plan(X, Z, init, 60)
    G = dense.dense_tensor([X] * 4, Z)
    F = [_norm_cols(f) for f in init]
    for n in range(4):
        ref = dense.dense_mttkrp(G, F, n)
        got = cpd.mttkrp(n).cpu().numpy()
        assert rel_err(got, ref) <= 1e-12


def test_trajectory_small_fp64_vs_dense_oracle():
    """N=20, R_thc=80, R_cp=60, 50 sweeps: every fit within 1e-10 (relative)
    of the dense textbook oracle and of the matrix-free oracle."""
    X, Z = make_thc(20, 80, 0)
    init = init_factors([20] * 4, 60, 1000)
    cpd = _plan(X, Z, init, 60, tol=0.0, fit_floor=0.0)
    fits = np.array(cpd.sweep(50))
    G = dense.dense_tensor([X] * 4, Z)
    r1 = dense.dense_cp_als(G, init, 50, tol=0.0, fit_floor=0.0)
    r2 = matfree.mf_cp_als([X] * 4, Z, init, 50, tol=0.0, fit_floor=0.0)
    f1, f2 = np.array(r1["fits"]), np.array(r2["fits"])
    say(f"fits gpu {fits[[0, 9, 49]]} max rel vs O1 {np.max(np.abs(fits - f1) / f1):.2e} "
        f"vs O2 {np.max(np.abs(fits - f2) / f2):.2e}")
    assert len(fits) == 50
    assert np.all(np.abs(fits - f1) <= 1e-10 * f1)
    assert np.all(np.abs(fits - f2) <= 1e-10 * f2)
    F, lam = cpd.factors()
    fe = max(rel_err(F[m].cpu().numpy(), r2["F"][m]) for m in range(4))
    st = cpd.stats()
    say(f"factor rel err vs O2 {fe:.2e}, cond_est {st['cond_est']:.2e}")
    assert fe <= 1e-8


def test_trajectory_general_fp64():
    """Distinct X_m and a non-symmetric core: 15 sweeps against O2."""
    X, Z, init = _general(5)
    cpd = _plan(X, Z, init, 50, tol=0.0, fit_floor=0.0)
    fits = np.array(cpd.sweep(15))
    ref = np.array(matfree.mf_cp_als(X, Z, init, 15, tol=0.0, fit_floor=0.0)["fits"])
    say(f"general fits {fits[-1]:.6f} vs {ref[-1]:.6f}")
    assert np.all(np.abs(fits - ref) <= 1e-10 * ref)


def test_trajectory_mid_fp64():
    """N=200, R_thc=R_cp=1000 (several 64-blocks, padded R): 8 sweeps vs O2."""
    X, Z = make_thc(200, 1000, 0)
    init = init_factors([200] * 4, 1000, 1000)
    cpd = _plan(X, Z, init, 1000, tol=0.0, fit_floor=0.0)
    fits = np.array(cpd.sweep(8))
    ref = np.array(matfree.mf_cp_als([X] * 4, Z, init, 8, tol=0.0, fit_floor=0.0)["fits"])
    say(f"mid fits gpu {fits} oracle {ref}")
    assert np.all(np.abs(fits - ref) <= 1e-10 * ref)


def test_ragged_rank_fp64():
    """R_cp = 100 (one full and one partial 64-block), R_thc = 130."""
    X, Z = make_thc(40, 130, 2)
    init = init_factors([40] * 4, 100, 1002)
    cpd = _plan(X, Z, init, 100, tol=0.0, fit_floor=0.0)
    fits = np.array(cpd.sweep(10))
    ref = np.array(matfree.mf_cp_als([X] * 4, Z, init, 10, tol=0.0, fit_floor=0.0)["fits"])
    assert np.all(np.abs(fits - ref) <= 1e-10 * ref)


def test_stopping_rule_matches_oracle():
    X, Z = make_thc(20, 80, 1)
    init = init_factors([20] * 4, 60, 1001)
    cpd = _plan(X, Z, init, 60, tol=1e-2)
    fits = cpd.sweep(200)
    ref = matfree.mf_cp_als([X] * 4, Z, init, 200, tol=1e-2)["fits"]
    assert len(fits) == len(ref) < 200
    assert cpd.stats()["converged"] == 1
    assert cpd.sweep(5) == []  # converged: further sweeps do nothing


def test_graph_replay_equals_direct_launch():
    X, Z = make_thc(20, 80, 3)
    init = init_factors([20] * 4, 60, 1003)
    a = _plan(X, Z, init, 60, tol=0.0, use_graph=True)
    b = _plan(X, Z, init, 60, tol=0.0, use_graph=False)
    fa, fb = a.sweep(12), b.sweep(12)
    assert fa == fb
    Fa, la = a.factors()
    Fb, lb = b.factors()
    for m in range(4):
        assert torch.equal(Fa[m], Fb[m])


def test_deterministic_bitwise():
    X, Z = make_thc(60, 240, 4)
    init = init_factors([60] * 4, 200, 1004)
    runs = []
    for _ in range(2):
        c = _plan(X, Z, init, 200, tol=0.0)
        runs.append((c.sweep(6), c.factors()))
    assert runs[0][0] == runs[1][0]
    for m in range(4):
        assert torch.equal(runs[0][1][0][m], runs[1][1][0][m])


def test_checkpoint_resume_bitwise():
    X, Z = make_thc(30, 120, 5)
    init = init_factors([30] * 4, 90, 1005)
    a = _plan(X, Z, init, 90, tol=0.0)
    f_first = a.sweep(6)
    F, lam = a.factors()
    f_rest = a.sweep(6)
    b = _plan(X, Z, init, 90, tol=0.0)
    b.set_factors(F, lam, prev_fit=f_first[-1], sweeps=6)
    assert b.sweep(6) == f_rest
    assert b.stats()["sweeps"] == 12


def test_fp32_error_report():
    """Plain FP32 (Cholesky included): per-sweep fit error vs FP64 stated,
    within the 1e-4 'same fit' tolerance over the first 10 sweeps (measured
    on one MI355X: <= 5.5e-6)."""
    X, Z = make_thc(200, 1000, 0)
    init = init_factors([200] * 4, 1000, 1000)
    f64 = np.array(_plan(X, Z, init, 1000, tol=0.0).sweep(10))
    f32 = np.array(_plan(X, Z, init, 1000, tol=0.0, precision="fp32").sweep(10))
    err = np.abs(f32 - f64) / f64
    say(f"fp32 per-sweep fit error vs fp64: {err}")
    assert np.all(err <= 1e-4)


def test_mixed_error_report():
    """Split BF16: fit (evaluated in FP64) per sweep vs the FP64 run, within
    the 1e-4 'same fit' tolerance over the first 10 sweeps (measured: <=
    2.3e-6)."""
    X, Z = make_thc(200, 1000, 0)
    init = init_factors([200] * 4, 1000, 1000)
    f64 = np.array(_plan(X, Z, init, 1000, tol=0.0).sweep(10))
    fmx = np.array(_plan(X, Z, init, 1000, tol=0.0, precision="mixed").sweep(10))
    err = np.abs(fmx - f64) / f64
    say(f"mixed per-sweep fit error vs fp64: {err}")
    assert np.all(err <= 1e-4)


def test_mixed_fit_every():
    X, Z = make_thc(20, 80, 0)
    init = init_factors([20] * 4, 60, 1000)
    c = _plan(X, Z, init, 60, tol=0.0, precision="mixed", fit_every=3)
    fits = c.sweep(9)
    assert len(fits) == 9
    assert [f > 0 for f in fits] == [False, False, True] * 3
    assert c.stats()["sweeps"] == 9


def test_zero_column_fallback_matches_oracle():
    """A zero initial column makes V singular: with the damped retry the
    run matches the oracle's identical policy; without it, NOT_SPD."""
    from paper_2502_17683_amd import CpdError
    X, Z = make_thc(20, 80, 6)
    init = init_factors([20] * 4, 60, 1006)
    init[1][:, 7] = 0.0
    c = _plan(X, Z, init, 60, tol=0.0)
    fits = np.array(c.sweep(5))
    ref = matfree.mf_cp_als([X] * 4, Z, init, 5, tol=0.0)
    assert ref["fallbacks"] > 0
    assert c.stats()["fallbacks"] == ref["fallbacks"]
    assert np.all(np.abs(fits - np.array(ref["fits"])) <= 1e-9 * np.array(ref["fits"]))
    c2 = _plan(X, Z, init, 60, tol=0.0, chol_fallback=False)
    with pytest.raises(CpdError) as e:
        c2.sweep(2)
    assert e.value.code == -3


@pytest.mark.parametrize("where", ["X", "Z"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nonfinite_input_is_reported(where, precision):
    """A NaN in X or an Inf in Z makes ||G||^2 non-finite: the plan is
    flagged at init, its sweeps do nothing, and the first synchronising
    call reports CPD_ERR_NONFINITE."""
    from paper_2502_17683_amd import CPD, CpdError
    X, Z = make_thc(20, 80, 7)
    init = init_factors([20] * 4, 60, 1007)
    if where == "X":
        X = X.copy()
        X[3, 5] = np.nan
    else:
        Z = Z.copy()
        Z[10, 10] = np.inf
    c = CPD(X, Z, 60, init, precision=precision, tol=0.0, fit_floor=0.0)
    with pytest.raises(CpdError) as e:
        c.sweep(2)
    assert e.value.code == -4
    c.close()


def test_workspace_too_small_is_rejected():
    from paper_2502_17683_amd import _lib
    lib = _lib.load()
    X, Z = make_thc(20, 80, 0)
    init = init_factors([20] * 4, 60, 1000)
    Xd, Zd = to_dev(X), to_dev(Z)
    In = [to_dev(f) for f in init]
    d = _lib.CpdDesc()
    for m in range(4):
        d.n[m] = 20
        d.X[m] = Xd.data_ptr()
        d.init[m] = In[m].data_ptr()
    d.Z = Zd.data_ptr()
    d.r_thc, d.r_cp = 80, 60
    need = lib.cpd_workspace_size(ctypes.byref(d))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    d.workspace = ws.data_ptr()
    d.workspace_bytes = need - 1
    plan = ctypes.c_void_p()
    assert lib.cpd_init(ctypes.byref(d), ctypes.byref(plan)) == _lib.CPD_ERR_WORKSPACE


def test_async_sweeps_match_synchronised_sweeps():
    """Asynchronous sweeps (damped retry inside the graph) and synchronised
    sweeps (fused factorisation + forward solve, host replay on a failed
    pivot) compute the same iterates bit for bit."""
    X, Z = make_thc(40, 160, 7)
    init = init_factors([40] * 4, 130, 1007)
    a = _plan(X, Z, init, 130, tol=0.0)
    fa = a.sweep(7)
    b = _plan(X, Z, init, 130, tol=0.0)
    b.sweep(7, sync=False)
    assert b.fit() == fa[-1]
    Fa, _ = a.factors()
    Fb, _ = b.factors()
    for m in range(4):
        assert torch.equal(Fa[m], Fb[m])


def test_async_fallback_matches_replay():
    X, Z = make_thc(20, 80, 6)
    init = init_factors([20] * 4, 60, 1006)
    init[2][:, 3] = 0.0
    a = _plan(X, Z, init, 60, tol=0.0)
    fa = a.sweep(4)
    b = _plan(X, Z, init, 60, tol=0.0)
    b.sweep(4, sync=False)
    assert b.fit() == fa[-1]
    assert a.stats()["fallbacks"] == b.stats()["fallbacks"] > 0


def test_run_logged_writes_one_line_per_sweep(tmp_path):
    """The per-sweep JSONL log follows the same trajectory as plain sweeps."""
    import json
    X, Z = make_thc(20, 80, 0)
    init = init_factors([20] * 4, 60, 1000)
    a = _plan(X, Z, init, 60, tol=0.0)
    ref = a.sweep(6)
    a.close()
    b = _plan(X, Z, init, 60, tol=0.0)
    path = tmp_path / "sweeps.jsonl"
    fits = b.run_logged(6, str(path))
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert fits == ref and len(lines) == 6
    assert [d["sweep"] for d in lines] == list(range(1, 7))
    assert [d["fit"] for d in lines] == ref
    assert lines[0]["dfit_rel"] is None and lines[1]["dfit_rel"] == abs(ref[1] - ref[0]) / ref[0]
    assert all(d["t_sweep_ms"] > 0 and d["chol_fallbacks"] == 0 for d in lines)
    b.close()
