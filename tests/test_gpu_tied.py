"""Particle-tied CP-ALS (symmetric ALS) on the GPU against oracle/tied.py."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, torch
from oracle import tied
from synth import init_factors, make_thc, planted_diag_thc

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _cpd(X, Z, init, r_cp, **kw):
    from paper_2502_17683_amd import CPD
    xs = [to_dev(x) for x in X] if isinstance(X, list) else to_dev(X)
    return CPD(xs, to_dev(Z), r_cp, [to_dev(f) for f in init], tied=True, **kw)


@pytest.mark.parametrize("aliased", [True, False])
def test_tied_trajectory_fp64_matches_oracle(aliased):
    X, Z = make_thc(20, 80, 11)
    if aliased:
        Xs = X
        Xo = [X] * 4
    else:
        # distinct X arrays with the tied dimensions: the tied projections are
        # formed by their own products, not copied
        rng = np.random.default_rng(12)
        X1 = X * rng.uniform(0.8, 1.2, X.shape)
        X2, _ = make_thc(20, 80, 13)
        Xs = Xo = [X, X1, X2, X2 * 1.1]
    init = init_factors([20] * 4, 60, 1011)
    say(f"[tied] fp64 aliased={aliased}")
    c = _cpd(Xs, Z, init, 60, precision="fp64", tol=0.0, fit_floor=0.0)
    fits = np.array(c.sweep(30))
    F, lam = c.factors()
    c.close()
    ref = tied.tied_cp_als(Xo, Z, init, 30, tol=0.0, fit_floor=0.0)
    rf = np.array(ref["fits"])
    err = np.abs(fits - rf) / rf
    say(f"[tied] max fit rel err {err.max():.2e}, last fit {fits[-1]:.6e}")
    # symmetric ALS amplifies rounding more than plain ALS (each half-step
    # also feeds its own previous value back): FP64 trajectories of other
    # seeds drift up to 2.5e-10 from the oracle's, against ~1e-12 untied
    assert np.all(err <= 2e-9)
    Fh = [f.cpu().numpy() for f in F]
    assert np.array_equal(Fh[0], Fh[1]) and np.array_equal(Fh[2], Fh[3])
    for m in (0, 2):
        np.testing.assert_allclose(Fh[m], ref["F"][m], rtol=0, atol=1e-8)
    np.testing.assert_allclose(lam.cpu().numpy(), ref["lam"], rtol=1e-8)


def test_tied_stopping_rule_and_direct_launch():
    X, Z = make_thc(20, 80, 14)
    init = init_factors([20] * 4, 60, 1014)
    ref = tied.tied_cp_als([X] * 4, Z, init, 200, tol=1e-4, fit_floor=0.0)
    a = _cpd(X, Z, init, 60, precision="fp64", tol=1e-4, fit_floor=0.0)
    fa = a.sweep(200)
    b = _cpd(X, Z, init, 60, precision="fp64", tol=1e-4, fit_floor=0.0, use_graph=False)
    fb = b.sweep(200)
    say(f"[tied] sweeps gpu {len(fa)} oracle {len(ref['fits'])}")
    assert len(fa) == len(ref["fits"]) and fa == fb
    assert a.stats()["converged"] == 1
    a.close()
    b.close()


def test_tied_exact_cpd_is_a_fixed_point():
    X, Zd = planted_diag_thc(24, 16, 15)
    c = _cpd(X, Zd, [X, X, X, X], 16, precision="fp64", tol=0.0, fit_floor=0.0)
    fits = c.sweep(3)
    c.close()
    say(f"[tied] planted fits {fits}")
    assert max(fits) < 1e-6


def test_tied_fp32_error_report():
    """FP32: the first sweep agrees with the FP64 oracle to FP32 rounding;
    later sweeps drift further than in plain ALS (observed up to 5.4e-2 at
    this seed, against 3e-4 untied), because the tied iteration amplifies
    rounding (see the FP64 test)."""
    X, Z = make_thc(20, 80, 16)
    init = init_factors([20] * 4, 60, 1016)
    c = _cpd(X, Z, init, 60, precision="fp32", tol=0.0, fit_floor=0.0)
    fits = np.array(c.sweep(20))
    c.close()
    rf = np.array(tied.tied_cp_als([X] * 4, Z, init, 20, tol=0.0, fit_floor=0.0)["fits"])
    err = np.abs(fits - rf) / rf
    say(f"[tied] fp32 first-sweep rel err {err[0]:.2e}, max {err.max():.2e}")
    assert err[0] <= 1e-5
    assert err.max() <= 0.1


def test_tied_rejects_mixed_and_mismatched_modes():
    from paper_2502_17683_amd import CpdError
    X, Z = make_thc(20, 80, 17)
    init = init_factors([20] * 4, 60, 1017)
    with pytest.raises(CpdError):
        _cpd(X, Z, init, 60, precision="mixed")
    X6, _ = make_thc(6, 80, 18)
    with pytest.raises(CpdError):
        _cpd([X, X6, X, X], Z, [init[0], init_factors([6], 60, 1)[0], init[2], init[3]], 60, precision="fp64")


def test_tied_batch_equals_single_runs():
    """Grouped tied problems of uneven size: each equals its single run, bit
    for bit (the grouped launches and tied copies are per problem)."""
    from paper_2502_17683_amd import CPD, CPDBatch
    probs = []
    for i, (n, rt, rc) in enumerate([(12, 48, 30), (20, 80, 60), (9, 40, 17)]):
        X, Z = make_thc(n, rt, 30 + i)
        probs.append({"X": X, "Z": Z, "r_cp": rc, "init": init_factors([n] * 4, rc, 1030 + i)})
    b = CPDBatch(probs, precision="fp64", tol=0.0, fit_floor=0.0, tied=True)
    fb = b.sweep(8)
    for i, pr in enumerate(probs):
        c = CPD(pr["X"], pr["Z"], pr["r_cp"], pr["init"], precision="fp64", tol=0.0, fit_floor=0.0, tied=True)
        fs = c.sweep(8)
        Fs, ls = c.factors()
        c.close()
        Fb, lb = b.factors(i)
        assert fb[i] == fs
        assert all(torch.equal(x, y) for x, y in zip(Fs, Fb)) and torch.equal(ls, lb)
    b.close()
