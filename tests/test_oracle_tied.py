"""Pins for oracle/tied.py: dense fit, half-steps against the plain ALS
update from the same tied state, and the exact tied CPD as a fixed point."""
import numpy as np
import pytest

from oracle import dense, matfree, tied
from synth import init_factors, make_thc, planted_diag_thc


def test_fit_matches_dense_reconstruction():
    X, Z = make_thc(6, 20, 2)
    rng = np.random.default_rng(3)
    Xs = [X, X, rng.standard_normal((6, 20)), rng.standard_normal((6, 20))]  # X2 != X0
    G = dense.dense_tensor(Xs, Z)
    st = tied.TiedCPALS(Xs, Z, init_factors([6] * 4, 5, 1002))
    for _ in range(3):
        f = st.sweep()
        ref = dense.dense_fit(G, st.lam, st.F)
        assert f == pytest.approx(ref, rel=1e-9)
        assert np.array_equal(st.F[0], st.F[1]) and np.array_equal(st.F[2], st.F[3])


def test_half_steps_are_plain_als_updates():
    # from a tied state, the tied mode-0 (mode-2) step is the plain ALS
    # update of mode 0 (mode 2), followed by the copy
    X, Z = make_thc(8, 24, 4)
    Xs = [X] * 4
    init = init_factors([8] * 4, 6, 1004)
    st = tied.TiedCPALS(Xs, Z, init)
    st.sweep()
    ref = matfree.MatFreeCPALS(Xs, Z, [f.copy() for f in st.F])
    ref.F = [f.copy() for f in st.F]
    ref.W = matfree.projections(Xs, ref.F)
    ref.gram = [f.T @ f for f in ref.F]
    st._update(0)
    ref.update(0)
    np.testing.assert_allclose(st.F[0], ref.F[0], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(st.lam, ref.lam, rtol=1e-10)
    ref.F[1] = ref.F[0].copy()
    ref.W[1] = Xs[1].T @ ref.F[1]
    ref.gram[1] = ref.F[1].T @ ref.F[1]
    st._update(2)
    ref.update(2)
    np.testing.assert_allclose(st.F[2], ref.F[2], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(st.lam, ref.lam, rtol=1e-10)


def test_exact_tied_cpd_is_a_fixed_point():
    # diagonal core and one X: G = sum_P z_P x_P o x_P o x_P o x_P, a tied
    # CPD with A = B = the columns of X
    X, Zd = planted_diag_thc(7, 5, 8)
    res = tied.tied_cp_als([X] * 4, Zd, [X, X, X, X], 3, tol=0.0, fit_floor=0.0)
    assert max(res["fits"]) < 1e-7


def test_tied_fit_decreases_on_a_thc_input():
    X, Z = make_thc(12, 48, 5)
    res = tied.tied_cp_als([X] * 4, Z, init_factors([12] * 4, 30, 1005), 60, tol=0.0)
    f = np.array(res["fits"])
    assert f[-1] < 0.5 * f[0]
    assert np.all(np.diff(f[5:]) <= 1e-9)
