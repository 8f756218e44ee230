"""Pins for O2 (oracle/matfree.py) against O1's dense tensor, closed forms,
planted decompositions, special cases and invariances."""
import numpy as np
import pytest

from oracle import dense, matfree
from synth import make_thc, init_factors, planted_diag_thc


def _general(seed, dims=(4, 5, 3, 6), r_thc=7, r_cp=5):
    rng = np.random.default_rng(seed)
    X = [rng.standard_normal((d, r_thc)) for d in dims]
    Z = rng.standard_normal((r_thc, r_thc))  # non-symmetric on purpose
    F = [rng.standard_normal((d, r_cp)) for d in dims]
    return X, Z, F


@pytest.mark.parametrize("n", range(4))
def test_mttkrp_matches_dense(n):
    """P1: matrix-free MTTKRP == G_(n) KR(others), every mode."""
    X, Z, F = _general(10 + n)
    G = dense.dense_tensor(X, Z)
    ref = dense.dense_mttkrp(G, F, n)
    np.testing.assert_allclose(matfree.mttkrp(X, Z, F, n), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_cached_core_product_in_sweep_matches_dense():
    """P1 for the reuse of Z(W2 o W3) in mode 1 and Z^T(W0 o W1) in mode 3."""
    X, Z, F = _general(21)
    G = dense.dense_tensor(X, Z)
    st = matfree.MatFreeCPALS(X, Z, F)
    for n in range(4):
        Fcur = [f.copy() for f in st.F]
        M = st.mttkrp(n)
        ref = dense.dense_mttkrp(G, Fcur, n)
        np.testing.assert_allclose(M, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
        st.update(n)


def test_norm2_closed_form():
    """P2: ||G||^2 = <Z, (S0 o S1) Z (S2 o S3)>."""
    X, Z, _ = _general(31)
    G = dense.dense_tensor(X, Z)
    assert matfree.thc_norm2(X, Z) == pytest.approx(float(np.sum(G * G)), rel=1e-13)


def test_norm2_symmetric_form():
    """P2, the symmetric special case: sum Z_PQ Z_P'Q' S_PP'^2 S_QQ'^2."""
    X, Z = make_thc(6, 9, 0)
    S = X.T @ X
    ref = np.einsum("PQ,pq,Pp,Qq->", Z, Z, S * S, S * S)
    assert matfree.thc_norm2([X] * 4, Z) == pytest.approx(ref, rel=1e-13)


def test_fit_terms_match_dense():
    """P3: <G,G~> and ||G~||^2 after a full sweep, against dense reconstruction."""
    X, Z, F = _general(41)
    G = dense.dense_tensor(X, Z)
    st = matfree.MatFreeCPALS(X, Z, F)
    st.sweep()
    Gt = dense.reconstruct(st.lam, st.F)
    inner, model2 = st.fit_terms()
    assert inner == pytest.approx(float(np.sum(G * Gt)), rel=1e-12)
    assert model2 == pytest.approx(float(np.sum(Gt * Gt)), rel=1e-12)
    assert st.fit() == pytest.approx(dense.dense_fit(G, st.lam, st.F), rel=1e-9)


def test_trajectory_matches_dense_small_molecule():
    """O2 and O1 follow the same iterates on the THC generator (N=20,
    R_thc=80, R_cp=60, 50 sweeps)."""
    X, Z = make_thc(20, 80, 0)
    init = init_factors([20] * 4, 60, 1000)
    G = dense.dense_tensor([X] * 4, Z)
    r1 = dense.dense_cp_als(G, init, max_sweeps=50, tol=0.0)
    r2 = matfree.mf_cp_als([X] * 4, Z, init, max_sweeps=50, tol=0.0)
    f1, f2 = np.array(r1["fits"]), np.array(r2["fits"])
    assert len(f1) == len(f2) == 50
    np.testing.assert_allclose(f2, f1, rtol=1e-8)
    assert f1[-1] < f1[0]


def test_planted_diagonal_core_recovered():
    """P4: Z = diag(z) makes G an exact rank-R_thc CP tensor with factors
    X diag(z^(1/4)); ALS started near it converges to a zero residual."""
    X, Z = planted_diag_thc(8, 6, 3)
    rng = np.random.default_rng(4)
    truth = X * np.diag(Z)[None, :] ** 0.25
    G = dense.dense_tensor([X] * 4, Z)
    np.testing.assert_allclose(dense.reconstruct(np.ones(6), [truth] * 4), G, atol=1e-14)
    init = [truth + 1e-3 * rng.standard_normal(truth.shape) for _ in range(4)]
    rd = dense.dense_cp_als(G, init, max_sweeps=200, tol=0.0, fit_floor=1e-11)
    assert rd["fits"][-1] <= 1e-10
    rm = matfree.mf_cp_als([X] * 4, Z, init, max_sweeps=200, tol=0.0, fit_floor=1e-8)
    assert rm["fits"][-1] <= 1e-7


def test_identity_factors_special_case():
    """P6: X = I (n = R_thc) gives G[p,p,r,r] = Z[p,r], else 0, so each
    MTTKRP is a Hadamard product with one matrix product."""
    rng = np.random.default_rng(6)
    R, r_cp = 5, 4
    Z = rng.standard_normal((R, R))
    X = [np.eye(R)] * 4
    G = dense.dense_tensor(X, Z)
    expect = np.zeros((R, R, R, R))
    for p in range(R):
        for r in range(R):
            expect[p, p, r, r] = Z[p, r]
    np.testing.assert_allclose(G, expect, atol=1e-15)
    F = [rng.standard_normal((R, r_cp)) for _ in range(4)]
    closed = [F[1] * (Z @ (F[2] * F[3])), F[0] * (Z @ (F[2] * F[3])),
              F[3] * (Z.T @ (F[0] * F[1])), F[2] * (Z.T @ (F[0] * F[1]))]
    for n in range(4):
        np.testing.assert_allclose(matfree.mttkrp(X, Z, F, n), closed[n], rtol=1e-13, atol=1e-13)


def test_core_scaling_invariance():
    """P8: Z -> cZ scales G, which leaves the fits unchanged."""
    X, Z = make_thc(10, 30, 2)
    init = init_factors([10] * 4, 12, 5)
    a = matfree.mf_cp_als([X] * 4, Z, init, max_sweeps=10, tol=0.0)["fits"]
    b = matfree.mf_cp_als([X] * 4, 3.7 * Z, init, max_sweeps=10, tol=0.0)["fits"]
    np.testing.assert_allclose(a, b, rtol=1e-9)


def test_mode_symmetry():
    """P8: with equal X_m and symmetric Z, G_pqrs = G_qprs = G_rspq, which maps
    MTTKRPs of different modes onto each other."""
    X, Z = make_thc(7, 15, 3)
    rng = np.random.default_rng(8)
    B, C, D = (rng.standard_normal((7, 4)) for _ in range(3))
    A = rng.standard_normal((7, 4))
    m0 = matfree.mttkrp([X] * 4, Z, [A, B, C, D], 0)
    m1 = matfree.mttkrp([X] * 4, Z, [B, A, C, D], 1)
    m2 = matfree.mttkrp([X] * 4, Z, [C, D, A, B], 2)
    np.testing.assert_allclose(m1, m0, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(m2, m0, rtol=1e-12, atol=1e-14)


def test_monotone_matrix_free():
    X, Z = make_thc(12, 40, 4)
    r = matfree.mf_cp_als([X] * 4, Z, init_factors([12] * 4, 20, 9), max_sweeps=30, tol=0.0)
    f = np.array(r["fits"])
    assert r["fallbacks"] == 0
    assert np.all(f[1:] <= f[:-1] * (1 + 1e-9))
