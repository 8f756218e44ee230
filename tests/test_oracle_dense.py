"""Pins for O1 (oracle/dense.py): brute force, planted recovery, monotonicity."""
import itertools

import numpy as np
import pytest

from oracle import dense


def _brute_tensor(X, Z):
    X0, X1, X2, X3 = X
    n = [x.shape[0] for x in X]
    R = Z.shape[0]
    G = np.zeros(n)
    for p, q, r, s in itertools.product(*[range(k) for k in n]):
        acc = 0.0
        for P in range(R):
            for Q in range(R):
                acc += X0[p, P] * X1[q, P] * Z[P, Q] * X2[r, Q] * X3[s, Q]
        G[p, q, r, s] = acc
    return G


def _brute_mttkrp(G, F, n):
    R = F[0].shape[1]
    M = np.zeros((G.shape[n], R))
    for idx in itertools.product(*[range(k) for k in G.shape]):
        for k in range(R):
            prod = G[idx]
            for m in range(4):
                if m != n:
                    prod *= F[m][idx[m], k]
            M[idx[n], k] += prod
    return M


def test_dense_tensor_brute_force():
    rng = np.random.default_rng(1)
    X = [rng.standard_normal((d, 3)) for d in (2, 3, 2, 3)]
    Z = rng.standard_normal((3, 3))  # general (non-symmetric) core
    np.testing.assert_allclose(dense.dense_tensor(X, Z), _brute_tensor(X, Z), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n", range(4))
def test_dense_mttkrp_brute_force(n):
    rng = np.random.default_rng(2 + n)
    G = rng.standard_normal((2, 3, 4, 3))
    F = [rng.standard_normal((d, 3)) for d in G.shape]
    np.testing.assert_allclose(dense.dense_mttkrp(G, F, n), _brute_mttkrp(G, F, n), rtol=1e-12, atol=1e-12)


def test_reconstruct_brute_force():
    rng = np.random.default_rng(7)
    lam = rng.uniform(0.5, 2, 3)
    F = [rng.standard_normal((d, 3)) for d in (2, 3, 2, 4)]
    G = np.zeros((2, 3, 2, 4))
    for idx in itertools.product(*[range(k) for k in G.shape]):
        G[idx] = sum(lam[k] * F[0][idx[0], k] * F[1][idx[1], k] * F[2][idx[2], k] * F[3][idx[3], k] for k in range(3))
    np.testing.assert_allclose(dense.reconstruct(lam, F), G, rtol=1e-13, atol=1e-14)
    assert dense.dense_fit(G, lam, F) < 1e-14


def test_planted_rank5_recovery():
    """P5: a random rank-5 tensor (N=10) is recovered exactly from a random
    start in most seeds, with congruent factors."""
    ok = 0
    seeds = range(10)
    for seed in seeds:
        rng = np.random.default_rng(100 + seed)
        true = [rng.standard_normal((10, 5)) for _ in range(4)]
        G = dense.reconstruct(np.ones(5), true)
        init = [rng.standard_normal((10, 5)) for _ in range(4)]
        res = dense.dense_cp_als(G, init, max_sweeps=500, tol=0.0, fit_floor=1e-12)
        if res["fits"][-1] < 1e-10:
            # congruence after matching columns
            Fn = [t / np.linalg.norm(t, axis=0) for t in true]
            C = np.abs(res["F"][0].T @ Fn[0]) * np.abs(res["F"][1].T @ Fn[1]) * \
                np.abs(res["F"][2].T @ Fn[2]) * np.abs(res["F"][3].T @ Fn[3])
            assert np.all(C.max(axis=1) > 1 - 1e-8)
            ok += 1
    assert ok >= 9


def test_monotone_fit():
    """P7: every block update is an exact least-squares minimiser, so the fit
    never increases (no fallbacks in this run)."""
    rng = np.random.default_rng(5)
    X = [rng.standard_normal((6, 10)) for _ in range(4)]
    Z = rng.standard_normal((10, 10))
    G = dense.dense_tensor(X, Z)
    init = [rng.standard_normal((6, 8)) for _ in range(4)]
    res = dense.dense_cp_als(G, init, max_sweeps=40, tol=0.0)
    assert res["fallbacks"] == 0
    f = np.array(res["fits"])
    assert np.all(f[1:] <= f[:-1] * (1 + 1e-12))
