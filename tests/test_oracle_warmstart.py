"""Pins of the warm-start oracle (oracle/warmstart.py): brute-force
feature loops, closed forms, invariances, the planted diagonal core and
planted label recovery."""
import math

import numpy as np

from oracle import warmstart as ws, matfree
from synth import make_thc, planted_diag_thc


def _brute_raw(X0, Z):
    n, R = X0.shape
    lg = lambda v: math.log(max(v, 1e-300))
    out = np.zeros((R, 8))
    for P in range(R):
        S_PP = sum(X0[p, P] ** 2 for p in range(n))
        S_row = [sum(X0[p, P] * X0[p, Q] for p in range(n)) for Q in range(R)]
        x4 = sum(X0[p, P] ** 4 for p in range(n))
        out[P, 0] = lg(Z[P, P])
        out[P, 1] = lg(sum(abs(Z[P, Q]) for Q in range(R)))
        out[P, 2] = lg(S_PP)
        out[P, 3] = lg(sum(s * s for s in S_row))
        out[P, 4] = lg(max(abs(X0[p, P]) for p in range(n)))
        out[P, 5] = S_PP ** 2 / (n * x4) if x4 > 0 else 0.0
        out[P, 6] = lg(sum(S_row[Q] ** 2 * abs(Z[P, Q]) for Q in range(R)))
        out[P, 7] = lg(Z[P, P] * S_PP ** 2)
    return out


def test_raw_features_match_loops():
    X, Z = make_thc(6, 14, 3)
    Z = Z + 0.01 * np.arange(14)[None, :]  # non-symmetric: pins the row (P) axis
    np.testing.assert_allclose(ws.raw_features(X, Z), _brute_raw(X, Z), rtol=1e-12, atol=1e-12)


def test_participation_ratio_closed_forms():
    n = 5
    X = np.zeros((n, 3))
    X[2, 0] = 3.0            # one-hot column: 1/n
    X[:, 1] = -0.7           # flat column: 1
    X[:, 2] = [1, 1, 0, 0, 0]  # two equal entries: 2/n
    f = ws.raw_features(X, np.eye(3))
    np.testing.assert_allclose(f[:, 5], [1 / n, 1.0, 2 / n], rtol=1e-15)


def test_standardised_features_invariances():
    X, Z = make_thc(10, 40, 1)
    f = ws.features(X, Z)
    np.testing.assert_allclose(f.mean(axis=0), 0.0, atol=1e-13)
    # the softened kernel has a constant diagonal Z_PP = 2: feature 0 is
    # constant up to rounding and standardises to 0, the others to unit variance
    assert np.all(f[:, 0] == 0)
    np.testing.assert_allclose(np.sqrt((f[:, 1:] ** 2).mean(axis=0)), 1.0, rtol=1e-13)
    np.testing.assert_allclose(ws.features(3.7 * X, Z), f, atol=1e-12)
    np.testing.assert_allclose(ws.features(X, 0.02 * Z), f, atol=1e-12)
    perm = np.random.default_rng(0).permutation(40)
    np.testing.assert_allclose(ws.features(X[:, perm], Z[np.ix_(perm, perm)]), f[perm], atol=1e-12)
    c = np.ones((5, 3))
    assert np.all(ws.standardise(c) == 0)  # constant feature -> 0


def test_selection_order_and_ties():
    s = np.array([0.5, 2.0, 0.5, -1.0, 2.0])
    assert list(ws.selection_order(s)) == [1, 4, 0, 2, 3]


def test_planted_diagonal_core_is_exact_after_selection():
    """With Z = diag(z), G = sum_P z_P x_P^(x4): choosing every grid point
    with ell_P = log(z_P)/4 gives an exact CPD."""
    n, R = 8, 6
    X, Z = planted_diag_thc(n, R, 2)
    z = np.diag(Z)
    s = np.random.default_rng(1).standard_normal(R)
    init = ws.select_init([X] * 4, s, 0.25 * np.log(z), R)
    from oracle import dense
    G = dense.dense_tensor([X] * 4, Z)
    Gt = dense.reconstruct(np.ones(R), init)
    assert np.linalg.norm(G - Gt) <= 1e-13 * np.linalg.norm(G)
    r = matfree.mf_cp_als([X] * 4, Z, init, 1, tol=0.0, fit_floor=0.0)
    assert r["fits"][0] <= 1e-7
    # the heuristic score is the diagonal contribution z_P S_PP^2
    np.testing.assert_allclose(ws.heuristic_scores(X, Z), np.log(z * (X ** 2).sum(0) ** 2), rtol=1e-14)


def test_labels_recover_planted_columns_and_scales():
    n, R_t, R_c = 12, 9, 5
    X, _ = make_thc(n, R_t, 4)
    Xs = [X, 1.3 * X, X, 0.6 * X]
    rng = np.random.default_rng(2)
    chosen = rng.choice(R_t, R_c, replace=False)
    c = rng.uniform(0.2, 3.0, (4, R_c)) * rng.choice([-1, 1], (4, R_c))
    F = [Xs[m][:, chosen] * c[m] for m in range(4)]
    norms = [np.sqrt((f ** 2).sum(0)) for f in F]
    lam = np.prod(norms, axis=0)
    Fn = [F[m] / norms[m] for m in range(4)]
    y, ell, mask = ws.match_labels(Xs, Fn, lam)
    assert set(np.nonzero(y)[0]) == set(chosen)
    assert np.array_equal(mask, y)
    np.testing.assert_allclose(ell[chosen], np.log(np.abs(c)).mean(axis=0), rtol=1e-12, atol=1e-12)


def _iterative_max_matching(A):
    R, Pn = A.shape
    match = np.full(R, -1)
    free_r, free_c = set(range(R)), set(range(Pn))
    while free_r and free_c:
        best = None
        for k in sorted(free_r):
            for P in sorted(free_c):
                if best is None or A[k, P] > A[best]:
                    best = (k, P)
        match[best[0]] = best[1]
        free_r.discard(best[0]); free_c.discard(best[1])
    return match


def test_greedy_matching_against_exhaustive_loop():
    rng = np.random.default_rng(9)
    for trial in range(30):
        R, Pn = rng.integers(1, 6), rng.integers(1, 8)
        A = rng.integers(0, 4, (R, Pn)).astype(np.float64)  # many ties
        assert np.array_equal(ws.greedy_match(A), _iterative_max_matching(A)), A


def test_blend_with_random_guess():
    """X-part plus an orthogonal random part: the column norm is
    exp(ell) ||x|| sqrt(1 + sigma^2) and the component along x is exp(ell) x."""
    rng = np.random.default_rng(6)
    n, R_t, R_c = 9, 7, 4
    X = [rng.standard_normal((n, R_t)) for _ in range(4)]
    s = rng.standard_normal(R_t)
    ell = 0.2 * rng.standard_normal(R_t)
    order = ws.selection_order(s)[:R_c]
    noise = []
    for m in range(4):
        Rm = 3.0 * rng.standard_normal((n, R_c))
        x = X[m][:, order]
        Rm -= x * ((x * Rm).sum(0) / (x * x).sum(0))  # orthogonal to its grid column
        noise.append(Rm)
    sigma = 0.35
    F = ws.select_init(X, s, ell, R_c, noise=noise, sigma=sigma)
    F0 = ws.select_init(X, s, ell, R_c)
    for m in range(4):
        x = X[m][:, order]
        e = np.exp(ell[order])
        np.testing.assert_allclose(np.linalg.norm(F[m], axis=0),
                                   e * np.linalg.norm(x, axis=0) * np.sqrt(1 + sigma ** 2), rtol=1e-13)
        np.testing.assert_allclose((F[m] * x).sum(0) / (x * x).sum(0), e, rtol=1e-13)
        np.testing.assert_allclose(F0[m], x * e, rtol=1e-15)
    assert np.array_equal(ws.select_init(X, s, ell, R_c, noise=noise, sigma=0.0)[0], F0[0])
