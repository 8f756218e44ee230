"""Pins for oracle/df.py: the THC form of a DF tensor is exact, and the
matrix-free CP-ALS on it follows the dense CP-ALS of the DF tensor."""
import itertools

import numpy as np

from oracle import dense, df, matfree
from synth import init_factors, make_df


def test_thc_form_is_the_df_tensor():
    n = 4
    B = make_df(n, 6, 3)
    X0, X1, Z = df.df_to_thc(B, n)
    G_thc = dense.dense_tensor([X0, X1, X0, X1], Z)
    G_df = df.df_tensor(B, n)
    for p, q, r, s in itertools.product(range(n), repeat=4):
        ref = sum(B[p * n + q, x] * B[r * n + s, x] for x in range(B.shape[1]))
        assert abs(G_df[p, q, r, s] - ref) <= 1e-13 * max(1.0, abs(ref))
    np.testing.assert_allclose(G_thc, G_df, rtol=1e-13, atol=1e-15)


def test_selection_factors():
    n = 3
    X0, X1, _ = df.df_to_thc(np.ones((n * n, 2)), n)
    assert X0.shape == (n, n * n) and X1.shape == (n, n * n)
    assert np.all(X0.sum(0) == 1) and np.all(X1.sum(0) == 1)
    assert X0[1, 1 * n + 2] == 1 and X1[2, 1 * n + 2] == 1 and X0[2, 1 * n + 2] == 0


def test_matfree_on_thc_form_follows_dense_df_als():
    n = 5
    B = make_df(n, 8, 4)
    X0, X1, Z = df.df_to_thc(B, n)
    init = init_factors([n] * 4, 6, 1004)
    ref = dense.dense_cp_als(df.df_tensor(B, n), init, 15, tol=0.0, fit_floor=0.0)
    mf = matfree.mf_cp_als([X0, X1, X0, X1], Z, init, 15, tol=0.0, fit_floor=0.0)
    np.testing.assert_allclose(mf["fits"], ref["fits"], rtol=1e-9)
