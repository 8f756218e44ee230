"""Pins for oracle/order3.py: the singleton fourth mode reproduces the
order-3 tensor and the three-way CP-ALS."""
import numpy as np

from oracle import dense, order3
from synth import init_factors, make_thc


def _case():
    X, Z = make_thc(7, 28, 2)
    rng = np.random.default_rng(5)
    X2 = rng.standard_normal((5, 28))
    return X, X2, Z


def test_singleton_mode_reproduces_order3_tensor():
    X, X2, Z = _case()
    G3 = order3.order3_tensor(X, X, X2, Z)
    G4 = dense.dense_tensor([X, X, X2, np.ones((1, 28))], Z)
    np.testing.assert_allclose(G4[:, :, :, 0], G3, rtol=1e-13, atol=1e-15)
    # brute force on one entry
    p, q, r = 3, 1, 4
    ref = sum(X[p, P] * X[q, P] * Z[P, Q] * X2[r, Q] for P in range(28) for Q in range(28))
    assert abs(G3[p, q, r] - ref) <= 1e-12 * abs(ref)


def test_order4_als_with_singleton_mode_is_three_way_als():
    X, X2, Z = _case()
    G3 = order3.order3_tensor(X, X, X2, Z)
    init = init_factors([7, 7, 5, 1], 6, 1002)
    ref = order3.cp3_als(G3, init[:3], 12)
    G4 = dense.dense_tensor([X, X, X2, np.ones((1, 28))], Z)
    got = dense.dense_cp_als(G4, init, 12, tol=0.0, fit_floor=0.0)["fits"]
    np.testing.assert_allclose(got, ref, rtol=1e-9)
