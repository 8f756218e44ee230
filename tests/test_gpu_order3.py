"""Order-3 THC-like tensors on the GPU: the order-4 plan with a singleton
fourth mode (n3 = 1, X3 = ones) against the three-way CP-ALS oracle."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, torch
from oracle import order3
from synth import init_factors, make_thc

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-3)])
def test_order3_through_singleton_mode(precision, tol):
    from paper_2502_17683_amd import CPD
    n, n2, rt, rc = 20, 14, 80, 30
    X, Z = make_thc(n, rt, 21)
    X2 = np.random.default_rng(22).uniform(0.0, 1.0, (n2, rt))
    ones = np.ones((1, rt))
    init = init_factors([n, n, n2, 1], rc, 1021)
    say(f"[order3] {precision}: n=({n},{n},{n2}) R_thc={rt} R_cp={rc}")
    Xd = to_dev(X)
    c = CPD([Xd, Xd, to_dev(X2), to_dev(ones)], to_dev(Z), rc, [to_dev(f) for f in init], precision=precision,
            tol=0.0, fit_floor=0.0)
    fits = np.array(c.sweep(20))
    c.close()
    ref = np.array(order3.cp3_als(order3.order3_tensor(X, X, X2, Z), init[:3], 20))
    err = np.abs(fits - ref) / ref
    say(f"[order3] {precision}: max fit rel err {err.max():.2e}, last fit {fits[-1]:.4e}")
    assert np.all(err <= tol)
