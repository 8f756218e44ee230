"""Pins for oracle/mp2.py: brute force, the canonical MP2 limit, and the
THC exchange term against the robust CPD+THC one for an exact CPD."""
import itertools

import numpy as np
import pytest

from oracle import dense, exchange, mp2
from synth import planted_diag_thc


def _eps(o, v, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.uniform(-1.5, -0.3, o)), np.sort(rng.uniform(0.1, 3.0, v))


def _brute_G(Xo, Xv, Z, i, a, j, b):
    acc = 0.0
    for P in range(Z.shape[0]):
        for Q in range(Z.shape[1]):
            acc += Xo[i, P] * Xv[a, P] * Z[P, Q] * Xo[j, Q] * Xv[b, Q]
    return acc


def _random(o, v, r, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((o, r)), rng.standard_normal((v, r)), rng.standard_normal((r, r)),
            *_eps(o, v, seed + 1))


@pytest.mark.parametrize("t", [0.0, 0.45])
def test_coulomb_and_exchange_brute_force(t):
    o, v = 2, 3
    Xo, Xv, Z, eo, ev = _random(o, v, 3, 7)   # non-symmetric Z
    J = K = 0.0
    for i, a, j, b in itertools.product(range(o), range(v), range(o), range(v)):
        s = np.exp(-(ev[a] + ev[b] - eo[i] - eo[j]) * t)
        g = _brute_G(Xo, Xv, Z, i, a, j, b)
        J += s * g * g
        K += s * g * _brute_G(Xo, Xv, Z, i, b, j, a)
    assert mp2.coulomb_term(Xo, Xv, Z, eo, ev, t) == pytest.approx(J, rel=1e-12)
    assert mp2.exchange_term(Xo, Xv, Z, eo, ev, t) == pytest.approx(K, rel=1e-12)


def test_fine_quadrature_gives_canonical_mp2():
    # eq. Emp2 with D = e_a + e_b - e_i - e_j; trapezoid in ln t (tails < 1e-15)
    o, v = 2, 4
    Xo, Xv, Z, eo, ev = _random(o, v, 4, 11)
    Z = Z @ Z.T  # a Coulomb-like core
    s = np.linspace(-35.0, 5.0, 801)
    ts, w = np.exp(s), (s[1] - s[0]) * np.exp(s)
    _, _, (e_j, e_k, e) = mp2.lt_mp2(Xo, Xv, Z, eo, ev, ts, w)
    G = dense.dense_tensor([Xo, Xv, Xo, Xv], Z)
    D = (ev[None, :, None, None] + ev[None, None, None, :] - eo[:, None, None, None] - eo[None, None, :, None])
    canonical = float(np.sum(G * (2.0 * G - G.transpose(0, 3, 2, 1)) / D))
    assert e == pytest.approx(canonical, rel=1e-10)
    assert e_j == pytest.approx(float(np.sum(2.0 * G * G / D)), rel=1e-10)


def test_thc_exchange_equals_robust_for_exact_cpd():
    o, v = 3, 4
    X, Zd = planted_diag_thc(o + v, 5, 13)
    Xo, Xv = X[:o], X[o:]
    eo, ev = _eps(o, v, 14)
    ts, w = np.array([0.2, 1.1]), np.array([0.4, 0.8])
    _, K, (_, e_k, _) = mp2.lt_mp2(Xo, Xv, Zd, eo, ev, ts, w)
    k1, k2 = exchange.exchange_terms(Xo, Xv, Zd, [Xo, Xv, Xo, Xv], np.diag(Zd), eo, ev, ts)
    np.testing.assert_allclose(k1, K, rtol=1e-12)
    assert exchange.robust_exchange(k1, k2, w) == pytest.approx(e_k, rel=1e-12)
