"""Pins for oracle/exchange.py: brute force, the symmetry identity, exactness
for an exact CPD, second-order robustness and the canonical limit."""
import itertools

import numpy as np
import pytest

from oracle import dense, exchange
from synth import planted_diag_thc


def _eps(o, v, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.uniform(-1.5, -0.3, o)), np.sort(rng.uniform(0.1, 3.0, v))


def _denominator(eo, ev):
    # D[i,a,j,b] = e_a + e_b - e_i - e_j
    return (ev[None, :, None, None] + ev[None, None, None, :]
            - eo[:, None, None, None] - eo[None, None, :, None])


def _brute_thc(Xo, Xv, Z, i, a, j, b):
    acc = 0.0
    for P in range(Z.shape[0]):
        for Q in range(Z.shape[1]):
            acc += Xo[i, P] * Xv[a, P] * Z[P, Q] * Xo[j, Q] * Xv[b, Q]
    return acc


def _brute_cp(F, lam, i, a, j, b):
    return sum(lam[r] * F[0][i, r] * F[1][a, r] * F[2][j, r] * F[3][b, r] for r in range(len(lam)))


def _random_case(o, v, r_thc, r_cp, seed):
    rng = np.random.default_rng(seed)
    Xo = rng.standard_normal((o, r_thc))
    Xv = rng.standard_normal((v, r_thc))
    Z = rng.standard_normal((r_thc, r_thc))  # general core: no symmetry used
    F = [rng.standard_normal((n, r_cp)) for n in (o, v, o, v)]
    lam = rng.uniform(0.5, 2.0, r_cp)
    eo, ev = _eps(o, v, seed + 1)
    return Xo, Xv, Z, F, lam, eo, ev


def _planted(o, v, r, seed):
    """Diagonal core: the THC tensor is exactly the CPD with factors
    (Xo, Xv, Xo, Xv) and weights z."""
    X, Zd = planted_diag_thc(o + v, r, seed)
    Xo, Xv = X[:o], X[o:]
    return Xo, Xv, Zd, [Xo, Xv, Xo, Xv], np.diag(Zd).copy()


@pytest.mark.parametrize("t", [0.0, 0.37])
def test_single_term_brute_force(t):
    o, v = 2, 3
    Xo, Xv, Z, F, lam, eo, ev = _random_case(o, v, 3, 2, 5)
    ref = 0.0
    for i, a, j, b in itertools.product(range(o), range(v), range(o), range(v)):
        s = np.exp(-(ev[a] + ev[b] - eo[i] - eo[j]) * t)
        ref += s * _brute_thc(Xo, Xv, Z, i, a, j, b) * _brute_cp(F, lam, i, b, j, a)
    got = exchange.k_single(Xo, Xv, Z, F, lam, eo, ev, t)
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_double_term_brute_force():
    o, v = 2, 3
    rng = np.random.default_rng(9)
    E = [rng.standard_normal((n, 3)) for n in (o, v, o, v)]
    F = [rng.standard_normal((n, 2)) for n in (o, v, o, v)]
    le, lf = rng.uniform(0.5, 2.0, 3), rng.uniform(0.5, 2.0, 2)
    ref = 0.0
    for i, a, j, b in itertools.product(range(o), range(v), range(o), range(v)):
        ref += _brute_cp(E, le, i, a, j, b) * _brute_cp(F, lf, i, b, j, a)
    assert exchange.k_double(E, le, F, lf) == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_lt_scaled_cpd_is_denominator_weighting():
    o, v = 2, 3
    _, _, _, F, lam, eo, ev = _random_case(o, v, 2, 2, 3)
    t = 0.8
    E = exchange.lt_cp_factors(F, eo, ev, t)
    for i, a, j, b in itertools.product(range(o), range(v), range(o), range(v)):
        s = np.exp(-(ev[a] + ev[b] - eo[i] - eo[j]) * t)
        assert _brute_cp(E, lam, i, a, j, b) == pytest.approx(s * _brute_cp(F, lam, i, a, j, b), rel=1e-13)


def test_symmetry_identity_scaling_moves_to_the_cpd():
    # the paper's remark: scaling the THC tensor or the CPD gives the same term
    Xo, Xv, Z, F, lam, eo, ev = _random_case(4, 6, 5, 4, 11)
    t = 1.3
    on_thc = exchange.k_single(Xo, Xv, Z, F, lam, eo, ev, t)
    on_cpd = exchange.k_single(Xo, Xv, Z, exchange.lt_cp_factors(F, eo, ev, t), lam, eo, ev, 0.0)
    assert on_cpd == pytest.approx(on_thc, rel=1e-12)


@pytest.mark.parametrize("t", [0.0, 0.25, 2.0])
def test_exact_cpd_gives_exact_exchange(t):
    o, v = 3, 4
    Xo, Xv, Z, F, lam = _planted(o, v, 5, 21)
    eo, ev = _eps(o, v, 22)
    G = dense.dense_tensor([Xo, Xv, Xo, Xv], Z)
    exact = float(np.sum(np.exp(-_denominator(eo, ev) * t) * G * G.transpose(0, 3, 2, 1)))
    k1, k2 = exchange.exchange_terms(Xo, Xv, Z, F, lam, eo, ev, [t])
    assert k1[0] == pytest.approx(exact, rel=1e-12)
    assert k2[0] == pytest.approx(exact, rel=1e-12)
    w = np.array([0.7])
    assert exchange.robust_exchange(k1, k2, w) == pytest.approx(-0.7 * exact, rel=1e-12)


def test_robust_error_is_second_order():
    o, v = 3, 4
    Xo, Xv, Z, F, lam = _planted(o, v, 5, 31)
    eo, ev = _eps(o, v, 32)
    ts, w = np.array([0.1, 0.6, 2.5]), np.array([0.3, 0.5, 0.9])
    G = dense.dense_tensor([Xo, Xv, Xo, Xv], Z)
    D = _denominator(eo, ev)
    exact = -sum(wk * np.sum(np.exp(-D * tk) * G * G.transpose(0, 3, 2, 1)) for tk, wk in zip(ts, w))
    rng = np.random.default_rng(33)
    delta = [rng.standard_normal(f.shape) for f in F]
    err_single, err_robust = [], []
    for s in (2e-3, 1e-3):
        Fs = [f + s * d for f, d in zip(F, delta)]
        k1, k2 = exchange.exchange_terms(Xo, Xv, Z, Fs, lam, eo, ev, ts)
        err_single.append(-float(np.sum(w * k1)) - exact)
        err_robust.append(exchange.robust_exchange(k1, k2, w) - exact)
    assert err_single[0] / err_single[1] == pytest.approx(2.0, rel=0.02)
    assert err_robust[0] / err_robust[1] == pytest.approx(4.0, rel=0.02)
    assert abs(err_robust[1]) < 1e-2 * abs(err_single[1])


def test_fine_quadrature_gives_canonical_exchange():
    # sum_k w_k exp(-D t_k) -> 1/D (eq. lt_D): trapezoid in s = ln t, with
    # both tails below 1e-15 for D in [0.8, 9]
    o, v = 2, 3
    Xo, Xv, Z, F, lam = _planted(o, v, 4, 41)
    eo, ev = _eps(o, v, 42)
    s = np.linspace(-35.0, 5.0, 801)
    ts, w = np.exp(s), (s[1] - s[0]) * np.exp(s)
    k1, k2 = exchange.exchange_terms(Xo, Xv, Z, F, lam, eo, ev, ts)
    G = dense.dense_tensor([Xo, Xv, Xo, Xv], Z)
    canonical = -float(np.sum(G * G.transpose(0, 3, 2, 1) / _denominator(eo, ev)))
    assert exchange.robust_exchange(k1, k2, w) == pytest.approx(canonical, rel=1e-10)


def test_absolute_bound_dominates():
    Xo, Xv, Z, F, lam, eo, ev = _random_case(4, 5, 6, 3, 51)
    k1, k2 = exchange.exchange_terms(Xo, Xv, Z, F, lam, eo, ev, [0.3, 1.0])
    a1, a2 = exchange.exchange_terms(Xo, Xv, Z, F, lam, eo, ev, [0.3, 1.0], absolute=True)
    assert np.all(a1 >= np.abs(k1)) and np.all(a2 >= np.abs(k2))
