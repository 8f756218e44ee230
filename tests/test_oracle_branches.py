"""Pins for the two run-control branches of the oracles that the GPU parity
tests lean on: the damped Cholesky retry and the stopping rule.

Damped retry (reading: one retry on V + mu I, mu = 1e-12 tr(V) / R, then
NotSPD).  Each oracle's solver is checked on matrices whose answer is known
in closed form: a diagonal V with a zero pivot (the retried solve is a
diagonal division, exact to rounding), the singular all-ones 2 x 2 matrix
(its null direction is divided by mu), an indefinite matrix (NotSPD after
the retry) and the retry switched off.  On whole runs a zero column in the
initial factor F3 makes every normal matrix singular: each mode update is
retried (4 per sweep; 2 for the tied model), the column stays exactly zero,
and the fits follow the run of rank R - 1 without that column up to the
mu-sized perturbation.

Stopping rule (Computational Details: relative change of the fit below a
tolerance; here also an absolute floor and a cadence fit_every): the rule is
checked on hand-made fit sequences with known answers, and on whole runs the
stop sweep must be the first sweep of the unstopped trajectory at which the
rule holds; the dense and matrix-free oracles must stop at the same sweep.
"""
import numpy as np
import pytest

from oracle import dense, matfree, tied
from synth import init_factors, make_thc, planted_diag_thc

SOLVERS = {
    "dense": (lambda V, M, fb: dense._normal_solve(V, M, fb), dense.NotSPDError),
    "matfree": (lambda V, M, fb: matfree.cholesky_solve(V, M, fb), matfree.NotSPD),
    "tied": (lambda V, M, fb: tied._solve(V, M, fb), tied.NotSPD),
}


@pytest.mark.parametrize("name", sorted(SOLVERS))
def test_damped_retry_diagonal_zero_pivot(name):
    solve, _ = SOLVERS[name]
    V = np.diag([4.0, 0.0, 2.0])
    M = np.array([[1.0, 3.0, -2.0], [0.5, -1.0, 6.0]])
    F, damped = solve(V, M, True)
    assert damped
    mu = 1e-12 * 6.0 / 3.0
    ref = M / np.array([4.0 + mu, mu, 2.0 + mu])[None, :]
    np.testing.assert_allclose(F, ref, rtol=4e-16 * 8, atol=0)


@pytest.mark.parametrize("name", sorted(SOLVERS))
def test_damped_retry_singular_ones(name):
    """V = [[1, 1], [1, 1]] (zero second pivot).  V + mu I has the
    eigenvectors (1, 1) and (1, -1) with eigenvalues 2 + mu and mu, mu =
    1e-12 here: (1, 1) maps to (1, 1) / (2 + mu) and (1, -1) to
    (1, -1) / mu.  The second direction has condition ~2e12, so its relative
    accuracy is ~1e-3 -- enough to tell mu from 2 mu or mu / R."""
    solve, _ = SOLVERS[name]
    V = np.ones((2, 2))
    F, damped = solve(V, np.array([[1.0, 1.0], [1.0, -1.0]]), True)
    assert damped
    mu = 1e-12
    np.testing.assert_allclose(F[0], [1 / (2 + mu)] * 2, rtol=1e-3)
    np.testing.assert_allclose(F[1], [1 / mu, -1 / mu], rtol=1e-2)


@pytest.mark.parametrize("name", sorted(SOLVERS))
def test_not_spd_after_retry_or_without_it(name):
    solve, err = SOLVERS[name]
    with pytest.raises(err):
        solve(np.array([[1.0, 2.0], [2.0, 1.0]]), np.ones((1, 2)), True)  # indefinite
    with pytest.raises(err):
        solve(np.diag([1.0, 0.0]), np.ones((1, 2)), False)  # retry switched off
    F, damped = solve(np.diag([2.0, 8.0]), np.array([[2.0, 4.0]]), False)  # SPD: no retry
    assert not damped
    np.testing.assert_allclose(F, [[1.0, 0.5]], rtol=1e-15)


def _zero_col_case(n=7, r_thc=16, r_cp=6, k=2, seed=3):
    X, Z = make_thc(n, r_thc, seed)
    init = init_factors([n] * 4, r_cp, 1000 + seed)
    init[3][:, k] = 0.0
    reduced = [np.delete(f, k, axis=1) for f in init]
    return X, Z, init, reduced, k


def test_zero_column_every_update_retried_matfree_and_dense():
    X, Z, init, reduced, k = _zero_col_case()
    sweeps = 6
    r2 = matfree.mf_cp_als([X] * 4, Z, init, sweeps, tol=0.0, fit_floor=0.0)
    G = dense.dense_tensor([X] * 4, Z)
    r1 = dense.dense_cp_als(G, init, sweeps, tol=0.0, fit_floor=0.0)
    ref = matfree.mf_cp_als([X] * 4, Z, reduced, sweeps, tol=0.0, fit_floor=0.0)
    assert ref["fallbacks"] == 0
    for r in (r1, r2):
        assert r["fallbacks"] == 4 * sweeps
        for m in range(4):
            assert np.all(r["F"][m][:, k] == 0.0)
        np.testing.assert_allclose(r["fits"], ref["fits"], rtol=1e-8)
    np.testing.assert_allclose(r1["fits"], r2["fits"], rtol=1e-10)


def test_zero_column_tied_model():
    # symmetric ALS is stable on this input (it is not on the tiny one
    # above, where mu-sized differences grow without bound)
    X, Z, init, reduced, k = _zero_col_case(n=12, r_thc=48, r_cp=30, seed=5)
    init[2][:, k] = 0.0  # the tied model starts B from init[2]
    reduced = [np.delete(f, k, axis=1) for f in init]
    sweeps = 8
    r = tied.tied_cp_als([X] * 4, Z, init, sweeps, tol=0.0, fit_floor=0.0)
    ref = tied.tied_cp_als([X] * 4, Z, reduced, sweeps, tol=0.0, fit_floor=0.0)
    assert ref["fallbacks"] == 0
    assert r["fallbacks"] == 2 * sweeps
    for m in range(4):
        assert np.all(r["F"][m][:, k] == 0.0)
    np.testing.assert_allclose(r["fits"], ref["fits"], rtol=1e-8)


RULES = {
    "dense": lambda f, tol, fl, fe: dense._stop(f, tol, fl, fe),
    "matfree": lambda f, tol, fl, fe: matfree.stops(f, tol, fl, fe),
    "tied": lambda f, tol, fl, fe: tied._rule_fires(f, tol, fl, fe),
}


@pytest.mark.parametrize("name", sorted(RULES))
def test_stopping_rule_hand_checked_sequences(name):
    rule = RULES[name]
    seq = [0.5, 0.3, 0.2, 0.19, 0.18999, 0.1899899]

    def first_stop(fits, tol, floor, every):
        for i in range(1, len(fits) + 1):
            if rule(fits[:i], tol, floor, every):
                return i
        return None

    # |0.18999 - 0.19| / 0.19 = 5.3e-5 <= 1e-4 at sweep 5; 0.01/0.2 = 5e-2 earlier
    assert first_stop(seq, 1e-4, 0.0, 1) == 5
    # tol 1e-6: 0.0000001 / 0.18999 = 5.3e-7 at sweep 6
    assert first_stop(seq, 1e-6, 0.0, 1) == 6
    assert first_stop(seq, 1e-7, 0.0, 1) is None
    # the first fit never stops by the relative rule, only by the floor
    assert first_stop([0.5, 0.5], 1.0, 0.0, 1) == 2
    assert first_stop([1e-8, 1e-8], 0.0, 1e-7, 1) == 1
    assert first_stop([0.3, 2e-7, 1e-7], 0.0, 1e-7, 1) == 3  # floor is inclusive
    # cadence 2: looked at after sweeps 2, 4, 6 and against the fit 2 sweeps back
    # sweep 4: |0.19 - 0.3| / 0.3 = 0.37; sweep 6: |0.1899899 - 0.19| / 0.19 = 5.3e-5
    assert first_stop(seq, 1e-4, 0.0, 2) == 6
    # sweep 5 satisfies the per-sweep rule but is not a rule sweep at cadence 2
    assert first_stop(seq[:5], 1e-4, 0.0, 2) is None
    # cadence 3: sweep 6 against sweep 3: |0.1899899 - 0.2| / 0.2 = 5e-2
    assert first_stop(seq, 1e-4, 0.0, 3) is None
    assert first_stop(seq, 6e-2, 0.0, 3) == 6
    # the floor is also looked at on rule sweeps only
    assert first_stop([0.3, 1e-8, 1e-8, 1e-8], 0.0, 1e-7, 3) == 3


@pytest.mark.parametrize("every", [1, 3])
def test_runs_stop_where_the_rule_first_holds(every):
    X, Z = make_thc(8, 24, 5)
    init = init_factors([8] * 4, 10, 1005)
    tol = 2e-3
    full = matfree.mf_cp_als([X] * 4, Z, init, 120, tol=0.0, fit_floor=0.0)["fits"]
    expect = next(i for i in range(1, len(full) + 1) if matfree.stops(full[:i], tol, 0.0, every))
    assert expect % every == 0 and expect > every
    r2 = matfree.mf_cp_als([X] * 4, Z, init, 120, tol=tol, fit_floor=0.0, fit_every=every)
    assert len(r2["fits"]) == expect
    G = dense.dense_tensor([X] * 4, Z)
    r1 = dense.dense_cp_als(G, init, 120, tol=tol, fit_floor=0.0, fit_every=every)
    assert len(r1["fits"]) == expect
    rt = tied.tied_cp_als([X] * 4, Z, init, 120, tol=tol, fit_floor=0.0, fit_every=every)
    ft = tied.tied_cp_als([X] * 4, Z, init, len(rt["fits"]) + 5, tol=0.0, fit_floor=0.0)["fits"]
    assert len(rt["fits"]) == next(i for i in range(1, len(ft) + 1) if tied._rule_fires(ft[:i], tol, 0.0, every))


def test_planted_cpd_stops_at_the_floor():
    """A planted exact CPD (diagonal core) started near the truth reaches the
    matrix-free floor; the run stops at the first sweep at or below it."""
    X, Z = planted_diag_thc(8, 6, 3)
    truth = X * np.diag(Z)[None, :] ** 0.25
    rng = np.random.default_rng(4)
    init = [truth + 1e-3 * rng.standard_normal(truth.shape) for _ in range(4)]
    full = matfree.mf_cp_als([X] * 4, Z, init, 60, tol=0.0, fit_floor=0.0)["fits"]
    floor = 1e-6
    first = next(i for i, f in enumerate(full, 1) if f <= floor)
    assert first > 1
    r = matfree.mf_cp_als([X] * 4, Z, init, 60, tol=0.0, fit_floor=floor)
    assert len(r["fits"]) == first and r["fits"][-1] <= floor
