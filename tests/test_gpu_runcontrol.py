"""Run control on the GPU through the C-ABI: the stopping rule at a fit
cadence (fit_every) in FP64 and split BF16, against the oracle at the same
cadence, and a dataflow solve wait that gives up inside a whole sweep."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev
from oracle import matfree
from synth import make_thc, init_factors

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _plan(X, Z, init, r_cp, **kw):
    from paper_2502_17683_amd import CPD
    return CPD(to_dev(X), to_dev(Z), r_cp, [to_dev(f) for f in init], **kw)


def _first_rule_sweep(fits, tol, every):
    """First sweep (1-based) at which the stopping rule fires on a given
    sequence of evaluated fits (the oracle's own rule)."""
    for i in range(1, len(fits) + 1):
        if matfree.stops(fits[:i], tol, 0.0, every):
            return i
    return None


@pytest.mark.parametrize("every", [1, 3])
def test_fp64_stop_sweep_at_cadence_matches_oracle(every):
    X, Z = make_thc(20, 80, 1)
    init = init_factors([20] * 4, 60, 1001)
    tol = 5e-3
    c = _plan(X, Z, init, 60, tol=tol, fit_floor=0.0, fit_every=every)
    fits = c.sweep(300)
    ref = matfree.mf_cp_als([X] * 4, Z, init, 300, tol=tol, fit_floor=0.0, fit_every=every)["fits"]
    say(f"fp64 cadence {every}: gpu stopped after {len(fits)} sweeps, oracle after {len(ref)}")
    assert len(fits) == len(ref) < 300
    assert len(fits) % every == 0
    assert np.all(np.abs(np.array(fits) - np.array(ref)) <= 1e-10 * np.array(ref))
    assert c.stats()["converged"] == 1
    assert c.sweep(3) == []


def test_mixed_stop_sweep_at_cadence():
    """Split BF16 evaluates its fit every 4th sweep; the device stops at the
    first fit sweep where the rule holds on its own reported fits, and (on
    this input, where split-BF16 and FP64 fits agree to ~1e-6 while the rule
    quantity crosses tol by far more) at the oracle's stop sweep for the
    same cadence."""
    X, Z = make_thc(20, 80, 1)
    init = init_factors([20] * 4, 60, 1001)
    tol, every = 5e-3, 4
    c = _plan(X, Z, init, 60, tol=tol, fit_floor=0.0, fit_every=every, precision="mixed")
    fits = c.sweep(300)
    assert all((f >= 0) == ((i + 1) % every == 0) for i, f in enumerate(fits))
    evaluated = [f for f in fits if f >= 0]
    dense_seq = []  # the evaluated fits at their sweep positions, for the rule
    for i, f in enumerate(fits):
        dense_seq.append(f if f >= 0 else float("nan"))
    host = None
    for i in range(every, len(fits) + 1, every):
        cur, prev = dense_seq[i - 1], dense_seq[i - 1 - every] if i > every else None
        if prev is not None and abs(cur - prev) <= tol * prev:
            host = i
            break
    ref = matfree.mf_cp_als([X] * 4, Z, init, 300, tol=tol, fit_floor=0.0, fit_every=every)["fits"]
    say(f"mixed cadence {every}: gpu stopped after {len(fits)} sweeps ({len(evaluated)} fits), "
        f"host rule {host}, oracle {len(ref)}")
    assert host == len(fits) < 300
    assert len(fits) == len(ref)
    assert c.stats()["converged"] == 1


def test_batch_fp64_cadence_stops_each_problem_like_the_oracle():
    from paper_2502_17683_amd import CPDBatch
    shapes = [(16, 64, 40, 2), (24, 96, 50, 3), (20, 80, 60, 1)]
    probs, refs = [], []
    tol, every = 5e-3, 2
    for n, rt, rc, seed in shapes:
        X, Z = make_thc(n, rt, seed)
        init = init_factors([n] * 4, rc, 1000 + seed)
        probs.append(dict(X=to_dev(X), Z=to_dev(Z), r_cp=rc, init=[to_dev(f) for f in init]))
        refs.append(matfree.mf_cp_als([X] * 4, Z, init, 300, tol=tol, fit_floor=0.0, fit_every=every)["fits"])
    b = CPDBatch(probs, precision="fp64", tol=tol, fit_floor=0.0, fit_every=every)
    fits = b.sweep(300)
    _, done, sweeps = b.states()
    say(f"batch cadence {every}: sweeps {list(sweeps)} oracle {[len(r) for r in refs]}")
    for i, r in enumerate(refs):
        assert done[i] and sweeps[i] == len(r)
        np.testing.assert_allclose(fits[i], r, rtol=1e-10)
    b.close()


def test_stalled_solve_wait_ends_the_run():
    """A dataflow wait that gives up (a zero-poll limit set from the host;
    every kernel still exits) inside a whole sweep: the call reports
    CPD_ERR_HIP, the problem is marked stopped, later sweeps run nothing and
    report the same error, and a new plan with the default limit is right."""
    from paper_2502_17683_amd import CpdError, test_flow_spin_limit
    X, Z = make_thc(60, 320, 7)
    init = init_factors([60] * 4, 300, 1007)
    ref = matfree.mf_cp_als([X] * 4, Z, init, 3, tol=0.0, fit_floor=0.0)["fits"]
    say("whole sweeps with a zero-poll dataflow wait limit")
    prev = test_flow_spin_limit(0)
    try:
        c = _plan(X, Z, init, 300, tol=0.0, fit_floor=0.0, use_graph=False)
        try:
            fits = c.sweep(3)
            outcome = "solved"
            np.testing.assert_allclose(fits, ref, rtol=1e-10)
        except CpdError as e:
            outcome = str(e)
            assert e.code == -2
            with pytest.raises(CpdError) as e2:
                c.sweep(2)
            assert e2.value.code == -2
    finally:
        test_flow_spin_limit(-1)
    say(f"zero-poll whole-sweep outcome: {outcome}")
    if outcome != "solved":
        from paper_2502_17683_amd import _lib
        import ctypes
        s = _lib.CpdStats()
        assert c.lib.cpd_stats(c.plan, ctypes.byref(s)) == 0
        assert s.converged == 1 and (s.flags & 4)
        assert s.sweeps <= 1
    c.close()
    d = _plan(X, Z, init, 300, tol=0.0, fit_floor=0.0, use_graph=False)
    np.testing.assert_allclose(d.sweep(3), ref, rtol=1e-10)
