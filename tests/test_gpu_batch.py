"""Batched (grouped) CP-ALS on the GPU: Laplace-transform row scaling,
batched == single bit for bit, per-problem parity with the oracle and
per-problem stopping."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, rel_err, torch
from oracle import lt, matfree
from synth import make_lt_system, init_factors, lt_points

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _small_batch(ts=(0.05, 1.0)):
    systems = [make_lt_system(o, v, 10 + i, rank_factor=4) for i, (o, v) in enumerate([(4, 12), (6, 18), (8, 24)])]
    return systems, list(ts)


def _init_fn(dims, r_cp, idx):
    return init_factors(dims, r_cp, 1000 + idx)


def _problems(systems, ts):
    from paper_2502_17683_amd import lt_batch_problems
    return lt_batch_problems(systems, ts, init_fn=_init_fn)


def test_lt_scale_rows_matches_oracle():
    from paper_2502_17683_amd import lt_scale_rows
    Xo, Xv, Z, eo, ev = make_lt_system(5, 9, 3, rank_factor=3)
    for t in (0.01, 0.7, 20.0):
        ref = lt.lt_factors(Xo, Xv, eo, ev, t)
        got0 = lt_scale_rows(to_dev(Xo), to_dev(eo), t, +1.0).cpu().numpy()
        got1 = lt_scale_rows(to_dev(Xv), to_dev(ev), t, -1.0).cpu().numpy()
        np.testing.assert_allclose(got0, ref[0], rtol=1e-14, atol=0)
        np.testing.assert_allclose(got1, ref[1], rtol=1e-14, atol=0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_bitwise(precision):
    from paper_2502_17683_amd import CPD, CPDBatch
    systems, ts = _small_batch()
    problems, meta = _problems(systems, ts)
    b = CPDBatch(problems, precision=precision, tol=0.0, fit_floor=0.0)
    fb = b.sweep(6)
    for i, pr in enumerate(problems):
        single = CPD(pr["X"], pr["Z"], pr["r_cp"], pr["init"], precision=precision, tol=0.0, fit_floor=0.0)
        fs = single.sweep(6)
        assert fs == fb[i], (i, meta[i])
        Fs, _ = single.factors()
        Fb, _ = b.factors(i)
        for m in range(4):
            assert torch.equal(Fs[m], Fb[m])


def test_batch_fp64_matches_oracle():
    from paper_2502_17683_amd import CPDBatch
    systems, ts = _small_batch()
    problems, meta = _problems(systems, ts)
    b = CPDBatch(problems, precision="fp64", tol=0.0, fit_floor=0.0)
    fb = b.sweep(8)
    for i, (si, t) in enumerate(meta):
        Xo, Xv, Z, eo, ev = systems[si]
        X = lt.lt_factors(Xo, Xv, eo, ev, t)
        o, v = Xo.shape[0], Xv.shape[0]
        ref = np.array(matfree.mf_cp_als(X, Z, _init_fn([o, v, o, v], 2 * (o + v), i), 8, tol=0.0,
                                         fit_floor=0.0)["fits"])
        # The matrix-free fit is f^2 = (||G||^2 - 2<G,G~> + ||G~||^2) / ||G||^2,
        # a difference of O(1) terms: its rounding floor is absolute in f^2
        # (about 1e4 eps here, summation order and ALS amplification), so the
        # comparison is on f^2 with that floor on top of 1e-10 relative.
        got = np.array(fb[i])
        assert np.all(np.abs(got ** 2 - ref ** 2) <= 2e-10 * ref ** 2 + 1e-12), (i, got, ref)


def test_batch_per_problem_stopping():
    from paper_2502_17683_amd import CPDBatch
    systems, ts = _small_batch((0.05, 0.5, 3.0))
    problems, meta = _problems(systems, ts)
    b = CPDBatch(problems, precision="fp64", tol=2e-3)
    fb = b.sweep(300)
    _, conv, sweeps = b.states()
    assert all(conv)
    for i, (si, t) in enumerate(meta):
        Xo, Xv, Z, eo, ev = systems[si]
        X = lt.lt_factors(Xo, Xv, eo, ev, t)
        o, v = Xo.shape[0], Xv.shape[0]
        ref = matfree.mf_cp_als(X, Z, _init_fn([o, v, o, v], 2 * (o + v), i), 300, tol=2e-3)["fits"]
        assert sweeps[i] == len(ref), (i, sweeps[i], len(ref))
    assert len(set(sweeps)) > 1  # problems really stopped at different sweeps


def test_lt_workload_runs():
    """The full batched workload (3 systems x 16 Laplace points = 48 CPDs of
    uneven size) in split BF16: a few sweeps, finite decreasing fits."""
    from paper_2502_17683_amd import CPDBatch
    from synth import LT_SYSTEMS
    systems = [make_lt_system(o, v, i) for i, (o, v) in enumerate(LT_SYSTEMS)]
    problems, meta = _problems(systems, lt_points())
    assert len(problems) == 48
    b = CPDBatch(problems, precision="mixed", tol=0.0, fit_floor=0.0)
    fb = np.array(b.sweep(4))
    promoted = [i for i in range(len(problems)) if b.stats(i)["fp64_path"]]
    say(f"LT batch fits after 4 sweeps: min {fb[:, -1].min():.3e} max {fb[:, -1].max():.3e}; "
        f"promoted to FP64: {[meta[i] for i in promoted]}")
    assert np.all(np.isfinite(fb))
    assert np.all(fb[:, -1] <= fb[:, 0] * (1 + 1e-6))


def test_split_autotune_on_the_laplace_batch():
    """The autotuner on a split-BF16 batch of the full Laplace workload's
    sizes: every split product kind gets a decision, the decision is one of
    the candidate launch shapes, and the tuned plan's fits (FP64-evaluated)
    equal the untuned plan's within the split rounding (different launch
    shapes only change the FP32 accumulation order)."""
    from paper_2502_17683_amd import CPDBatch
    from synth import LT_SYSTEMS
    systems = [make_lt_system(o, v, i) for i, (o, v) in enumerate(LT_SYSTEMS)]
    problems, _ = _problems(systems, (0.01, 0.3))
    a = CPDBatch(problems, precision="mixed", tol=0.0, fit_floor=0.0, autotune=True)
    log = a.autotune_log()
    say(f"split autotune log:\n{log}")
    kinds = {line.split(",")[0]: int(line.split("=")[1]) for line in log.splitlines() if line}
    for k in ("bf16core", "bf16back", "bf16proj", "f64gram"):
        assert k in kinds
    valid = {64 + 10000, 128 + 10000} | {bm + 1000 + 10000 * kp for bm in (128, 256) for kp in (1, 2, 4)}
    assert all(v in valid for k, v in kinds.items() if k.startswith("bf16"))
    fa = a.sweep(6)
    a.close()
    b = CPDBatch(problems, precision="mixed", tol=0.0, fit_floor=0.0, autotune=False)
    fb = b.sweep(6)
    b.close()
    for x, y in zip(fa, fb):
        x, y = np.array(x), np.array(y)
        assert np.all(np.abs(x - y) <= 1e-4 * y)


def test_fit_target_stops_each_problem_at_its_target():
    """cpd_desc.fit_target: each problem of an FP64 batch stops at the first
    sweep whose fit is at or below its own target (here the oracle's fit
    after 3, 7 and 11 sweeps), and its fits up to there follow the oracle."""
    from paper_2502_17683_amd import CPDBatch
    from synth import make_thc
    stops = (3, 7, 11)
    probs, refs = [], []
    for k, (n, rt, rc) in enumerate(((16, 64, 40), (24, 96, 50), (20, 80, 60))):
        X, Z = make_thc(n, rt, 30 + k)
        init = init_factors([n] * 4, rc, 1030 + k)
        probs.append(dict(X=to_dev(X), Z=to_dev(Z), r_cp=rc, init=[to_dev(f) for f in init]))
        refs.append(matfree.mf_cp_als([X] * 4, Z, init, 20, tol=0.0, fit_floor=0.0)["fits"])
    targets = [refs[i][stops[i] - 1] * (1 + 1e-12) for i in range(3)]
    b = CPDBatch(probs, precision="fp64", tol=0.0, fit_floor=0.0, fit_targets=targets)
    fits = b.sweep(20)
    _, done, sweeps = b.states()
    say(f"fit_target stops: {list(sweeps)}")
    for i in range(3):
        assert done[i] and sweeps[i] == stops[i]
        np.testing.assert_allclose(fits[i], refs[i][:stops[i]], rtol=1e-10)
    b.close()
