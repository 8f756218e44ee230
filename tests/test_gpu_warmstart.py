"""Learned warm start on the GPU against the oracle: features, selection,
labels, the network's FP32 forward/backward/Adam (gradients to 1e-4) and
BF16 inference (within its rounding bound), the fallback chain, and a
small end-to-end run showing that the warm start reaches the random-init
fit in fewer sweeps."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev, torch
from oracle import matfree, mlp as omlp, warmstart as ows
from synth import make_thc, init_factors, mlp_init_params, minibatch_order

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("n,r_thc,seed", [(12, 60, 0), (30, 300, 1), (40, 513, 2)])
def test_features_match_oracle(n, r_thc, seed):
    from paper_2502_17683_amd import ws_features
    X, Z = make_thc(n, r_thc, seed)
    say(f"features n={n} r_thc={r_thc} seed={seed}")
    feat, heur = ws_features(to_dev(X), to_dev(Z))
    ref = ows.features(X, Z)
    got = feat.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-6)
    np.testing.assert_allclose(heur.cpu().numpy(), ows.heuristic_scores(X, Z), rtol=1e-12, atol=0)


def test_features_of_scaled_lt_factor():
    """Occupied-orbital factor scaled by exp(eps t): features stay defined."""
    from paper_2502_17683_amd import ws_features
    from synth import make_lt_system
    from oracle import lt
    Xo, Xv, Z, eo, ev = make_lt_system(6, 18, 5, rank_factor=4)
    X0 = lt.lt_factors(Xo, Xv, eo, ev, 3.0)[0]
    feat, heur = ws_features(to_dev(X0), to_dev(Z))
    np.testing.assert_allclose(feat.cpu().numpy(), ows.features(X0, Z), rtol=0, atol=2e-6)
    np.testing.assert_allclose(heur.cpu().numpy(), ows.heuristic_scores(X0, Z), rtol=1e-12)


@pytest.mark.parametrize("r_thc,r_cp", [(70, 1), (70, 33), (300, 240), (64, 64)])
def test_select_init_matches_oracle(r_thc, r_cp):
    from paper_2502_17683_amd import ws_select_init
    rng = np.random.default_rng(r_thc + r_cp)
    X = [rng.standard_normal((n, r_thc)) for n in (7, 9, 7, 9)]
    s = np.round(rng.standard_normal(r_thc) * 4) / 4  # coarse: many ties
    s = s.astype(np.float32)
    ell = (0.3 * rng.standard_normal(r_thc)).astype(np.float32)
    noise = [rng.standard_normal((n, r_cp)) for n in (7, 9, 7, 9)]
    say(f"select r_thc={r_thc} r_cp={r_cp}")
    # exp of the same FP32 input may differ by one ulp between libraries,
    # and the blend's norms by their summation order: a few ulps apart,
    # while a wrong column would differ at O(1).
    for nz, sigma in ((None, 0.0), (noise, 0.4)):
        got = ws_select_init([to_dev(x) for x in X], s, ell, r_cp, noise=nz, sigma=sigma)
        ref = ows.select_init(X, s.astype(np.float64), ell.astype(np.float64), r_cp, noise=nz, sigma=sigma)
        for m in range(4):
            np.testing.assert_allclose(got[m].cpu().numpy(), ref[m], rtol=1e-15, atol=1e-15 * np.abs(ref[m]).max())


def test_labels_match_oracle():
    from paper_2502_17683_amd import ws_labels
    n, r_thc, r_cp = 14, 70, 50
    X, Z = make_thc(n, r_thc, 3)
    r = matfree.mf_cp_als([X] * 4, Z, init_factors([n] * 4, r_cp, 1003), 6, tol=0.0, fit_floor=0.0)
    F, lam = r["F"], r["lam"]
    y, ell, mask = ws_labels(to_dev(X), [to_dev(f) for f in F], to_dev(lam))
    ry, rell, rmask = ows.match_labels([X] * 4, F, lam)
    assert np.array_equal(y.cpu().numpy(), ry.astype(np.float32))
    assert np.array_equal(mask.cpu().numpy(), rmask.astype(np.float32))
    np.testing.assert_allclose(ell.cpu().numpy(), rell, rtol=1e-6, atol=1e-6)
    assert int(ry.sum()) == r_cp


def test_labels_recover_planted_columns():
    from paper_2502_17683_amd import ws_labels
    n, r_thc, r_cp = 20, 90, 40
    X, _ = make_thc(n, r_thc, 8)
    rng = np.random.default_rng(3)
    chosen = rng.choice(r_thc, r_cp, replace=False)
    c = rng.uniform(0.3, 2.0, (4, r_cp))
    F = [X[:, chosen] * c[m] for m in range(4)]
    nr = [np.sqrt((f ** 2).sum(0)) for f in F]
    lam = np.prod(nr, axis=0)
    y, ell, mask = ws_labels(to_dev(X), [to_dev(F[m] / nr[m]) for m in range(4)], to_dev(lam))
    assert set(np.nonzero(y.cpu().numpy())[0]) == set(chosen)
    np.testing.assert_allclose(ell.cpu().numpy()[chosen], np.log(c).mean(0), rtol=1e-6, atol=1e-6)


def _mlp_case(rows, total, seed):
    rng = np.random.default_rng(seed)
    theta = mlp_init_params(seed).astype(np.float64)
    theta += 0.05 * rng.standard_normal(theta.size)
    theta = theta.astype(np.float32)
    x = rng.standard_normal((total, 8)).astype(np.float32)
    y = (rng.random(total) < 0.5).astype(np.float32)
    ell = rng.standard_normal(total).astype(np.float32)
    mask = (rng.random(total) < 0.6).astype(np.float32)
    idx = rng.choice(total, rows, replace=False).astype(np.int32)
    return theta, x, y, ell, mask, idx


@pytest.mark.parametrize("rows,total", [(1, 5), (300, 300), (700, 1000)])
def test_mlp_forward_loss_backward_match_oracle(rows, total):
    from paper_2502_17683_amd import WarmStartMLP
    theta, x, y, ell, mask, idx = _mlp_case(rows, total, rows)
    say(f"mlp rows={rows} total={total}")
    net = WarmStartMLP(theta)
    d = lambda a, dt=torch.float32: torch.as_tensor(a, dtype=dt, device="cuda")
    xi = d(idx, torch.int32)
    out = net.forward(d(x), xi)
    loss, dout = net.loss(out, d(y), d(ell), d(mask), xi)
    g = net.backward(d(x), dout, xi).cpu().numpy().astype(np.float64)
    th = theta.astype(np.float64)
    rout, cache = omlp.forward(th, x[idx].astype(np.float64))
    rloss, rdout = omlp.loss(rout, y[idx].astype(np.float64), ell[idx].astype(np.float64),
                             mask[idx].astype(np.float64))
    rg = omlp.backward(th, cache, rdout)
    np.testing.assert_allclose(out.cpu().numpy(), rout, rtol=0, atol=2e-5 * max(1.0, np.abs(rout).max()))
    assert abs(float(loss.item()) - rloss) <= 1e-5 * abs(rloss)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in omlp.SHAPES])
    for b in range(len(omlp.SHAPES)):
        gb, rb = g[offs[b]:offs[b + 1]], rg[offs[b]:offs[b + 1]]
        scale = np.abs(rb).max()
        err = np.abs(gb - rb).max()
        say(f"  block {b}: max |g| {scale:.3e} max err {err:.3e}")
        assert err <= 1e-4 * scale + 1e-12, (b, err, scale)


def test_adam_matches_oracle():
    from paper_2502_17683_amd import WarmStartMLP
    theta = mlp_init_params(11)
    net = WarmStartMLP(theta)
    rng = np.random.default_rng(5)
    th, m, v = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    for step in range(1, 4):
        g = rng.standard_normal(theta.size).astype(np.float32)
        net.grads.copy_(torch.as_tensor(g, device="cuda"))
        net.adam(lr=1e-2)
        th, m, v = omlp.adam_step(th, g.astype(np.float64), m, v, step, 1e-2)
    np.testing.assert_allclose(net.params.cpu().numpy(), th, rtol=0, atol=2e-6)


@pytest.mark.parametrize("rows", [1, 64, 500, 2001])
def test_infer_bf16_within_rounding_bound(rows):
    """BF16 inference against the FP64 forward: h1 and W2 are rounded to
    BF16 (unit roundoff u = 2^-9, taken as 2^-8 for slack), so
    |d a2| <= 2u (|h1| |W2|), |d h2| <= 1.1 |d a2| (|silu'| <= 1.1) and
    |d out| <= |d h2| |W3|; FP32 accumulation adds far less."""
    from paper_2502_17683_amd import WarmStartMLP
    theta, x, *_ = _mlp_case(rows, rows, 100 + rows)
    net = WarmStartMLP(theta)
    out = net.infer_bf16(torch.as_tensor(x, device="cuda")).cpu().numpy()
    th = theta.astype(np.float64)
    rout, (_, a1, h1, a2, h2) = omlp.forward(th, x.astype(np.float64))
    W1, b1, W2, b2, W3, b3 = omlp.unpack(th)
    u = 2.0 ** -8
    da2 = 2 * u * (np.abs(h1) @ np.abs(W2))
    bound = (1.1 * da2) @ np.abs(W3)
    err = np.abs(out - rout)
    say(f"bf16 rows={rows}: max err {err.max():.3e}, max bound {bound.max():.3e}")
    assert np.all(err <= bound + 1e-5)


def test_ws_init_fallback_chain():
    from paper_2502_17683_amd import ws_init, WarmStartMLP
    n, r_thc, r_cp = 10, 50, 40
    X, Z = make_thc(n, r_thc, 4)
    init0 = init_factors([n] * 4, r_cp, 1004)
    # no network: heuristic (FP64 scores, scale 1), blended with the random guess
    got, src = ws_init(to_dev(X), to_dev(Z), r_cp, noise=[to_dev(f) for f in init0], sigma=0.25)
    assert src == "heuristic"
    ref = ows.select_init([X] * 4, ows.heuristic_scores(X, Z), np.zeros(r_thc), r_cp, noise=init0, sigma=0.25)
    for m in range(4):
        np.testing.assert_allclose(got[m].cpu().numpy(), ref[m], rtol=1e-15, atol=1e-15 * np.abs(ref[m]).max())
    got, src = ws_init(to_dev(X), to_dev(Z), r_cp, sigma=0.0)
    ref = ows.select_init([X] * 4, ows.heuristic_scores(X, Z), np.zeros(r_thc), r_cp)
    for m in range(4):
        np.testing.assert_array_equal(got[m].cpu().numpy(), ref[m])
    # a network with non-finite output falls back to the heuristic
    bad = mlp_init_params(1)
    bad[-2:] = np.nan
    net = WarmStartMLP(bad)
    got, src = ws_init(to_dev(X), to_dev(Z), r_cp, packed=net.pack())
    assert src == "heuristic"
    # a working network: its own selection, which equals select_init of its scores
    net = WarmStartMLP(mlp_init_params(2))
    packed = net.pack()
    got, src = ws_init(to_dev(X), to_dev(Z), r_cp, packed=packed, noise=[to_dev(f) for f in init0])
    assert src == "network"
    from paper_2502_17683_amd import ws_features, ws_select_init
    feat, _ = ws_features(to_dev(X), to_dev(Z))
    out = net.infer_bf16(feat, packed)
    again = ws_select_init(to_dev(X), out[:, 0].contiguous(), out[:, 1].contiguous(), r_cp,
                           noise=[to_dev(f) for f in init0], sigma=0.25)
    for m in range(4):
        assert torch.equal(got[m], again[m])
    # non-finite core: neither score is usable, init is left unchanged
    Zn = Z.copy()
    Zn[3, 3] = np.nan
    got, src = ws_init(to_dev(X), to_dev(Zn), r_cp, noise=[to_dev(f) for f in init0])
    assert src == "unchanged"
    for m in range(4):
        np.testing.assert_array_equal(got[m].cpu().numpy(), init0[m])


def _sweeps_to(fits, target):
    hit = np.nonzero(np.asarray(fits) <= target)[0]
    return int(hit[0]) + 1 if len(hit) else None


def test_warm_start_training_and_gain():
    """Train on converged CPDs of small problems (the 5:4 THC-to-CP rank
    ratio of the warm-start workload), then on held-out problems count the
    sweeps the learned, heuristic and random starts need to reach the
    random start's best fit (1 + 1e-4): the learned start needs at most
    half the random start's median, and at most 1.5x the heuristic's."""
    from paper_2502_17683_amd import WarmStartMLP, CPDBatch, training_set, ws_init
    n, r_thc, r_cp = 24, 120, 96
    train = []
    for k in range(48):
        X, Z = make_thc(n, r_thc, 10000 + k)
        train.append({"X": X, "Z": Z, "r_cp": r_cp, "init": init_factors([n] * 4, r_cp, 11000 + k)})
    data = training_set(train, sweeps=120, tol=1e-4)
    feat, y, ell, mask = data
    say(f"training rows {feat.shape[0]}, positive fraction {float(y.mean()):.3f}")
    net = WarmStartMLP(mlp_init_params(7))
    order = minibatch_order(feat.shape[0], 3)
    losses = net.train(data, order, batch_rows=1024, lr=2e-3, epochs=25)
    say(f"loss: first {losses[:3]}, last {losses[-3:]}")
    assert np.all(np.isfinite(losses))
    assert losses[-5:].mean() < 0.8 * losses[:5].mean()
    packed = net.pack()
    budget = 150
    probs, kinds = [], []
    for k in range(6):
        X, Z = make_thc(n, r_thc, 20000 + k)
        rnd = init_factors([n] * 4, r_cp, 21000 + k)
        learned, src = ws_init(to_dev(X), to_dev(Z), r_cp, packed=packed, noise=rnd)
        assert src == "network"
        heur, _ = ws_init(to_dev(X), to_dev(Z), r_cp, noise=rnd)
        for kind, init in (("random", rnd), ("learned", learned), ("heuristic", heur)):
            probs.append({"X": X, "Z": Z, "r_cp": r_cp, "init": init})
            kinds.append((k, kind))
    b = CPDBatch(probs, precision="fp64", tol=0.0, fit_floor=0.0)
    fits = b.sweep(budget)
    res = {}
    for (k, kind), f in zip(kinds, fits):
        res.setdefault(k, {})[kind] = np.asarray(f)
    sweeps = {"random": [], "learned": [], "heuristic": []}
    for k, r in res.items():
        target = r["random"].min() * (1 + 1e-4)
        s = {kind: _sweeps_to(r[kind], target) for kind in r}
        say(f"held-out {k}: sweeps to random-best fit {s}; final fits "
            f"{ {kind: float(v[-1]) for kind, v in r.items()} }")
        for kind in sweeps:
            sweeps[kind].append(s[kind] or budget + 1)
    med = {kind: float(np.median(v)) for kind, v in sweeps.items()}
    say(f"median sweeps to the random start's best fit: {med}")
    reached = sum(v <= budget for v in sweeps["learned"])
    assert reached >= 5 and med["learned"] <= 0.5 * med["random"], (sweeps, med)
    # against the heuristic score (one of the network's input features):
    # the network is not expected to beat it -- at the configured size the
    # two are equal within a few sweeps -- only to keep its gain
    assert med["learned"] <= 1.5 * med["heuristic"] + 2, (sweeps, med)
