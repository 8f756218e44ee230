"""Pins of the warm-start network oracle (oracle/mlp.py): finite
differences for the hand-written backward pass, closed forms for the loss
and for Adam."""
import numpy as np

from oracle import mlp
from synth import mlp_init_params


def _data(rows, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((rows, mlp.D_IN))
    y = (rng.random(rows) < 0.6).astype(np.float64)
    ell_t = rng.standard_normal(rows)
    mask = (rng.random(rows) < 0.7).astype(np.float64)
    return x, y, ell_t, mask


def _loss_at(theta, x, y, ell_t, mask):
    out, _ = mlp.forward(theta, x)
    return mlp.loss(out, y, ell_t, mask)[0]


def test_param_layout():
    theta = mlp_init_params(3).astype(np.float64)
    assert theta.size == mlp.param_count() == 8 * 256 + 256 + 256 * 256 + 256 + 256 * 2 + 2
    blocks = mlp.unpack(theta)
    assert np.array_equal(mlp.pack(blocks), theta)
    assert all(np.all(b == 0) for b in (blocks[1], blocks[3], blocks[5]))


def test_backward_matches_central_differences():
    x, y, ell_t, mask = _data(12, 1)
    theta = mlp_init_params(5).astype(np.float64)
    theta += 0.05 * np.random.default_rng(2).standard_normal(theta.size)  # non-zero biases
    out, cache = mlp.forward(theta, x)
    _, dout = mlp.loss(out, y, ell_t, mask)
    g = mlp.backward(theta, cache, dout)
    rng = np.random.default_rng(7)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in mlp.SHAPES])
    h = 1e-6
    for b in range(len(mlp.SHAPES)):
        idx = rng.choice(np.arange(offs[b], offs[b + 1]), size=min(24, offs[b + 1] - offs[b]), replace=False)
        for i in idx:
            tp = theta.copy(); tp[i] += h
            tm = theta.copy(); tm[i] -= h
            fd = (_loss_at(tp, x, y, ell_t, mask) - _loss_at(tm, x, y, ell_t, mask)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (b, i, fd, g[i])


def test_loss_closed_forms():
    R = 10
    out = np.zeros((R, 2))
    y = np.r_[np.ones(4), np.zeros(6)]
    L, dout = mlp.loss(out, y, np.zeros(R), np.zeros(R))
    assert abs(L - np.log(2.0)) < 1e-15  # logit 0: cross-entropy log 2 for either label
    assert np.allclose(dout[:, 0], (0.5 - y) / R, rtol=0, atol=1e-17)
    assert np.all(dout[:, 1] == 0)
    mask = np.r_[np.ones(5), np.zeros(5)]
    L2, d2 = mlp.loss(np.c_[np.zeros(R), np.ones(R)], y, np.zeros(R), mask)
    assert abs(L2 - (np.log(2.0) + 1.0)) < 1e-15  # unit scale error on the masked rows
    assert np.allclose(d2[:, 1], 2.0 * mask / 5)
    # confident and right: loss -> 0; confident and wrong: loss ~ |logit|
    L3, _ = mlp.loss(np.array([[40.0, 0.0]]), np.array([1.0]), np.zeros(1), np.zeros(1))
    L4, _ = mlp.loss(np.array([[40.0, 0.0]]), np.array([0.0]), np.zeros(1), np.zeros(1))
    assert L3 < 1e-16 and abs(L4 - 40.0) < 1e-12


def test_zero_weights_give_output_bias():
    theta = np.zeros(mlp.param_count())
    theta[-2:] = [0.25, -1.5]
    out, _ = mlp.forward(theta, np.random.default_rng(0).standard_normal((7, 8)))
    assert np.all(out == np.array([0.25, -1.5]))


def test_silu_closed_forms():
    assert mlp.silu(0.0) == 0.0 and mlp.silu_grad(0.0) == 0.5
    a = np.array([-30.0, 30.0])
    assert np.allclose(mlp.silu(a), [0.0, 30.0], atol=1e-11)
    assert np.allclose(mlp.silu_grad(a), [0.0, 1.0], atol=1e-11)


def test_adam_first_two_steps_closed_form():
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(50)
    g1, g2 = rng.standard_normal(50), rng.standard_normal(50)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    t1, m, v = mlp.adam_step(theta, g1, np.zeros(50), np.zeros(50), 1, lr, b1, b2, eps)
    # bias-corrected moments of one step are g and g^2
    assert np.allclose(t1, theta - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    t2, _, _ = mlp.adam_step(t1, g2, m, v, 2, lr, b1, b2, eps)
    mhat = (b1 * g1 + g2) / (1 + b1)
    vhat = (b2 * g1 ** 2 + g2 ** 2) / (1 + b2)
    assert np.allclose(t2, t1 - lr * mhat / (np.sqrt(vhat) + eps), rtol=0, atol=1e-15)
