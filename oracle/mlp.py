"""Warm-start network in float64 NumPy (test infrastructure only).

A three-layer perceptron maps the eight standardised features of one grid
point to two outputs: a selection logit s (is this grid point the support
of a CP column?) and a log-scale ell of that column:

  a1 = x W1 + b1,   h1 = silu(a1)         8 -> 256
  a2 = h1 W2 + b2,  h2 = silu(a2)       256 -> 256
  out = h2 W3 + b3                      256 -> 2      (s, ell)

silu(a) = a sigmoid(a).  Parameters are one flat vector in the order
W1 (8 x 256, row-major), b1, W2 (256 x 256), b2, W3 (256 x 2), b3.

Loss over R rows with targets (y, ell_t) and a mask of rows whose scale
target is defined:
  L = (1/R) sum_r BCE(s_r, y_r) + (1/max(1, sum mask)) sum_r mask_r (ell_r - ell_t,r)^2
with the logistic cross-entropy BCE(s, y) = max(s, 0) - s y + log(1 + exp(-|s|)).

The backward pass is written out by hand (chain rule, layer by layer) and
Adam follows Kingma and Ba (2015) with bias correction.

Pins (tests/test_oracle_mlp.py): central finite differences of the loss
for every parameter block; closed-form loss values; closed-form first and
second Adam steps; zero weights give the output bias.
"""
import numpy as np

D_IN, WIDTH, D_OUT = 8, 256, 2
SHAPES = [(D_IN, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH, D_OUT), (D_OUT,)]


def param_count():
    return int(sum(np.prod(s) for s in SHAPES))


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def pack(blocks):
    return np.concatenate([np.asarray(b, dtype=np.float64).ravel() for b in blocks])


def sigmoid(a):
    return 0.5 * (1.0 + np.tanh(0.5 * a))


def silu(a):
    return a * sigmoid(a)


def silu_grad(a):
    g = sigmoid(a)
    return g * (1.0 + a * (1.0 - g))


def forward(theta, x):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ W1 + b1
    h1 = silu(a1)
    a2 = h1 @ W2 + b2
    h2 = silu(a2)
    out = h2 @ W3 + b3
    return out, (x, a1, h1, a2, h2)


def loss(out, y, ell_t, mask):
    s, ell = out[:, 0], out[:, 1]
    R = out.shape[0]
    msum = max(1.0, float(np.sum(mask)))
    bce = np.maximum(s, 0.0) - s * y + np.log1p(np.exp(-np.abs(s)))
    L = bce.sum() / R + np.sum(mask * (ell - ell_t) ** 2) / msum
    dout = np.empty_like(out)
    dout[:, 0] = (sigmoid(s) - y) / R
    dout[:, 1] = 2.0 * mask * (ell - ell_t) / msum
    return float(L), dout


def backward(theta, cache, dout):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    x, a1, h1, a2, h2 = cache
    gW3 = h2.T @ dout
    gb3 = dout.sum(axis=0)
    da2 = (dout @ W3.T) * silu_grad(a2)
    gW2 = h1.T @ da2
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ W2.T) * silu_grad(a1)
    gW1 = x.T @ da1
    gb1 = da1.sum(axis=0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
