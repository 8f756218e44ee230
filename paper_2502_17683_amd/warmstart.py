"""Learned warm start for CP-ALS through libthccp.so.

With a diagonal core the THC form is already an exact CP decomposition
whose columns are the grid columns X_m[:, P] (eq. THC), so the initial CP is
built from R_cp scaled grid columns.  A three-layer network (8 -> 256 ->
256 -> 2) scores each grid point from eight standardised features of
(X0, Z, S = X0^T X0); it is trained (FP32, Adam) on targets taken from
converged CPDs and run in BF16 for inference.  Fallbacks: the heuristic
score log(Z_PP S_PP^2), then the caller's random guess.

Every computation runs in the library's kernels; this module marshals
arguments, owns the torch tensors that back parameters and workspaces,
and loops over training steps.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check
from .cpd import _ptr, _stream, _dev_f64, CPDBatch

N_FEATURES = 8


def _n4(n):
    return (ctypes.c_int32 * 4)(*[int(v) for v in n])


def _vp4(ts):
    return (ctypes.c_void_p * 4)(*[t.data_ptr() for t in ts])


def _four(X, device):
    if not isinstance(X, (list, tuple)):
        X = [X] * 4
    seen, out = {}, []
    for x in X:
        if id(x) not in seen:
            seen[id(x)] = _dev_f64(x, device)
        out.append(seen[id(x)])
    return out


def _ws(lib, n0, r_thc, r_cp, device):
    size = lib.cpd_ws_workspace_size(int(n0), int(r_thc), int(r_cp))
    if size == 0:
        raise ValueError(f"bad warm-start sizes n0={n0} r_thc={r_thc} r_cp={r_cp}")
    return torch.empty(size, dtype=torch.uint8, device=device)


def ws_features(X0, Z, device="cuda"):
    """(feat r_thc x 8 float32, heuristic score r_thc float64) on the device."""
    lib = _lib.load()
    dev = torch.device(device)
    X0 = _dev_f64(X0, dev)
    Z = _dev_f64(Z, dev)
    n0, r_thc = X0.shape
    feat = torch.empty(r_thc, N_FEATURES, dtype=torch.float32, device=dev)
    heur = torch.empty(r_thc, dtype=torch.float64, device=dev)
    ws = _ws(lib, n0, r_thc, 1, dev)
    check(lib.cpd_ws_features(n0, r_thc, _ptr(X0), _ptr(Z), _ptr(feat), _ptr(heur), _ptr(ws), ws.numel(),
                              _stream(dev)), "cpd_ws_features")
    return feat, heur


def ws_features_noalloc(X0, Z, device="cuda"):
    """ws_features through the allocation-free entry point (static device
    scratch inside the library; r_thc <= 2048)."""
    lib = _lib.load()
    dev = torch.device(device)
    X0 = _dev_f64(X0, dev)
    Z = _dev_f64(Z, dev)
    n0, r_thc = X0.shape
    feat = torch.empty(r_thc, N_FEATURES, dtype=torch.float32, device=dev)
    heur = torch.empty(r_thc, dtype=torch.float64, device=dev)
    check(lib.cpd_ws_features_noalloc(n0, r_thc, _ptr(X0), _ptr(Z), _ptr(feat), _ptr(heur), _stream(dev)),
          "cpd_ws_features_noalloc")
    return feat, heur


def ws_select_init(X, s, ell, r_cp, stride=1, noise=None, sigma=0.0, device="cuda"):
    """Initial factors from the top-r_cp grid points by score s (float32),
    optionally blended with the random guess `noise` (four n_m x r_cp)."""
    lib = _lib.load()
    dev = torch.device(device)
    X = _four(X, dev)
    n = [int(x.shape[0]) for x in X]
    r_thc = int(X[0].shape[1])
    s = torch.as_tensor(s, dtype=torch.float32, device=dev).contiguous()
    ell = None if ell is None else torch.as_tensor(ell, dtype=torch.float32, device=dev).contiguous()
    init = [torch.empty(n[m], r_cp, dtype=torch.float64, device=dev) for m in range(4)]
    nz = None if noise is None else [_dev_f64(f, dev) for f in noise]
    ws = _ws(lib, n[0], r_thc, r_cp, dev)
    check(lib.cpd_ws_select_init(_n4(n), r_thc, int(r_cp), _vp4(X), _ptr(s), _ptr(ell), int(stride),
                                 None if nz is None else ctypes.pointer(_vp4(nz)), float(sigma), _vp4(init),
                                 _ptr(ws), ws.numel(), _stream(dev)), "cpd_ws_select_init")
    return init


def ws_labels(X, F, lam, device="cuda"):
    """Training targets (y, ell, mask), float32 r_thc each, from a converged
    CPD with unit columns F and weights lam."""
    lib = _lib.load()
    dev = torch.device(device)
    X = _four(X, dev)
    F = [_dev_f64(f, dev) for f in F]
    lam = _dev_f64(lam, dev)
    n = [int(x.shape[0]) for x in X]
    r_thc, r_cp = int(X[0].shape[1]), int(F[0].shape[1])
    y, ell, mask = (torch.empty(r_thc, dtype=torch.float32, device=dev) for _ in range(3))
    ws = _ws(lib, n[0], r_thc, r_cp, dev)
    check(lib.cpd_ws_labels(_n4(n), r_thc, r_cp, _vp4(X), _vp4(F), _ptr(lam), _ptr(y), _ptr(ell), _ptr(mask),
                            _ptr(ws), ws.numel(), _stream(dev)), "cpd_ws_labels")
    return y, ell, mask


SOURCES = ("network", "heuristic", "unchanged")
# Weight of the random unit column blended into each selected grid column.
DEFAULT_SIGMA = 0.25


def ws_init(X, Z, r_cp, packed=None, noise=None, sigma=DEFAULT_SIGMA, device="cuda"):
    """Warm-start factors: the network's selection if `packed` (from
    WarmStartMLP.pack) is given and its scores are finite, else the
    heuristic; each selected grid column is blended with the random guess
    `noise` (four n_m x r_cp; None: plain grid columns).  If neither score
    is usable the result is `noise` itself (zeros without it).  Returns
    (factors, source name)."""
    lib = _lib.load()
    dev = torch.device(device)
    X = _four(X, dev)
    Z = _dev_f64(Z, dev)
    n = [int(x.shape[0]) for x in X]
    r_thc = int(Z.shape[0])
    if noise is None:
        init = [torch.zeros(n[m], r_cp, dtype=torch.float64, device=dev) for m in range(4)]
        nz = None
    else:
        init = [_dev_f64(f, dev).clone() for f in noise]
        nz = ctypes.pointer(_vp4(init))  # the blend reads each element before overwriting it
    ws = _ws(lib, n[0], r_thc, r_cp, dev)
    src = ctypes.c_int32(-1)
    check(lib.cpd_ws_init(_n4(n), r_thc, int(r_cp), _vp4(X), _ptr(Z), _ptr(packed), nz, float(sigma), _vp4(init),
                          ctypes.byref(src), _ptr(ws), ws.numel(), _stream(dev)), "cpd_ws_init")
    return init, SOURCES[src.value]


class WarmStartMLP:
    """The warm-start network: FP32 parameters and Adam state on the device."""

    def __init__(self, params, device="cuda"):
        self.lib = _lib.load()
        self.device = torch.device(device)
        count = self.lib.cpd_mlp_param_count()
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32), device=self.device).contiguous()
        if self.params.numel() != count:
            raise ValueError(f"expected {count} parameters, got {self.params.numel()}")
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = None
        self._ws_rows = 0

    def _workspace(self, rows):
        if rows > self._ws_rows:
            size = self.lib.cpd_mlp_workspace_size(int(rows))
            self._ws = torch.empty(size, dtype=torch.uint8, device=self.device)
            self._ws_rows = rows
        return self._ws

    def forward(self, x, idx=None, rows=None):
        """FP32 forward of x[idx] (or x); returns rows x 2 (logit, log-scale)."""
        rows = int(idx.numel() if idx is not None else x.shape[0]) if rows is None else rows
        out = torch.empty(rows, 2, dtype=torch.float32, device=self.device)
        ws = self._workspace(rows)
        check(self.lib.cpd_mlp_forward(_ptr(self.params), _ptr(x), _ptr(idx), rows, _ptr(out), _ptr(ws), ws.numel(),
                                       _stream(self.device)), "cpd_mlp_forward")
        return out

    def loss(self, out, y, ell, mask, idx=None):
        rows = int(out.shape[0])
        dout = torch.empty_like(out)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        ws = self._workspace(rows)
        check(self.lib.cpd_mlp_loss(_ptr(out), _ptr(y), _ptr(ell), _ptr(mask), _ptr(idx), rows, _ptr(dout),
                                    _ptr(loss), _ptr(ws), ws.numel(), _stream(self.device)), "cpd_mlp_loss")
        return loss, dout

    def backward(self, x, dout, idx=None):
        rows = int(dout.shape[0])
        ws = self._workspace(rows)
        check(self.lib.cpd_mlp_backward(_ptr(self.params), _ptr(x), _ptr(idx), _ptr(dout), rows, _ptr(self.grads),
                                        _ptr(ws), ws.numel(), _stream(self.device)), "cpd_mlp_backward")
        return self.grads

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        check(self.lib.cpd_mlp_adam(_ptr(self.params), _ptr(self.grads), _ptr(self.m), _ptr(self.v), self.step,
                                    lr, beta1, beta2, eps, _stream(self.device)), "cpd_mlp_adam")

    def train(self, data, order, batch_rows=8192, lr=1e-3, epochs=1):
        """Minibatch Adam over data = (feat, y, ell, mask) on the device;
        `order` is the row permutation (int32) used for every epoch.
        Returns the loss of every step (one synchronisation at the end)."""
        feat, y, ell, mask = data
        order = torch.as_tensor(order, dtype=torch.int32, device=self.device)
        total = int(order.numel())
        losses = []
        for _ in range(epochs):
            for a in range(0, total, batch_rows):
                idx = order[a:a + batch_rows]
                out = self.forward(feat, idx)
                loss, dout = self.loss(out, y, ell, mask, idx)
                self.backward(feat, dout, idx)
                self.adam(lr)
                losses.append(loss)
        return torch.cat(losses).cpu().numpy() if losses else np.zeros(0)

    def pack(self):
        packed = torch.empty(self.lib.cpd_mlp_packed_size(), dtype=torch.uint8, device=self.device)
        check(self.lib.cpd_mlp_pack(_ptr(self.params), _ptr(packed), _stream(self.device)), "cpd_mlp_pack")
        return packed

    def infer_bf16(self, x, packed=None):
        packed = self.pack() if packed is None else packed
        rows = int(x.shape[0])
        out = torch.empty(rows, 2, dtype=torch.float32, device=self.device)
        check(self.lib.cpd_mlp_infer_bf16(_ptr(packed), _ptr(x), rows, _ptr(out), _stream(self.device)),
              "cpd_mlp_infer_bf16")
        return out


def training_set(problems, sweeps=200, tol=1e-4, precision="fp64", device="cuda", chunk=32):
    """Features and targets over the grid points of every problem.

    problems: dicts with X (tensor or four), Z, r_cp, init (four random
    initial factors).  Each problem is run to convergence (batched CP-ALS,
    `chunk` problems per batch); its converged factors give the targets.
    Returns (feat, y, ell, mask) concatenated over the problems, on the
    device."""
    dev = torch.device(device)
    feats, ys, ells, masks = [], [], [], []
    for a in range(0, len(problems), chunk):
        part = problems[a:a + chunk]
        b = CPDBatch(part, precision=precision, tol=tol, fit_floor=1e-7, device=device)
        b.sweep(sweeps)
        for i, pr in enumerate(part):
            F, lam = b.factors(i)
            X = _four(pr["X"], dev)
            y, ell, mask = ws_labels(X, F, lam, device=device)
            f, _ = ws_features(X[0], pr["Z"], device=device)
            feats.append(f)
            ys.append(y)
            ells.append(ell)
            masks.append(mask)
        del b
    return torch.cat(feats), torch.cat(ys), torch.cat(ells), torch.cat(masks)
