"""Laplace-transform LT-MP2 workloads: one order-4 CPD per (system, t_k),
and the robust CPD+THC exchange energy.

Section 2.2: with the Laplace transform of the energy denominator
(eq. lt_D), the LT-MP2 energy is a sum of independent terms over the
quadrature points; each point needs the (ia|jb) tensor with its rows scaled
by exp(+eps_i t) (occupied) and exp(-eps_a t) (virtual) -- in THC form only
the factor rows change (eq. mp1_t and the THC-LT amplitude after it).  The
scaling runs on the GPU (cpd_lt_scale_rows); Z is shared by all points of a
system.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check
from .cpd import lt_scale_rows, _ptr, _stream


def lt_batch_problems(systems, t_points, rank_factors=(4, 2), init_fn=None, device="cuda"):
    """Build the CPDBatch problem list.

    systems: list of (X_occ, X_virt, Z, eps_occ, eps_virt) host arrays (one
    molecular system each); t_points: Laplace points; rank_factors:
    (R_thc / (o+v) is fixed by the input, R_cp = rank_factors[1] * (o+v));
    init_fn(dims, r_cp, index) -> 4 host arrays of initial factors.
    Returns (problems, meta) with meta[i] = (system index, t).
    """
    dev = torch.device(device)
    problems, meta = [], []
    idx = 0
    for si, (Xo, Xv, Z, eo, ev) in enumerate(systems):
        Xo_d = torch.as_tensor(Xo, dtype=torch.float64, device=dev)
        Xv_d = torch.as_tensor(Xv, dtype=torch.float64, device=dev)
        eo_d = torch.as_tensor(eo, dtype=torch.float64, device=dev)
        ev_d = torch.as_tensor(ev, dtype=torch.float64, device=dev)
        Zd = torch.as_tensor(Z, dtype=torch.float64, device=dev)
        o, v = Xo.shape[0], Xv.shape[0]
        r_cp = rank_factors[1] * (o + v)
        for t in t_points:
            X0 = lt_scale_rows(Xo_d, eo_d, t, +1.0)
            X1 = lt_scale_rows(Xv_d, ev_d, t, -1.0)
            init = init_fn([o, v, o, v], r_cp, idx)
            problems.append({"X": [X0, X1, X0, X1], "Z": Zd, "r_cp": r_cp, "init": init})
            meta.append((si, float(t)))
            idx += 1
    return problems, meta


def lt_exchange_workspace_bytes(n_occ, n_virt, r_thc, r_cp, n_points, per_point_cpds=False):
    return int(_lib.load().cpd_lt_exchange_workspace(n_occ, n_virt, r_thc, r_cp, n_points, int(per_point_cpds)))


def lt_exchange(X_occ, X_virt, Z, eps_occ, eps_virt, t_points, weights, F, lam=None, E=None, lam_e=None,
                workspace=None):
    """Robust CPD+THC LT-MP2 exchange energy of one system (Section 2.2,
    eq. cpd_single_k, the double-CPD term, eq. rob_K) on the GPU.

    X_occ, X_virt, Z, eps_*, F[0..3] (modes i, a, j, b) and lam: float64
    device tensors; t_points, weights: host sequences.  E: optional list
    (one per point) of 4 device factor tensors, separate CPDs of the scaled
    tensors (default: the LT-scaled F); lam_e: their weights (list of
    device tensors or None).  Returns device tensors (k_single[n_t],
    k_double[n_t], e_k[1]).  workspace: optional uint8 device tensor of at
    least lt_exchange_workspace_bytes(...) bytes.
    """
    lib = _lib.load()
    o, v = int(X_occ.shape[0]), int(X_virt.shape[0])
    r_thc, r_cp = int(Z.shape[0]), int(F[0].shape[1])
    t_h = np.ascontiguousarray(np.asarray(t_points, dtype=np.float64))
    w_h = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    n = int(t_h.shape[0])
    if w_h.shape[0] != n:
        raise ValueError("t_points and weights differ in length")
    dev = X_occ.device
    args = [x.contiguous() for x in (X_occ, X_virt, Z, eps_occ, eps_virt, *F)]
    lam_c = lam.contiguous() if lam is not None else None
    k1 = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    k2 = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    ek = torch.empty(1, dtype=torch.float64, device=dev)
    E_arr = lam_arr = None
    keep = []
    if E is not None:
        if len(E) != n or any(len(e) != 4 for e in E):
            raise ValueError("E needs 4 factors per Laplace point")
        keep = [f.contiguous() for e in E for f in e]
        E_arr = (ctypes.c_void_p * (4 * n))(*[f.data_ptr() for f in keep])
        if lam_e is not None:
            lk = [None if x is None else x.contiguous() for x in lam_e]
            keep += [x for x in lk if x is not None]
            lam_arr = (ctypes.c_void_p * n)(*[0 if x is None else x.data_ptr() for x in lk])
    need = lib.cpd_lt_exchange_workspace(o, v, r_thc, r_cp, n, int(E is not None))
    if workspace is None:
        workspace = torch.empty(max(int(need), 1), dtype=torch.uint8, device=dev)
    check(lib.cpd_lt_exchange(o, v, r_thc, r_cp, n, *[_ptr(a) for a in args[:5]],
                              ctypes.c_void_p(t_h.ctypes.data), ctypes.c_void_p(w_h.ctypes.data),
                              *[_ptr(a) for a in args[5:]], _ptr(lam_c),
                              ctypes.cast(E_arr, ctypes.c_void_p) if E_arr is not None else None,
                              ctypes.cast(lam_arr, ctypes.c_void_p) if lam_arr is not None else None,
                              _ptr(k1), _ptr(k2), _ptr(ek), _ptr(workspace), workspace.numel(),
                              _stream(dev)), "cpd_lt_exchange")
    return k1[:n], k2[:n], ek


def lt_mp2_workspace_bytes(n_occ, n_virt, r_thc, n_points, thc_exchange=True, z_symmetric=False):
    return int(_lib.load().cpd_lt_mp2_workspace(n_occ, n_virt, r_thc, n_points, int(thc_exchange),
                                                int(z_symmetric)))


def lt_mp2(X_occ, X_virt, Z, eps_occ, eps_virt, t_points, weights, thc_exchange=True, z_symmetric=False,
           workspace=None):
    """THC LT-MP2 Coulomb (and, with thc_exchange, exchange) terms and the
    energies (E_J, E_K, E_J + E_K) on the GPU (eq. thc_Ej, thc_Ek, LT-Emp2).
    Returns device tensors (J[n_t], K[n_t] or None, energies[3])."""
    lib = _lib.load()
    o, v, r_thc = int(X_occ.shape[0]), int(X_virt.shape[0]), int(Z.shape[0])
    t_h = np.ascontiguousarray(np.asarray(t_points, dtype=np.float64))
    w_h = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    n = int(t_h.shape[0])
    if w_h.shape[0] != n:
        raise ValueError("t_points and weights differ in length")
    dev = X_occ.device
    args = [x.contiguous() for x in (X_occ, X_virt, Z, eps_occ, eps_virt)]
    J = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    K = torch.empty(max(n, 1), dtype=torch.float64, device=dev) if thc_exchange else None
    e = torch.empty(3, dtype=torch.float64, device=dev)
    need = lib.cpd_lt_mp2_workspace(o, v, r_thc, n, int(thc_exchange), int(z_symmetric))
    if workspace is None:
        workspace = torch.empty(max(int(need), 1), dtype=torch.uint8, device=dev)
    check(lib.cpd_lt_mp2(o, v, r_thc, n, *[_ptr(a) for a in args],
                         ctypes.c_void_p(t_h.ctypes.data), ctypes.c_void_p(w_h.ctypes.data),
                         int(thc_exchange), int(z_symmetric), _ptr(J), _ptr(K), _ptr(e),
                         _ptr(workspace), workspace.numel(), _stream(dev)), "cpd_lt_mp2")
    return J[:n], (K[:n] if K is not None else None), e
