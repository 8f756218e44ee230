"""Batched Laplace-transform workload: one order-4 CPD per (system, t_k).

Section 2.2: with the Laplace transform of the energy denominator
(eq. lt_D), the LT-MP2 energy is a sum of independent terms over the
quadrature points; each point needs the (ia|jb) tensor with its rows scaled
by exp(+eps_i t) (occupied) and exp(-eps_a t) (virtual) -- in THC form only
the factor rows change (eq. mp1_t and the THC-LT amplitude after it).  The
scaling runs on the GPU (cpd_lt_scale_rows); Z is shared by all points of a
system.
"""
import torch

from .cpd import lt_scale_rows


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
