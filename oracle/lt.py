"""Laplace-transform row scaling of the THC factors (test infrastructure only).

Section 2.2: the energy denominator is replaced by a sum over Laplace
points t (eq. lt_D), and one integral tensor is multiplied by the
exponentials of the orbital energies (eq. mp1_t), which in THC form only
rescales the rows of the factor matrices (the THC-LT amplitude right after
eq. mp1_t).  For an (ia|jb)-shaped tensor with modes (i, a, j, b):

  X0 = diag(exp(+eps_occ t)) X_occ     X1 = diag(exp(-eps_virt t)) X_virt
  X2 = X0                              X3 = X1

so that G_iajb(t) = exp(-(eps_a + eps_b - eps_i - eps_j) t) (ia|jb).
The paper splits each exponential over two factors with a Fermi-level shift
eps_f and the square root of the quadrature weight; eps_f cancels within
each particle and the weight only scales the whole tensor, which leaves the
relative fit and the ALS iterates unchanged, so both are omitted here.

Pin (tests/test_oracle_lt.py): the dense tensor of the scaled factors
equals the denominator-weighted dense (ia|jb) tensor entry by entry.
"""
import numpy as np


def lt_factors(X_occ, X_virt, eps_occ, eps_virt, t):
    X0 = np.exp(eps_occ * t)[:, None] * X_occ
    X1 = np.exp(-eps_virt * t)[:, None] * X_virt
    return [X0, X1, X0.copy(), X1.copy()]
