"""THC LT-MP2 Coulomb and exchange terms and the LT-MP2 energy (test
infrastructure only).

Section 2.2, with the (i, a, j, b) mode order and Laplace scaling of
oracle/exchange.py (G[i,a,j,b] = (ia|jb) in THC form; T(t) the THC tensor
with its rows scaled, i.e. exp(-D t) G):

  J(t) = sum_{iajb} T(t)[i,a,j,b] G[i,a,j,b]     Coulomb pairing, eq. thc_Ej
  K(t) = sum_{iajb} T(t)[i,a,j,b] G[i,b,j,a]     exchange pairing, eq. thc_Ek
  E_J = 2 sum_t w_t J(t),   E_K = - sum_t w_t K(t),   E = E_J + E_K
                                                   (eq. LT-Emp2)

coulomb_term follows the bracket order the paper gives for eq. thc_Ej:
the occupied and virtual grid overlaps of the scaled and the bare factors,
multiplied element-wise (M), then contracted with Z twice and with M
again; O(R_thc^3).  exchange_term uses the plain definition: the dense
(ia|jb) tensor from the THC factors and the weighted swapped contraction
(the paper's own THC exchange, O(N^2 R^2) per point in the cited scheme,
has the same value).

Pins (tests/test_oracle_mp2.py): both terms against brute-force loops
over every (i,a,j,b); with a fine quadrature, E equals the canonical MP2
energy sum g^{ab}_{ij} (2 g^{ab}_{ij} - g^{ba}_{ij}) / D (eq. Emp2); the
THC exchange term equals the robust CPD+THC one for an exact CPD.
"""
import numpy as np

from . import dense, lt


def coulomb_term(X_occ, X_virt, Z, eps_occ, eps_virt, t):
    """J(t) in the bracket order of eq. thc_Ej."""
    Xo_t, Xv_t, _, _ = lt.lt_factors(X_occ, X_virt, eps_occ, eps_virt, t)
    M = (Xv_t.T @ X_virt) * (Xo_t.T @ X_occ)   # [P, S]
    A = M.T @ Z                                  # sum_P M[P,S] Z[P,Q]  -> [S, Q]
    B = A.T @ Z                                  # sum_S A[S,Q] Z[S,T]  -> [Q, T]
    return float(np.sum(B * M))                  # sum_{Q,T} B[Q,T] M[Q,T]


def exchange_term(X_occ, X_virt, Z, eps_occ, eps_virt, t, G=None):
    """K(t) from the dense tensor (plain definition); G: the dense tensor,
    if already formed."""
    if G is None:
        G = dense.dense_tensor([X_occ, X_virt, X_occ, X_virt], Z)
    D = (eps_virt[None, :, None, None] + eps_virt[None, None, None, :]
         - eps_occ[:, None, None, None] - eps_occ[None, None, :, None])
    return float(np.sum(np.exp(-D * t) * G * G.transpose(0, 3, 2, 1)))


def lt_mp2(X_occ, X_virt, Z, eps_occ, eps_virt, t_points, weights, exchange=True):
    """Per-point J and K (K only if exchange) and (E_J, E_K, E)."""
    J = np.array([coulomb_term(X_occ, X_virt, Z, eps_occ, eps_virt, t) for t in t_points])
    K = None
    if exchange:
        G = dense.dense_tensor([X_occ, X_virt, X_occ, X_virt], Z)
        K = np.array([exchange_term(X_occ, X_virt, Z, eps_occ, eps_virt, t, G) for t in t_points])
    w = np.asarray(weights, dtype=np.float64)
    e_j = 2.0 * float(np.sum(w * J))
    e_k = -float(np.sum(w * K)) if exchange else None
    return J, K, (e_j, e_k, None if e_k is None else e_j + e_k)
