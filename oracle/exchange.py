"""Robust CPD+THC LT-MP2 exchange energy (test infrastructure only).

Section 2.2.  Tensors use the (i, a, j, b) mode order of the batched
Laplace workload (occupied, virtual, occupied, virtual):

  G[i,a,j,b]  = (ia|jb) = sum_PQ Xo[i,P] Xv[a,P] Z[P,Q] Xo[j,Q] Xv[b,Q]
                                                         (THC, eq. THC)
  G~[i,a,j,b] = sum_r lam_r F0[i,r] F1[a,r] F2[j,r] F3[b,r]
                                                         (CPD of G, eq. cp4)

At a Laplace point t the amplitude tensor carries exp(-D t) with
D = e_a + e_b - e_i - e_j (eq. lt_D and eq. mp1_t).  In THC form that
rescales the rows of Xo by exp(+e_i t) and of Xv by exp(-e_a t) (see
oracle/lt.py).  The LT-scaled CPD likewise rescales the rows of F0 and F2
(occupied) and of F1 and F3 (virtual).

Exchange pairing: K(T, S) = sum_{iajb} T[i,a,j,b] S[i,b,j,a].  This is
g^{ba}_{ij}, with the two virtual indices swapped.

  k_single(t) = K(T_thc(t), G~)   the single-CPD term (eq. cpd_single_k),
                evaluated in the paper's bracket order: two projected,
                Hadamard-multiplied factors per CP column, one contraction
                with Z, then the sum over grid points and columns.
  k_double(t) = K(T_cpd(t), G~)   the double-CPD term: a sum over column
                pairs (r, r') of the product of four small overlaps.
  E_K = - sum_t w_t [2 k_single(t) - k_double(t)]      (eq. rob_K)

Readings where the paper is silent or at odds with itself:
* The printed double-CPD term pairs the occupied index of one particle
  with the other particle's factor.  For a CPD whose two particles differ,
  that is the Coulomb pairing, not the exchange one.  Here both terms use
  the pairing that follows from the definition of g^{ba}_{ij}, the same as
  the single-CPD term.  The pin below shows this is the reading under
  which an exact CPD reproduces the exact exchange energy.
* T_cpd(t) is the LT-scaled CPD of the bare tensor.  This is the reading of
  the paper's symmetry remark: scaling the bare tensor or the one inside
  the amplitude gives the same term.  Under this reading the robust
  combination cancels the first-order CPD error.  A separate CPD of T(t)
  may be passed instead (argument E).
* The amplitude carries the whole exp(-D t) and the whole weight w_t, so
  that sum_t w_t exp(-D t) approximates 1/D (eq. lt_D).  The paper's
  quarter powers of |w| and the half exponents are the split of that
  factor over the two tensors of a product.  The Fermi level cancels.

Pins (tests/test_oracle_exchange.py):
* both terms against brute-force loops over every (i,a,j,b);
* the symmetry identity (moving the LT scaling from the THC tensor onto
  the CPD leaves k_single unchanged);
* an exact CPD (diagonal Z) giving k_single = k_double = the dense exact
  term;
* the robust energy's error quadratic in the CPD error, while the
  single-CPD energy's is linear;
* a fine quadrature reproducing the canonical MP2 exchange
  -sum g^{ab}_{ij} g^{ba}_{ij} / D.
"""
import numpy as np

from . import lt


def lt_cp_factors(F, eps_occ, eps_virt, t):
    """Rows of the CPD factors (modes i, a, j, b) scaled for Laplace point t."""
    so = np.exp(eps_occ * t)[:, None]
    sv = np.exp(-eps_virt * t)[:, None]
    return [so * F[0], sv * F[1], so * F[2], sv * F[3]]


def k_single(X_occ, X_virt, Z, F, lam, eps_occ, eps_virt, t, absolute=False):
    """K(T_thc(t), G~), eq. cpd_single_k.

    With absolute=True every operand is replaced by its absolute value.  The
    result bounds the sum of |terms| under any summation order (used for
    error bounds).
    """
    Xo, Xv, _, _ = lt.lt_factors(X_occ, X_virt, eps_occ, eps_virt, t)
    F0, F1, F2, F3 = F
    lam = np.ones(F0.shape[1]) if lam is None else np.asarray(lam, dtype=np.float64)
    if absolute:
        Xo, Xv, Z = np.abs(Xo), np.abs(Xv), np.abs(Z)
        F0, F1, F2, F3 = (np.abs(f) for f in F)
        lam = np.abs(lam)
    # particle 1: virtual a against the CPD's a-slot of g^{ba} (F3), occupied
    # i against its i-slot (F0); both share the grid index P
    left = (Xv.T @ F3) * (Xo.T @ F0)
    # particle 2: virtual b against F1, occupied j against F2, grid index Q
    right = (Xv.T @ F1) * (Xo.T @ F2)
    inner = Z @ right
    return float(np.sum(lam[None, :] * left * inner))


def k_double(E, lam_e, F, lam_f, absolute=False):
    """K(T_cpd, G~) for T_cpd = sum_r lam_e[r] E0 o E1 o E2 o E3: the sum over
    (r, r') of lam_e[r] lam_f[r'] (E0^T F0)(E1^T F3)(E2^T F2)(E3^T F1)[r, r']."""
    lam_e = np.ones(E[0].shape[1]) if lam_e is None else np.asarray(lam_e, dtype=np.float64)
    lam_f = np.ones(F[0].shape[1]) if lam_f is None else np.asarray(lam_f, dtype=np.float64)
    if absolute:
        E = [np.abs(e) for e in E]
        F = [np.abs(f) for f in F]
        lam_e, lam_f = np.abs(lam_e), np.abs(lam_f)
    prod = (E[0].T @ F[0]) * (E[1].T @ F[3]) * (E[2].T @ F[2]) * (E[3].T @ F[1])
    return float(lam_e @ prod @ lam_f)


def exchange_terms(X_occ, X_virt, Z, F, lam, eps_occ, eps_virt, t_points, E=None, lam_e=None,
                   absolute=False):
    """k_single and k_double at every Laplace point.

    E: optional list (one per point) of separate CPDs of T(t); by default
    T_cpd(t) is the LT-scaled CPD of the bare tensor, with weights lam.
    """
    k1 = np.empty(len(t_points))
    k2 = np.empty(len(t_points))
    for n, t in enumerate(t_points):
        k1[n] = k_single(X_occ, X_virt, Z, F, lam, eps_occ, eps_virt, t, absolute=absolute)
        if E is None:
            Et, lt_ = lt_cp_factors(F, eps_occ, eps_virt, t), lam
        else:
            Et, lt_ = E[n], (None if lam_e is None else lam_e[n])
        k2[n] = k_double(Et, lt_, F, lam, absolute=absolute)
    return k1, k2


def robust_exchange(k1, k2, w):
    """E_K = - sum_t w_t (2 k_single(t) - k_double(t)), eq. rob_K."""
    return float(-np.sum(np.asarray(w) * (2.0 * np.asarray(k1) - np.asarray(k2))))
