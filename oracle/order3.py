"""Order-3 THC-like tensors through the order-4 form (test infrastructure
only).

The paper's conclusions extend the method to other THC-like networks and
orders.  The order-3 network

  G3[p,q,r] = sum_{P,Q} X0[p,P] X1[q,P] Z[P,Q] X2[r,Q]

is the order-4 THC tensor (eq. THC) with a singleton fourth mode, n3 = 1
and X3 = a row of ones: G[p,q,r,0] = G3[p,q,r].  A rank-R CPD of G with
F3 of size 1 x R is a rank-R CPD of G3 (F3's unit-norm entries are signs,
absorbed into lambda).  This module holds the plain three-way CP-ALS
(Kolda-Bader: modes 0, 1, 2; Khatri-Rao of the other two factors;
Hadamard of their Grams; unit-norm columns, weights from the last update)
on the dense G3, against which the order-4 runs with a singleton mode are
pinned.

Pins (tests/test_oracle_order3.py): the dense order-4 tensor with the
singleton mode equals G3; the order-4 dense CP-ALS with a singleton mode
follows this three-way CP-ALS.
"""
import numpy as np
import scipy.linalg


def order3_tensor(X0, X1, X2, Z):
    return np.einsum("pP,qP,PQ,rQ->pqr", X0, X1, Z, X2, optimize=True)


def _unfold(G, n):
    return np.reshape(np.moveaxis(G, n, 0), (G.shape[n], -1), order="F")


def _khatri_rao(A, B):
    # row index of B varies fastest
    return (A[:, None, :] * B[None, :, :]).reshape(-1, A.shape[1])


def cp3_als(G, init, max_sweeps):
    """Three-way CP-ALS from the given (column-normalised) initial factors;
    returns the fits ||G - G~|| / ||G|| per sweep."""
    F = [f / np.linalg.norm(f, axis=0) for f in (np.array(x, dtype=np.float64) for x in init)]
    lam = np.ones(F[0].shape[1])
    nG = np.linalg.norm(G)
    fits = []
    for _ in range(max_sweeps):
        for n in range(3):
            others = [m for m in range(3) if m != n]
            # unfold(G, n) columns: lowest remaining mode fastest, so the
            # Khatri-Rao product takes the higher mode first
            KR = _khatri_rao(F[others[1]], F[others[0]])
            M = _unfold(G, n) @ KR
            V = (F[others[0]].T @ F[others[0]]) * (F[others[1]].T @ F[others[1]])
            Fn = scipy.linalg.solve(V, M.T, assume_a="pos").T
            lam = np.linalg.norm(Fn, axis=0)
            F[n] = Fn / lam
        Gt = np.einsum("k,pk,qk,rk->pqr", lam, F[0], F[1], F[2])
        fits.append(float(np.linalg.norm(G - Gt) / nG))
    return fits
