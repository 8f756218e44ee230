"""O1 -- dense textbook CP-ALS on the explicitly formed tensor (test infrastructure only).

This is the plain definition the matrix-free method must reproduce, for
tiny mode sizes (the tensor has n0*n1*n2*n3 entries).

* Tensor: the THC form (Section 2.1, eq. THC), written in chemists'
  notation with particle 1 on indices (p, q) / grid index P and particle 2
  on (r, s) / Q:  G[p,q,r,s] = sum_{P,Q} X0[p,P] X1[q,P] Z[P,Q] X2[r,Q] X3[s,Q].
* Model: order-4 CP with column weights lambda (eq. cp4), four independent
  factor matrices.
* Loss: half the squared Frobenius residual (eq. loss), minimised by
  alternating least squares (Section 2.1; Kolda-Bader review cited there).
* Each mode update solves the normal equations F_n V_n = M_n with the
  MTTKRP M_n = G_(n) (Khatri-Rao of the other factors) and
  V_n = Hadamard product of the other factors' Gram matrices.
* Fit: the paper's definition fit = ||T - T~|| / ||T|| (Computational
  Details), here by explicit reconstruction -- deliberately a different
  formula from the matrix-free one.
* Stopping: relative change of the fit below ``tol`` (Computational
  Details use 1e-3), or fit below ``fit_floor``, or ``max_sweeps``.  With
  ``fit_every`` = k > 1 the rule is looked at only after sweeps k, 2k, ...
  and the change is measured against the fit k sweeps earlier (the
  cadence at which the mixed-precision path evaluates its fit).

Readings where the paper is silent: modes are updated in order 0,1,2,3;
columns are normalised to unit 2-norm after every update and the weights
come from the last update; the initial factors are column-normalised
before the first sweep; a failed Cholesky is retried once on
V + mu I with mu = 1e-12 tr(V) / R.

Pins (tests/test_oracle_dense.py): MTTKRP against a brute-force loop over
all tensor entries; exact recovery of planted low-rank tensors; monotone
decrease of the fit.
"""
import numpy as np
import scipy.linalg


class NotSPDError(RuntimeError):
    pass


def dense_tensor(X, Z):
    """G[p,q,r,s] = sum_PQ X0[p,P] X1[q,P] Z[P,Q] X2[r,Q] X3[s,Q]."""
    X0, X1, X2, X3 = X
    return np.einsum("pP,qP,PQ,rQ,sQ->pqrs", X0, X1, Z, X2, X3, optimize=True)


def unfold(G, n):
    """Mode-n unfolding (Kolda-Bader): rows i_n, columns ordered with the
    lowest remaining mode varying fastest."""
    return np.reshape(np.moveaxis(G, n, 0), (G.shape[n], -1), order="F")


def khatri_rao(mats):
    """Column-wise Kronecker product; the LAST matrix's row index varies fastest."""
    out = mats[0]
    for B in mats[1:]:
        r = out.shape[1]
        out = (out[:, None, :] * B[None, :, :]).reshape(-1, r)
    return out


def dense_mttkrp(G, F, n):
    """M_n = G_(n) (F_3 (.) ... F_{n+1} (.) F_{n-1} (.) ... F_0), all m != n."""
    others = [F[m] for m in reversed(range(4)) if m != n]
    return unfold(G, n) @ khatri_rao(others)


def reconstruct(lam, F):
    """[[lambda; F0, F1, F2, F3]] as a dense array."""
    return np.einsum("k,pk,qk,rk,sk->pqrs", lam, F[0], F[1], F[2], F[3], optimize=True)


def dense_fit(G, lam, F):
    return np.linalg.norm(G - reconstruct(lam, F)) / np.linalg.norm(G)


def _normal_solve(V, M, allow_fallback):
    """Solve F V = M for F by Cholesky; one damped retry (see module header)."""
    damped = False
    try:
        c = scipy.linalg.cho_factor(V, lower=True, check_finite=True)
    except (np.linalg.LinAlgError, ValueError):
        if not allow_fallback:
            raise NotSPDError("Gram-Hadamard matrix is not positive definite")
        mu = 1e-12 * np.trace(V) / V.shape[0]
        try:
            c = scipy.linalg.cho_factor(V + mu * np.eye(V.shape[0]), lower=True)
        except (np.linalg.LinAlgError, ValueError):
            raise NotSPDError("damped Gram-Hadamard matrix is not positive definite")
        damped = True
    return scipy.linalg.cho_solve(c, M.T).T, damped


def _normalise(F):
    lam = np.sqrt((F * F).sum(axis=0))
    safe = np.where(lam > 0, lam, 1.0)
    return F / safe[None, :], lam


def _stop(fits, tol, fit_floor, fit_every):
    """The stopping rule of the module header, looked at after every
    fit_every-th sweep only: the fit is at or below fit_floor, or its
    change since the previous such sweep is at most tol times that
    earlier fit."""
    k = len(fits)
    if k % fit_every:
        return False
    if fits[k - 1] <= fit_floor:
        return True
    if k - fit_every < 1:
        return False
    earlier = fits[k - 1 - fit_every]
    return abs(fits[k - 1] - earlier) <= tol * earlier


def dense_cp_als(G, init, max_sweeps, tol=1e-4, fit_floor=1e-7, allow_fallback=True, fit_every=1):
    """Run CP-ALS on the dense tensor G from the given initial factors.

    Returns dict(fits=[...], lam=..., F=[...], fallbacks=int).
    """
    F = [_normalise(np.array(f, dtype=np.float64))[0] for f in init]
    lam = np.ones(F[0].shape[1])
    fits, fallbacks = [], 0
    for sweep in range(max_sweeps):
        for n in range(4):
            M = dense_mttkrp(G, F, n)
            V = np.ones((M.shape[1], M.shape[1]))
            for m in range(4):
                if m != n:
                    V = V * (F[m].T @ F[m])
            Fn, damped = _normal_solve(V, M, allow_fallback)
            fallbacks += int(damped)
            F[n], lam = _normalise(Fn)
        fits.append(dense_fit(G, lam, F))
        if _stop(fits, tol, fit_floor, fit_every):
            break
    return dict(fits=fits, lam=lam, F=F, fallbacks=fallbacks)
