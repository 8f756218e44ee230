"""Particle-tied CP-ALS on the THC tensor (test infrastructure only).

The paper's CPD form (eq. cp4) uses one factor matrix for both indices of
a particle: with particle 1 on modes (0, 1) and particle 2 on modes (2, 3)
(chemists' order, as in oracle/dense.py),

    G ~ sum_k lam_k A[:,k] o A[:,k] o B[:,k] o B[:,k].

The paper gives no update rule for this model (its ALS is the plain one).
Reading: symmetric ALS.  A is updated by the mode-0 normal equations with
the other copy of A held at its current value, then copied to mode 1; B
likewise through mode 2 and copied to mode 3.  A sweep is therefore:

  mode 0:  Y  = Z (W2 o W3),        M0 = X0 (W1 o Y),
           V0 = G1 o G2 o G3,        A  = normalise(M0 V0^{-1}), lam
           tie: F1 = A (W1 = X1^T A, G1 = A^T A)
  mode 2:  Y' = Z^T (W0 o W1),      M2 = X2 (W3 o Y'),
           V2 = G0 o G1 o G3,        B  = normalise(M2 V2^{-1}), lam
           tie: F3 = B (W3 = X3^T B, G3 = B^T B)
  fit:     M3 = X3 (W2 o Y')  (the mode-3 MTTKRP of the tied factors),
           <G,G~> = sum_k lam_k sum_s B[s,k] M3[s,k],
           ||G~||^2 = lam^T (G0 o G1 o G2 o G3) lam,
           fit = sqrt(max(||G||^2 - 2 <G,G~> + ||G~||^2, 0)) / ||G||.

Each step is the plain ALS step of oracle/matfree.py applied to the tied
factors; the stopping rule, normalisation and damped retry are those of
oracle/dense.py.  Initial factors: A from init[0], B from init[2].

Pins (tests/test_oracle_tied.py): the fit against the dense reconstruction
of the tied model; each half-step against the plain matrix-free ALS update
from the same tied state; an exact tied CPD (diagonal core, one X) is a
fixed point.
"""
import numpy as np
import scipy.linalg


class NotSPD(RuntimeError):
    pass


def _normalise(F):
    lam = np.sqrt(np.einsum("ik,ik->k", F, F))
    return F / np.where(lam > 0, lam, 1.0)[None, :], lam


def _solve(V, M, allow_fallback):
    damped = False
    try:
        L = scipy.linalg.cholesky(V, lower=True)
    except np.linalg.LinAlgError:
        if not allow_fallback:
            raise NotSPD("V not positive definite")
        mu = 1e-12 * np.trace(V) / V.shape[0]
        try:
            L = scipy.linalg.cholesky(V + mu * np.eye(V.shape[0]), lower=True)
        except np.linalg.LinAlgError:
            raise NotSPD("damped V not positive definite")
        damped = True
    return scipy.linalg.cho_solve((L, True), M.T).T, damped


class TiedCPALS:
    def __init__(self, X, Z, init, allow_fallback=True):
        self.X = [np.asarray(x, dtype=np.float64) for x in X]
        self.Z = np.asarray(Z, dtype=np.float64)
        self.allow_fallback = allow_fallback
        S = [x.T @ x for x in self.X]
        self.norm2 = float(np.sum(self.Z * ((S[0] * S[1]) @ self.Z @ (S[2] * S[3]))))
        A, _ = _normalise(np.array(init[0], dtype=np.float64))
        B, _ = _normalise(np.array(init[2], dtype=np.float64))
        self.F = [A, A.copy(), B, B.copy()]
        self.lam = np.ones(A.shape[1])
        self.W = [self.X[m].T @ self.F[m] for m in range(4)]
        self.gram = [f.T @ f for f in self.F]
        self.fallbacks = 0
        self.Yp = None

    def _update(self, n):
        if n == 0:
            Y = self.Z @ (self.W[2] * self.W[3])
            M = self.X[0] @ (self.W[1] * Y)
        else:
            Y = self.Z.T @ (self.W[0] * self.W[1])
            self.Yp = Y
            M = self.X[2] @ (self.W[3] * Y)
        V = np.ones_like(self.gram[0])
        for m in range(4):
            if m != n:
                V = V * self.gram[m]
        Fn, damped = _solve(V, M, self.allow_fallback)
        self.fallbacks += int(damped)
        F, self.lam = _normalise(Fn)
        for m in (n, n + 1):  # the update and its tied copy
            self.F[m] = F.copy()
            self.W[m] = self.X[m].T @ F
            self.gram[m] = F.T @ F

    def sweep(self):
        self._update(0)
        self._update(2)
        return self.fit()

    def fit(self):
        M3 = self.X[3] @ (self.W[2] * self.Yp)
        inner = float(np.dot(self.lam, np.einsum("sk,sk->k", self.F[3], M3)))
        H = self.gram[0] * self.gram[1] * self.gram[2] * self.gram[3]
        model2 = float(self.lam @ H @ self.lam)
        return np.sqrt(max(self.norm2 - 2.0 * inner + model2, 0.0)) / np.sqrt(self.norm2)


def _rule_fires(fits, tol, fit_floor, fit_every):
    # the stopping rule of oracle/dense.py, looked at every fit_every sweeps
    k = len(fits)
    if k % fit_every != 0:
        return False
    if fits[-1] <= fit_floor:
        return True
    return k > fit_every and abs(fits[-1] - fits[-1 - fit_every]) <= tol * fits[-1 - fit_every]


def tied_cp_als(X, Z, init, max_sweeps, tol=1e-4, fit_floor=1e-7, allow_fallback=True, fit_every=1):
    """Tied CP-ALS with the stopping rule of oracle/dense.py."""
    st = TiedCPALS(X, Z, init, allow_fallback)
    fits = []
    for _ in range(max_sweeps):
        fits.append(st.sweep())
        if _rule_fires(fits, tol, fit_floor, fit_every):
            break
    return dict(fits=fits, lam=st.lam, F=st.F, fallbacks=st.fallbacks, state=st)
