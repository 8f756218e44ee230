"""O2 -- matrix-free THC-based CP-ALS (test infrastructure only).

The paper's method (Section 2.1, eq. lossF): the CP-ALS of the tensor given
in THC form is run without ever forming the tensor.  With
G[p,q,r,s] = sum_PQ X0[p,P] X1[q,P] Z[P,Q] X2[r,Q] X3[s,Q] and factors
F0..F3 (n_m x R columns), every quantity ALS needs factors through the
projections W_m = X_m^T F_m (R_thc x R):

  MTTKRP, mode 0:  M0 = X0 (W1 o Y),   Y  = Z   (W2 o W3)
          mode 1:  M1 = X1 (W0 o Y)     (Y reused: F2, F3 unchanged)
          mode 2:  M2 = X2 (W3 o Y'),  Y' = Z^T (W0 o W1)
          mode 3:  M3 = X3 (W2 o Y')    (Y' reused)
  ('o' is the Hadamard product.)  Each equals G_(n) times the Khatri-Rao
  product of the other factors exactly; cost O(n R_thc R + R_thc^2 R),
  storage O(R^2) -- the complexity the paper states for eq. lossF.

  Normal equations: V_n = Hadamard product of F_m^T F_m over m != n,
  F_n = M_n V_n^{-1} by Cholesky (FP64), then unit-norm columns and
  weights lambda (eq. cp4).

  ||G||^2 = <Z, T01 Z T23>_F with S_m = X_m^T X_m, T01 = S0 o S1,
  T23 = S2 o S3 (for a symmetric Z and equal X_m this is
  sum Z_PQ Z_P'Q' S_PP'^2 S_QQ'^2).
  <G, G~> = sum_k lambda_k sum_s F3[s,k] M3[s,k]   (M3 from the last mode),
  ||G~||^2 = lambda^T (o_m F_m^T F_m) lambda,
  fit = sqrt(max(||G||^2 - 2<G,G~> + ||G~||^2, 0)) / ||G||
  -- the paper's fit ||T - T~|| / ||T|| (Computational Details).

Readings shared with O1 (mode order 0..3, normalisation, damped Cholesky
retry, stopping rule) are listed in oracle/dense.py.  This module shares no
code with O1 or with the HIP library.

Pins (tests/test_oracle_matfree.py): MTTKRP, ||G||^2, <G,G~>, ||G~||^2
element-wise against O1's dense tensor; whole trajectories against O1;
planted exact CPD from a diagonal core; X = identity special case;
invariances (core scaling, mode symmetries).
"""
import numpy as np
import scipy.linalg


class NotSPD(RuntimeError):
    pass


def thc_norm2(X, Z):
    """||G||^2 = <Z, (S0 o S1) Z (S2 o S3)>_F."""
    S = [x.T @ x for x in X]
    T01 = S[0] * S[1]
    T23 = S[2] * S[3]
    return float(np.sum(Z * (T01 @ Z @ T23)))


def projections(X, F):
    return [X[m].T @ F[m] for m in range(4)]


def mttkrp(X, Z, F, n):
    """Matrix-free MTTKRP of mode n (fresh projections, no reuse)."""
    W = projections(X, F)
    if n in (0, 1):
        Y = Z @ (W[2] * W[3])
        partner = 1 - n
    else:
        Y = Z.T @ (W[0] * W[1])
        partner = 5 - n
    return X[n] @ (W[partner] * Y)


def cholesky_solve(V, M, allow_fallback=True):
    """F = M V^{-1}; returns (F, damped)."""
    damped = False
    try:
        L = np.linalg.cholesky(V)
    except np.linalg.LinAlgError:
        if not allow_fallback:
            raise NotSPD("V not positive definite")
        mu = 1e-12 * np.trace(V) / V.shape[0]
        try:
            L = np.linalg.cholesky(V + mu * np.eye(V.shape[0]))
        except np.linalg.LinAlgError:
            raise NotSPD("damped V not positive definite")
        damped = True
    Gt = scipy.linalg.solve_triangular(L, M.T, lower=True)
    Ft = scipy.linalg.solve_triangular(L.T, Gt, lower=False)
    return Ft.T, damped


def column_normalise(F):
    lam = np.sqrt(np.einsum("ik,ik->k", F, F))
    return F / np.where(lam > 0, lam, 1.0)[None, :], lam


class MatFreeCPALS:
    """State of one matrix-free CP-ALS run; ``sweep()`` does modes 0..3 and
    returns the fit."""

    def __init__(self, X, Z, init, allow_fallback=True):
        self.X = [np.asarray(x, dtype=np.float64) for x in X]
        self.Z = np.asarray(Z, dtype=np.float64)
        self.allow_fallback = allow_fallback
        self.norm2 = thc_norm2(self.X, self.Z)
        self.F = [column_normalise(np.array(f, dtype=np.float64))[0] for f in init]
        self.lam = np.ones(self.F[0].shape[1])
        self.W = projections(self.X, self.F)
        self.gram = [f.T @ f for f in self.F]
        self.Y = None
        self.M = None
        self.fallbacks = 0

    def mttkrp(self, n):
        if n == 0:
            self.Y = self.Z @ (self.W[2] * self.W[3])
        elif n == 2:
            self.Y = self.Z.T @ (self.W[0] * self.W[1])
        partner = {0: 1, 1: 0, 2: 3, 3: 2}[n]
        return self.X[n] @ (self.W[partner] * self.Y)

    def update(self, n):
        M = self.mttkrp(n)
        V = np.ones_like(self.gram[0])
        for m in range(4):
            if m != n:
                V = V * self.gram[m]
        Fn, damped = cholesky_solve(V, M, self.allow_fallback)
        self.fallbacks += int(damped)
        self.F[n], self.lam = column_normalise(Fn)
        self.gram[n] = self.F[n].T @ self.F[n]
        self.W[n] = self.X[n].T @ self.F[n]
        self.M = M

    def fit_terms(self):
        """(<G,G~>, ||G~||^2) after a mode-3 update."""
        inner = float(np.dot(self.lam, np.einsum("sk,sk->k", self.F[3], self.M)))
        H = self.gram[0] * self.gram[1] * self.gram[2] * self.gram[3]
        model2 = float(self.lam @ H @ self.lam)
        return inner, model2

    def fit(self):
        inner, model2 = self.fit_terms()
        res2 = max(self.norm2 - 2.0 * inner + model2, 0.0)
        return np.sqrt(res2) / np.sqrt(self.norm2)

    def sweep(self):
        for n in range(4):
            self.update(n)
        return self.fit()


def stops(fits, tol, fit_floor, fit_every=1):
    """Stopping rule (Computational Details: relative change in fit below a
    tolerance), read as in oracle/dense.py and checked after the sweep that
    produced fits[-1].  The rule is looked at on every fit_every-th sweep
    only; there it fires when the fit is at or below fit_floor, or when it
    changed by at most tol relative to the fit of the previous such sweep
    (fit_every sweeps earlier)."""
    k = len(fits)
    if k == 0 or k % fit_every:
        return False
    if fits[-1] <= fit_floor:
        return True
    if k <= fit_every:
        return False
    prev = fits[-1 - fit_every]
    return abs(fits[-1] - prev) <= tol * prev


def mf_cp_als(X, Z, init, max_sweeps, tol=1e-4, fit_floor=1e-7, allow_fallback=True, fit_every=1):
    """Matrix-free CP-ALS with the stopping rule ``stops``."""
    st = MatFreeCPALS(X, Z, init, allow_fallback)
    fits = []
    for _ in range(max_sweeps):
        fits.append(st.sweep())
        if stops(fits, tol, fit_floor, fit_every):
            break
    return dict(fits=fits, lam=st.lam, F=st.F, fallbacks=st.fallbacks, state=st)
