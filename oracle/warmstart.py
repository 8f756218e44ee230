"""Warm-start inputs and targets for CP-ALS (test infrastructure only).

The paper observes (Results, around the cost discussion of the CPD) that
the number of ALS sweeps depends strongly on the initial guess and leaves a
better guess to future work.  The warm start built here starts the CP
factors from columns of the THC factors themselves: with a diagonal core Z
the THC form is already an exact CP decomposition whose factor columns are
the grid columns X_m[:, P] (eq. THC with Z_PQ = z_P delta_PQ), so a
selection of R_cp grid points, each scaled, is a natural initial CP.

Everything here is plain float64 NumPy written from those definitions:

  features(X0, Z)     per grid point P, eight numbers computable from
                      (X0, Z, S = X0^T X0) before any CP exists:
                        0 log Z_PP            1 log sum_Q |Z_PQ|
                        2 log S_PP            3 log sum_Q S_PQ^2
                        4 log max_p |X0_pP|   5 participation ratio of
                          X0[:, P], (sum x^2)^2 / (n sum x^4)
                        6 log sum_Q S_PQ^2 |Z_PQ|
                        7 log Z_PP S_PP^2  (the heuristic ranking score)
                      log(v) means log(max(v, 1e-300)).  Each feature is
                      standardised over the grid points of its problem
                      (population mean and standard deviation; a feature
                      whose deviation is below 1e-9 max(1, |mean|), i.e.
                      constant up to rounding, becomes 0), which makes the features
                      independent of N and of the scale of X and Z.
  heuristic_scores    the raw feature 7: grid points with a large diagonal
                      contribution Z_PP S_PP^2 to ||G||^2 come first.
  select_init         top-R_cp grid points by score (ties: smaller P first),
                      F_m[:, k] = exp(ell_{P_k}) X_m[:, P_k], optionally
                      blended with the caller's random guess R:
                      + sigma ||X_m[:, P_k]|| R_m[:, k] / ||R_m[:, k]|| inside
                      the bracket.  The grid columns are positive and
                      overlap strongly, so a pure column start is nearly
                      degenerate; the blend breaks that symmetry.
  match_labels        training targets from a converged CPD: greedy
                      one-to-one matching of its mode-0 columns to grid
                      columns by |cosine| (largest first; ties: smaller k,
                      then smaller P); a matched P gets target 1 and the
                      log of its least-squares scale, averaged over modes.

Pins (tests/test_oracle_warmstart.py): closed-form participation ratios,
invariance of the standardised features under X -> cX, Z -> cZ, grid-point
permutation equivariance, zero mean / unit variance; the planted diagonal
core, where the selected and scaled grid columns are an exact CPD (one ALS
sweep reaches the fit floor); the blend's norm identity for a random part
orthogonal to the grid column; label recovery of a planted column choice
with known scales; greedy matching against an exhaustive pick-the-maximum
loop on small inputs.
"""
import numpy as np

N_FEATURES = 8
_TINY = 1e-300


def _log(v):
    return np.log(np.maximum(v, _TINY))


def raw_features(X0, Z):
    n = X0.shape[0]
    S = X0.T @ X0
    x2 = (X0 ** 2).sum(axis=0)
    x4 = (X0 ** 4).sum(axis=0)
    pr = np.where(x4 > 0, x2 ** 2 / (n * np.where(x4 > 0, x4, 1.0)), 0.0)
    zd = np.diag(Z)
    sd = np.diag(S)
    f = np.empty((X0.shape[1], N_FEATURES))
    f[:, 0] = _log(zd)
    f[:, 1] = _log(np.abs(Z).sum(axis=1))
    f[:, 2] = _log(sd)
    f[:, 3] = _log((S ** 2).sum(axis=1))
    f[:, 4] = _log(np.abs(X0).max(axis=0))
    f[:, 5] = pr
    f[:, 6] = _log((S ** 2 * np.abs(Z)).sum(axis=1))
    f[:, 7] = _log(zd * sd ** 2)
    return f


def standardise(f):
    mu = f.mean(axis=0)
    sd = np.sqrt(((f - mu) ** 2).mean(axis=0))
    out = np.zeros_like(f)
    ok = sd > 1e-9 * np.maximum(1.0, np.abs(mu))
    out[:, ok] = (f[:, ok] - mu[ok]) / sd[ok]
    return out


def features(X0, Z):
    return standardise(raw_features(X0, Z))


def heuristic_scores(X0, Z):
    return raw_features(X0, Z)[:, 7]


def selection_order(s):
    """Grid points by decreasing score, ties broken by the smaller index."""
    s = np.asarray(s, dtype=np.float64)
    return np.lexsort((np.arange(len(s)), -s))


def select_init(X, s, ell, r_cp, noise=None, sigma=0.0):
    """Initial CP factors from the top-r_cp grid points P_k:
    F_m[:, k] = exp(ell_{P_k}) (X_m[:, P_k] + sigma ||X_m[:, P_k]|| R_m[:, k] / ||R_m[:, k]||)
    with R = noise (the caller's random guess; sigma = 0 or noise None: the
    plain grid columns)."""
    order = selection_order(s)[:r_cp]
    scale = np.exp(np.asarray(ell, dtype=np.float64)[order])
    out = []
    for m, x in enumerate(X):
        cols = x[:, order]
        if noise is not None and sigma != 0.0:
            R = np.asarray(noise[m], dtype=np.float64)
            rn = np.sqrt((R ** 2).sum(axis=0))
            xn = np.sqrt((cols ** 2).sum(axis=0))
            unit = np.where(rn > 0, R / np.where(rn > 0, rn, 1.0), 0.0)
            cols = cols + sigma * xn[None, :] * unit
        out.append(cols * scale[None, :])
    return out


def _abs_cosines(F0, X0):
    fn = np.sqrt((F0 ** 2).sum(axis=0))
    xn = np.sqrt((X0 ** 2).sum(axis=0))
    C = F0.T @ X0
    den = fn[:, None] * xn[None, :]
    return np.where(den > 0, np.abs(C) / np.where(den > 0, den, 1.0), 0.0)


def greedy_match(A):
    """One-to-one matching of rows k to columns P of A, largest entry first,
    ties: smaller k, then smaller P.  Returns match[k] = P."""
    R, Pn = A.shape
    order = np.lexsort((np.tile(np.arange(Pn), R), np.repeat(np.arange(R), Pn), -A.ravel()))
    match = np.full(R, -1, dtype=np.int64)
    used = np.zeros(Pn, dtype=bool)
    left = min(R, Pn)
    for idx in order:
        k, P = divmod(int(idx), Pn)
        if match[k] < 0 and not used[P]:
            match[k] = P
            used[P] = True
            left -= 1
            if left == 0:
                break
    return match


def match_labels(X, F, lam):
    """Targets (y, ell, mask) over the grid points of one problem from a
    converged CPD (F with unit columns, weights lam)."""
    r_thc = X[0].shape[1]
    match = greedy_match(_abs_cosines(F[0], X[0]))
    y = np.zeros(r_thc)
    ell = np.zeros(r_thc)
    mask = np.zeros(r_thc)
    w = np.abs(np.asarray(lam, dtype=np.float64)) ** 0.25
    for k, P in enumerate(match):
        if P < 0:
            continue
        y[P] = 1.0
        logs = []
        ok = True
        for m in range(4):
            xx = float(X[m][:, P] @ X[m][:, P])
            if xx <= 0:
                ok = False
                break
            c = w[k] * float(F[m][:, k] @ X[m][:, P]) / xx
            logs.append(np.log(max(abs(c), _TINY)))
        if ok:
            ell[P] = np.mean(logs)
            mask[P] = 1.0
    return y, ell, mask
