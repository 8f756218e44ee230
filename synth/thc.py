"""Synthetic THC inputs (X, Z) shaped like the paper's molecular systems.

The paper factorises the two-electron integrals of water clusters and L7
complexes (Computational Details).  Those geometries, basis sets and THC
builds are not available, so a stand-in with the same structure is drawn
here: N normalised 3-D Gaussian orbitals sampled on R_thc grid points with
positive quadrature weights, and a positive-definite Coulomb-like kernel on
the grid (eq. THC: g ~= sum_PQ X_pP X_qP Z_PQ X_rQ X_sQ).

Recipe (all draws from one ``numpy.random.default_rng(seed)`` in this order):
  alpha_p ~ U[0.3, 2.0]            orbital exponents        (N,)
  c_p     ~ U[-3, 3]^3             orbital centres           (N, 3)
  r_P     ~ U[-4, 4]^3             grid points               (R, 3)
  w_P     ~ U[0.5, 1.5]            grid weights              (R,)
  X[p, P] = (2 alpha_p / pi)^(3/4) exp(-alpha_p |r_P - c_p|^2) sqrt(w_P)
  Z[P, Q] = PSD part of 1 / sqrt(|r_P - r_Q|^2 + 0.25)
The Gaussian prefactor makes each orbital unit-norm in L2.  The softened
Coulomb kernel is strictly positive definite; the eigenvalue clip is a
safeguard that is a no-op in practice.
"""
import numpy as np

# Paired (occupied, virtual) sizes of the batched Laplace-transform workload.
LT_SYSTEMS = ((20, 100), (40, 200), (80, 400))


def _thc_from_rng(rng, n, r_thc):
    alpha = rng.uniform(0.3, 2.0, n)
    centres = rng.uniform(-3.0, 3.0, (n, 3))
    grid = rng.uniform(-4.0, 4.0, (r_thc, 3))
    weights = rng.uniform(0.5, 1.5, r_thc)
    d2 = ((grid[None, :, :] - centres[:, None, :]) ** 2).sum(-1)
    X = ((2.0 * alpha / np.pi) ** 0.75)[:, None] * np.exp(-alpha[:, None] * d2)
    X *= np.sqrt(weights)[None, :]
    gg = ((grid[:, None, :] - grid[None, :, :]) ** 2).sum(-1)
    kern = 1.0 / np.sqrt(gg + 0.25)
    ev, vec = np.linalg.eigh(kern)
    ev = np.clip(ev, 0.0, None)
    Z = (vec * ev[None, :]) @ vec.T
    Z = 0.5 * (Z + Z.T)
    return np.ascontiguousarray(X), np.ascontiguousarray(Z)


def make_thc(n, r_thc, seed):
    """Return (X, Z): X is n x r_thc, Z is r_thc x r_thc, both float64 C-order."""
    return _thc_from_rng(np.random.default_rng(seed), n, r_thc)


def init_factors(dims, r_cp, seed):
    """Initial CP factors F_m ~ N(0,1)/sqrt(n_m), drawn for m = 0..3 in order."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((n, r_cp)) / np.sqrt(n) for n in dims]


def init_factors_uniform(dims, r_cp, seed):
    """The paper's initial guess: entries uniform on [-1, 1] (Computational Details)."""
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1.0, 1.0, (n, r_cp)) for n in dims]


def lt_points(count=16, t_min=0.01, t_max=20.0):
    """Log-spaced Laplace points t_k (quadrature weights are not needed: a
    scalar multiple of the tensor leaves the relative fit unchanged)."""
    return np.logspace(np.log10(t_min), np.log10(t_max), count)


def lt_quadrature(count=16, t_min=0.01, t_max=20.0):
    """Laplace points (as lt_points) with trapezoid weights in ln t:
    w_k = h t_k, h the step of ln t, so that sum_k w_k exp(-D t_k)
    approximates the integral of exp(-D t) over the covered range.  A
    synthetic stand-in for the paper's Legendre-based quadrature (12 points
    in Computational Details)."""
    t = lt_points(count, t_min, t_max)
    h = (np.log(t_max) - np.log(t_min)) / (count - 1) if count > 1 else 1.0
    return t, h * t


def make_lt_system(n_occ, n_virt, seed, rank_factor=4):
    """One molecular system of the batched workload.

    Returns (X_occ, X_virt, Z, eps_occ, eps_virt).  X comes from
    ``make_thc(n_occ + n_virt, rank_factor * (n_occ + n_virt), seed)``; rows
    0..n_occ-1 are occupied orbitals, the rest virtual.  Orbital energies are
    drawn after X and Z from the same generator: eps_occ ~ U[-1.5, -0.3],
    eps_virt ~ U[0.1, 3.0] (Hartree).
    """
    n = n_occ + n_virt
    r_thc = rank_factor * n
    rng = np.random.default_rng(seed)
    X, Z = _thc_from_rng(rng, n, r_thc)
    eps_occ = np.sort(rng.uniform(-1.5, -0.3, n_occ))
    eps_virt = np.sort(rng.uniform(0.1, 3.0, n_virt))
    return (np.ascontiguousarray(X[:n_occ]), np.ascontiguousarray(X[n_occ:]), Z,
            eps_occ, eps_virt)


def make_df(n, n_aux, seed, rank_factor=4):
    """Synthetic density-fitting factor B ((n n) x n_aux, row (p, q) = p n + q)
    of a Coulomb-like tensor, g[p,q,r,s] ~= sum_X B[(p,q),X] B[(r,s),X]
    (eq. df_loss).  Built from the THC stand-in of make_thc(n, rank_factor
    n, seed): the core Z is truncated to its n_aux leading eigenpairs,
    Z ~= C C^T with C = U sqrt(Lambda), and B[(p,q), X] = sum_P X[p,P] X[q,P]
    C[P,X]."""
    X, Z = make_thc(n, rank_factor * n, seed)
    ev, U = np.linalg.eigh(Z)
    top = np.argsort(ev)[::-1][:n_aux]
    C = U[:, top] * np.sqrt(np.clip(ev[top], 0.0, None))[None, :]
    pairs = (X[:, None, :] * X[None, :, :]).reshape(n * n, -1)
    return np.ascontiguousarray(pairs @ C)


def planted_diag_thc(n, r_thc, seed):
    """THC input with a diagonal core: Z = diag(z), z > 0.

    Then G = sum_P z_P x_P (x) x_P (x) x_P (x) x_P is exactly a rank-r_thc CP
    tensor with factors X diag(z^(1/4)); used to check that CP-ALS recovers a
    planted decomposition.
    """
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, r_thc)) / np.sqrt(n)
    z = rng.uniform(0.5, 2.0, r_thc)
    return np.ascontiguousarray(X), np.ascontiguousarray(np.diag(z))


def mlp_init_params(seed, shapes=((8, 256), (256,), (256, 256), (256,), (256, 2), (2,))):
    """Initial warm-start network parameters as one float32 vector: each
    weight matrix (fan_in x fan_out) ~ N(0, 1/fan_in), biases zero, blocks
    in the given order."""
    rng = np.random.default_rng(seed)
    out = []
    for s in shapes:
        if len(s) == 2:
            out.append((rng.standard_normal(s) / np.sqrt(s[0])).ravel())
        else:
            out.append(np.zeros(s))
    return np.concatenate(out).astype(np.float32)


def minibatch_order(rows, seed):
    """Seeded permutation of the training rows (int32)."""
    return np.random.default_rng(seed).permutation(rows).astype(np.int32)
