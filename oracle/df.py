"""Density-fitting (DF) tensors and their exact THC form (test
infrastructure only).

The DF approximation of the two-electron tensor (eq. df_loss),

  G[p,q,r,s] = sum_X B[(p,q), X] B[(r,s), X]      (row (p, q) = p n + q),

is a THC tensor (eq. THC) whose grid index runs over the orbital pairs:
with P = (p', q') and Q = (r', s'),

  X0[p, P] = [p = p'],  X1[q, P] = [q = q'],  X2 = X0,  X3 = X1,
  Z[P, Q]  = sum_X B[P, X] B[Q, X]                 (Z = B B^T, n^2 x n^2),

since sum_{P,Q} X0[p,P] X1[q,P] Z[P,Q] X2[r,Q] X3[s,Q] = Z[(p,q),(r,s)].
The matrix-free CP-ALS of the THC form is then CP-ALS on the DF loss, at
the O(n^4 R_cp) cost per sweep the paper gives for the DF variant
(R_thc = n^2), against O(n R_thc R_cp + R_thc^2 R_cp) with a THC rank
proportional to n.

Pins (tests/test_oracle_df.py): the dense tensor of the THC form equals
the DF tensor entry by entry; the matrix-free CP-ALS of the THC form
follows the dense CP-ALS of the DF tensor.
"""
import numpy as np


def df_tensor(B, n):
    """G[p,q,r,s] = sum_X B[(p,q),X] B[(r,s),X] (dense; tiny n only)."""
    return (B @ B.T).reshape(n, n, n, n)


def df_to_thc(B, n):
    """(X0, X1, Z) of the exact THC form: selection matrices and B B^T."""
    pairs = np.arange(n * n)
    X0 = (pairs[None, :] // n == np.arange(n)[:, None]).astype(np.float64)
    X1 = (pairs[None, :] % n == np.arange(n)[:, None]).astype(np.float64)
    return X0, X1, B @ B.T
