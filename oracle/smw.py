"""Oracle: Sherman-Morrison-Woodbury recovery and the final residual.

Test infrastructure only (see the package docstring).

Procedure * step 3, (update1) / Section 4 (composi): with y_hat, W_hat the
approximate solutions of A~ y = b and A~ W = U and V = (e_{j_1}..e_{j_s}),
    x_hat = y_hat - W_hat (I + V^T W_hat)^{-1} (V^T y_hat),
V^T y_hat = y_hat[D], V^T W_hat = W_hat[D, :].  c = ||(I + V^T W_hat)^{-1} V^T y_hat||
(the constant of the Section 4 theorem) and rr = ||b - A x_hat|| / ||b||  (rrnorm).
The s x s system is solved by LAPACK's LU with partial pivoting.
"""
from __future__ import annotations

import numpy as np


class SingularK(np.linalg.LinAlgError):
    """I + V^T W is singular: by Theorem 3.1 A itself is singular."""


def recover(y, W, D):
    """Return (x_hat, z, c)."""
    y = np.asarray(y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64).reshape(y.size, -1)
    D = np.asarray(D, dtype=np.int64)
    s = D.size
    if s == 0:
        return y.copy(), np.zeros(0), 0.0
    K = np.eye(s) + W[D, :]
    try:
        z = np.linalg.solve(K, y[D])
    except np.linalg.LinAlgError as e:
        raise SingularK(str(e)) from e
    x = y - W @ z
    return x, z, float(np.linalg.norm(z))


def relres(A, x, b) -> float:
    """rr = ||b - A x|| / ||b||  (rrnorm), with the original A."""
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
