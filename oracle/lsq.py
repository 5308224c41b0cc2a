"""Oracle: the column least-squares problems that define M.

Test infrastructure only (see the package docstring).

Section 2, (miniz) -> (subprob) -> (lsprob): min ||A M - I||_F over the pattern
splits into n independent problems min ||A~ m_k - e_k||; with J_k the pattern
of m_k and I_k the nonzero rows of A~(:, J_k) the problem reduces to the dense
min ||A~(I_k, J_k) m_hat - e_k(I_k)||, solved by a QR decomposition.  The
oracle forms the dense block, factors it with LAPACK's Householder QR
(numpy.linalg.qr), applies Q^T to e_hat and back-substitutes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .pattern import as_csc, rows_of


def dense_block(C, I, J) -> np.ndarray:
    """A~(I, J) as a dense float64 |I| x |J| array."""
    pos = {int(i): t for t, i in enumerate(np.asarray(I).tolist())}
    Ah = np.zeros((len(I), len(J)))
    for c, j in enumerate(np.asarray(J).tolist()):
        lo, hi = C.indptr[j], C.indptr[j + 1]
        for i, v in zip(C.indices[lo:hi].tolist(), C.data[lo:hi].tolist()):
            Ah[pos[i], c] = v
    return Ah


def solve_column(C, J, k: int):
    """Return (I_k, m_hat, res_k) for column k with pattern J (sorted).

    res_k = ||A~(:, J) m_hat - e_k||, which equals the reduced residual because
    A~(:, J) is zero outside the rows I_k.
    """
    J = np.asarray(J, dtype=np.int64)
    I = rows_of(C, J)
    Ah = dense_block(C, I, J)
    e = (I == k).astype(np.float64)
    Q, R = np.linalg.qr(Ah, mode="reduced")
    m = sla.solve_triangular(R, Q.T @ e, lower=False)
    res = float(np.linalg.norm(Ah @ m - e))
    return I, m, res


def build_columns(At, patterns, cols=None):
    """Solve the LS problem of every column; returns (I list, m list, res array)."""
    C = as_csc(At)
    ks = range(C.shape[0]) if cols is None else cols
    Is, ms, rs = [], [], []
    for t, k in enumerate(ks):
        I, m, r = solve_column(C, patterns[t], int(k))
        Is.append(I)
        ms.append(m)
        rs.append(r)
    return Is, ms, np.asarray(rs)
