"""Oracle: PSAI(tol), the adaptive power-pattern SAI of Section 2.2, on A~.

Test infrastructure only (see the package docstring).

Column k starts from a^(0) = e_k and S^(0) = {k} (the BPSAI start of Section
2.2).  Loop l = 0, 1, ..., l_max:
  a^(l+1) = A~ a^(l);  S^(l+1) = P(a^(l+1)) union S^(l);
  m_k = argmin ||A~(L, S^(l+1)) m - e_k(L)||, L = nonzero rows of A~(:, S^(l+1))
        (the augmented (lsprob));
  the entries of the newly computed m_k with |m_jk| <= tol_k are dropped,
        tol_k = delta / (nnz(m_k) ||A~||_1)                                  (tolk);
  stop when ||A~ m_k - e_k|| <= delta, or after loop l_max.

Readings fixed here:
* P(a^(l+1)) is taken structurally (boolean): the nonzero rows of
  A~(:, P(a^(l))), as for P(|A~|^2), so no numeric cancellation removes an index;
* dropping applies to the pattern of m_k only; the power pattern P(a^(l)) keeps
  growing undropped;
* the drop is the TOLK rule of ``drop`` (nnz(m_k) = |S^(l+1)| before dropping,
  the entry of largest magnitude always kept), and kept entries keep their
  values (no re-solve);
* the stopping test uses the residual of the solution just computed (before
  its entries are dropped); the column of M is the dropped m_k of the last loop;
* each augmented problem is solved from scratch (the paper updates the QR
  factors; the minimiser is the same).
"""
from __future__ import annotations

import numpy as np

from .drop import drop_column, norm1
from .lsq import solve_column
from .pattern import as_csc, rows_of


def psai_tol_column(C, k: int, delta: float, lmax: int, a1: float):
    """Return (S, m, res, loops) for column k: the final (dropped) pattern and
    values, the residual norm of the last undropped solution, and the number of
    loops run (1 .. lmax + 1)."""
    S = np.array([k], dtype=np.int64)
    F = np.array([k], dtype=np.int64)
    res = np.inf
    m = np.zeros(0)
    for l in range(lmax + 1):
        F = rows_of(C, F)
        S = np.union1d(S, F)
        _, m, res = solve_column(C, S, k)
        keep = drop_column(m, delta / (S.size * a1))
        S, m = S[keep], m[keep]
        if res <= delta:
            return S, m, res, l + 1
    return S, m, res, lmax + 1


def psai_tol(At, delta: float = 0.4, lmax: int = 10, cols=None):
    """PSAI(tol) for every column (or ``cols``): lists of patterns and values,
    residual norms and loop counts."""
    C = as_csc(At)
    a1 = norm1(C)
    ks = range(C.shape[0]) if cols is None else cols
    Ss, ms, rs, ls = [], [], [], []
    for k in ks:
        S, m, r, nl = psai_tol_column(C, int(k), delta, lmax, a1)
        Ss.append(S)
        ms.append(m)
        rs.append(r)
        ls.append(nl)
    return Ss, ms, np.asarray(rs), np.asarray(ls)
