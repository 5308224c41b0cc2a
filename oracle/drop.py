"""Oracle: dropping small entries of m_k and assembling M.

Test infrastructure only (see the package docstring).

Section 2.2, PSAI(tol): after m_k is computed, entries with |m_jk| <= tol_k
are dropped, with tol_k = delta / (nnz(m_k) * ||A||_1)   (tolk).
Readings fixed here:
* "abs" uses one absolute threshold tau for every column; "tolk" uses (tolk)
  with ||A~||_1 (M approximates the inverse of A~) and nnz(m_k) = |J_k|, the
  count before dropping; "none" keeps every entry.
* the entry of largest magnitude in a column is never dropped (first one on
  ties), so no column of M becomes empty;
* dropped entries are removed without re-solving the LS problem.
M is returned in CSC (column k = m_k on its pattern) with sorted rows.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def norm1(At) -> float:
    """||A~||_1 = max column absolute sum."""
    return float(np.max(np.asarray(abs(sp.csc_matrix(At)).sum(axis=0)).ravel()))


def drop_column(m: np.ndarray, thr: float) -> np.ndarray:
    """Boolean keep-mask for one column."""
    keep = np.abs(m) > thr
    if m.size:
        keep[int(np.argmax(np.abs(m)))] = True
    return keep


def assemble(n, patterns, values, mode="none", tau=1e-3, delta=0.4, At=None,
             cols=None):
    """Build M (CSC, n x n) from per-column patterns and values after dropping."""
    ks = list(range(n)) if cols is None else list(cols)
    a1 = norm1(At) if mode == "tolk" else None
    rows, cidx, vals = [], [], []
    for t, k in enumerate(ks):
        J = np.asarray(patterns[t], dtype=np.int64)
        m = np.asarray(values[t], dtype=np.float64)
        if mode == "none":
            keep = np.ones(m.size, dtype=bool)
        elif mode == "abs":
            keep = drop_column(m, tau)
        elif mode == "tolk":
            keep = drop_column(m, delta / (J.size * a1))
        else:
            raise ValueError(mode)
        rows.append(J[keep])
        cidx.append(np.full(int(keep.sum()), k, dtype=np.int64))
        vals.append(m[keep])
    M = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cidx))),
                      shape=(n, n))
    M.sort_indices()
    return M
