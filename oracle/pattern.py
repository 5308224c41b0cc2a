"""Oracle: static sparsity patterns of M and the row sets of the LS problems.

Test infrastructure only (see the package docstring).

* P(A~): J_k = rows of A~(:, k).
* P(|A~|^2): J_k = union over j in P(A~(:, k)) of P(A~(:, j)) - the l = 2 member
  of the BPSAI envelope P((I + |A~|)^l) of Section 2.2; taken structurally
  (boolean), so no numeric cancellation can remove an index.  Because A~ has a
  full diagonal, P(|A~|^2) = P((I + |A~|)^2).
* I_k (the paper's L_k): the nonzero rows of A~(:, J_k), i.e. the union of
  P(A~(:, j)) over j in J_k (Section 2, text before (lsprob)).

All index lists are returned sorted ascending, as int64 arrays.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def as_csc(At) -> sp.csc_matrix:
    C = sp.csc_matrix(At)
    C.sort_indices()
    return C


def col_rows(C: sp.csc_matrix, j: int) -> np.ndarray:
    return C.indices[C.indptr[j]:C.indptr[j + 1]].astype(np.int64)


def pattern_A(C: sp.csc_matrix, k: int) -> np.ndarray:
    return col_rows(C, k)


def pattern_A2(C: sp.csc_matrix, k: int) -> np.ndarray:
    out = set()
    for j in col_rows(C, k).tolist():
        out.update(col_rows(C, j).tolist())
    return np.array(sorted(out), dtype=np.int64)


def rows_of(C: sp.csc_matrix, J) -> np.ndarray:
    """I = sorted union of P(A~(:, j)) for j in J."""
    out = set()
    for j in np.asarray(J).tolist():
        out.update(col_rows(C, j).tolist())
    return np.array(sorted(out), dtype=np.int64)


def static_pattern(At, kind: str, cols=None):
    """J_k for every k (or for ``cols``) under ``kind`` in {"A", "A2"}."""
    C = as_csc(At)
    n = C.shape[0]
    f = {"A": pattern_A, "A2": pattern_A2}[kind]
    ks = range(n) if cols is None else cols
    return [f(C, int(k)) for k in ks]
