"""Oracle: split A = A~ + U V^T (Procedure *, step 1; Section 3 (split); Section 4).

Test infrastructure only (see the package docstring).

Definitions followed:
* p = floor(nnz(A)/n), the average number of nonzeros per column (Section 4,
  first issue; it matches the p column of Table 3 for every listed matrix).
* column j is irregular iff its nonzero count exceeds ``dense_factor * p``
  (the paper uses 10p; "exceeds" is read as strict >).
* each irregular column keeps its diagonal and the ``keep - 1`` off-diagonal
  nonzeros nearest to the diagonal, ties broken by the smaller row index;
  keep = p by default (Section 4, second issue, p_hat = p).  The alternative
  rule keeps the largest-magnitude entries instead.
* U holds the dropped entries, column d of U belongs to the d-th irregular
  column in ascending order, V = (e_{j_1}, ..., e_{j_s}) (Section 3 (split)).
* A~ is A with the dropped entries removed: values are copied, never recomputed.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


class ZeroDiagonal(ValueError):
    """An irregular column has no diagonal entry (the paper applies dmperm first)."""


@dataclasses.dataclass
class Split:
    At: sp.csr_matrix       # A~ (CSR, sorted)
    U: sp.csc_matrix        # n x s, dropped entries
    D: np.ndarray           # irregular column indices j_1 < ... < j_s
    p: int
    keep: int

    @property
    def s(self) -> int:
        return int(self.D.size)


def split(A: sp.csr_matrix, dense_factor: float = 10.0, keep: int | None = None,
          rule: str = "nearest", dense_cols=None) -> Split:
    """Split A = A~ + U V^T.  ``dense_cols`` (optional, ascending) names the
    irregular columns instead of the count rule; each is then split by the same
    keep rule."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    p = A.nnz // n
    C = A.tocsc()
    C.sort_indices()
    counts = np.diff(C.indptr)
    D = (np.flatnonzero(counts > dense_factor * p) if dense_cols is None
         else np.asarray(list(dense_cols), dtype=np.int64))
    keep_n = p if keep is None else int(keep)
    if keep_n < 1:
        raise ValueError("keep must be >= 1")

    drop_rows, drop_cols, drop_vals, drop_d = [], [], [], []
    for d, j in enumerate(D):
        lo, hi = C.indptr[j], C.indptr[j + 1]
        rows = C.indices[lo:hi].tolist()
        vals = C.data[lo:hi].tolist()
        if j not in rows:
            raise ZeroDiagonal(f"irregular column {j} has no diagonal entry")
        off = [(i, v) for i, v in zip(rows, vals) if i != j]
        if rule == "nearest":
            off.sort(key=lambda t: (abs(t[0] - j), t[0]))
        elif rule == "largest":
            off.sort(key=lambda t: (-abs(t[1]), t[0]))
        else:
            raise ValueError(rule)
        for i, v in off[keep_n - 1:]:
            drop_rows.append(i)
            drop_cols.append(j)
            drop_vals.append(v)
            drop_d.append(d)

    drop_rows = np.asarray(drop_rows, dtype=np.int64)
    drop_cols = np.asarray(drop_cols, dtype=np.int64)
    keys_drop = drop_rows * n + drop_cols
    rows_all = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.indptr))
    keys_all = rows_all * n + A.indices.astype(np.int64)
    keep_mask = ~np.isin(keys_all, keys_drop)

    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows_all[keep_mask] + 1, 1)
    indptr = np.cumsum(indptr)
    At = sp.csr_matrix((A.data[keep_mask].copy(), A.indices[keep_mask].copy(), indptr),
                       shape=(n, n))
    U = sp.csc_matrix((np.asarray(drop_vals, dtype=np.float64),
                       (drop_rows, np.asarray(drop_d, dtype=np.int64))), shape=(n, D.size))
    U.sort_indices()
    return Split(At=At, U=U, D=D.astype(np.int64), p=int(p), keep=keep_n)


def dense_U(S: Split) -> np.ndarray:
    """U as a dense n x s float64 array."""
    return S.U.toarray()
