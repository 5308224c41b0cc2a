"""Oracle: SPAI adaptive pattern (Grote-Huckle augmentation) on A~.

Test infrastructure only (see the package docstring).

Section 2.1.  For column k with current pattern S (= J_k) and LS solution
m_hat on the rows L_k (= I_k):
  r = A~(:, S) m_hat - e_k; stop when ||r|| <= delta;
  L = rows where r is nonzero, taken structurally as I_k (every row of I_k
      carries a generically nonzero residual);
  N = indices of nonzero columns of A~(L, :);  candidates J~ = N \\ S   (candi);
  for j in J~ the 1-D problem min_mu ||r + mu A~ e_j||                (ls1d)
      has mu_j = -r^T A~ e_j / ||A~ e_j||^2                           (muj)
      and new residual norm rho_j^2 = ||r||^2 - (r^T A~ e_j)^2/||A~ e_j||^2  (rhoj);
  the few candidates of smallest rho_j are added to S, I_k is recomputed and
  the LS problem is solved again.

Readings fixed here:
* the initial pattern is P(A~(:, k)) ("A", default) or {k} ("diag", the
  paper's experiments);
* exactly min(per_step, |J~|) indices are added per step;
* candidates are ranked by the gain g_j = (r^T A~ e_j)^2 / ||A~ e_j||^2,
  largest first, which orders them exactly as rho_j^2 = ||r||^2 - g_j
  smallest first but without the cancellation in that subtraction; ties go
  to the smaller column index;
* the augmented problem is re-solved from scratch (the paper updates the QR
  factors instead; both give the same m_hat in exact arithmetic);
* at most ``steps`` augmentations, then a final solve on the last pattern.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .lsq import dense_block, solve_column
from .pattern import as_csc, col_rows


def column_norms2(C: sp.csc_matrix) -> np.ndarray:
    """||A~ e_j||^2 for every column j."""
    out = np.zeros(C.shape[1])
    for j in range(C.shape[1]):
        v = C.data[C.indptr[j]:C.indptr[j + 1]]
        out[j] = float(np.dot(v, v))
    return out


def candidate_gains(C, R, cn2, J, I, r):
    """Return (J~ sorted, tau_j = r^T A~ e_j, g_j, rho_j^2) for the current step."""
    Jset = set(np.asarray(J).tolist())
    N = set()
    for i in np.asarray(I).tolist():
        N.update(R.indices[R.indptr[i]:R.indptr[i + 1]].tolist())
    cand = np.array(sorted(N - Jset), dtype=np.int64)
    rpos = {int(i): t for t, i in enumerate(np.asarray(I).tolist())}
    tau = np.zeros(cand.size)
    for t, j in enumerate(cand.tolist()):
        lo, hi = C.indptr[j], C.indptr[j + 1]
        acc = 0.0
        for i, v in zip(C.indices[lo:hi].tolist(), C.data[lo:hi].tolist()):
            if i in rpos:
                acc += r[rpos[i]] * v
        tau[t] = acc
    g = tau * tau / cn2[cand]
    rho2 = float(np.dot(r, r)) - g
    return cand, tau, g, rho2


def select(cand, g, count):
    """Indices of the ``count`` largest gains, ties to the smaller column index."""
    order = sorted(range(cand.size), key=lambda t: (-g[t], cand[t]))
    return np.sort(cand[order[:count]])


def spai_column(C, R, cn2, k, steps=3, per_step=5, delta=0.4, init="A"):
    """Return (J_k final, I_k, m_hat, res_k, number of augmentation steps taken)."""
    J = col_rows(C, k) if init == "A" else np.array([k], dtype=np.int64)
    taken = 0
    for _ in range(steps):
        I, m, res = solve_column(C, J, k)
        if res <= delta:
            return J, I, m, res, taken
        Ah = dense_block(C, I, J)
        r = Ah @ m - (I == k).astype(np.float64)
        cand, tau, g, rho2 = candidate_gains(C, R, cn2, J, I, r)
        if cand.size == 0:
            return J, I, m, res, taken
        add = select(cand, g, min(per_step, cand.size))
        J = np.array(sorted(set(J.tolist()) | set(add.tolist())), dtype=np.int64)
        taken += 1
    I, m, res = solve_column(C, J, k)
    return J, I, m, res, taken


def spai(At, steps=3, per_step=5, delta=0.4, init="A", cols=None):
    C = as_csc(At)
    R = sp.csr_matrix(At)
    R.sort_indices()
    cn2 = column_norms2(C)
    ks = range(C.shape[0]) if cols is None else cols
    out = []
    for k in ks:
        out.append(spai_column(C, R, cn2, int(k), steps, per_step, delta, init))
    return out
