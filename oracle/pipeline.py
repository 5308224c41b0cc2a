"""Oracle: Procedure * end to end (split, build M on A~, s+1 solves, SMW recovery).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import drop as drop_mod
from . import krylov, lsq, pattern, smw, spai
from . import split as split_mod


def build_M(S, kind="A2", drop="none", tau=1e-3, delta=0.4, steps=3, per_step=5,
            init="A", cols=None):
    """Build M (CSC) for A~ of split S; returns (M, info dict)."""
    At = S.At
    n = At.shape[0]
    ks = list(range(n)) if cols is None else list(cols)
    if kind in ("A", "A2"):
        J = pattern.static_pattern(At, kind, ks)
        Is, ms, res = lsq.build_columns(At, J, ks)
    elif kind == "spai":
        out = spai.spai(At, steps, per_step, delta, init, ks)
        J = [o[0] for o in out]
        Is = [o[1] for o in out]
        ms = [o[2] for o in out]
        res = np.asarray([o[3] for o in out])
    else:
        raise ValueError(kind)
    M = drop_mod.assemble(n, J, ms, drop, tau, delta, At, ks)
    return M, dict(J=J, I=Is, m=ms, res=res)


def equilibration_factor(A, b) -> float:
    """Section 4's scaling of b: alpha = rho / ||b|| with rho = ||A||_F / sqrt(n), the
    root-mean-square column norm of A, so that ||alpha b|| is comparable to the
    column norms of A (and so to the ||u_j||)."""
    n = A.shape[0]
    rho = float(sp.linalg.norm(sp.csr_matrix(A))) / np.sqrt(n)
    b0 = float(np.linalg.norm(b))
    return rho / b0 if b0 > 0.0 and rho > 0.0 else 1.0


def solve(A, b, S, M, eps=1e-8, method="bicgstab", restart=30, maxit=500, equilibrate=False):
    """Solve the s+1 systems and recover x_hat; returns dict with x, rr, c, iters.
    With equilibrate, A (alpha x) = alpha b is solved instead (alpha from
    ``equilibration_factor``) and x is scaled back; rr is relative to b."""
    n = A.shape[0]
    s = S.s
    b_in = np.asarray(b, dtype=np.float64)
    alpha = equilibration_factor(A, b_in) if equilibrate else 1.0
    b = alpha * b_in if alpha != 1.0 else b_in
    R = np.zeros((n, s + 1))
    R[:, 0] = b
    if s:
        R[:, 1:] = S.U.toarray()
    thr = krylov.thresholds(float(np.linalg.norm(b)), s, eps)
    At = sp.csr_matrix(S.At)
    Mr = sp.csr_matrix(M)
    X, its, sts = krylov.solve_block(At, Mr, R, thr, method, restart, maxit)
    x, z, c = smw.recover(X[:, 0], X[:, 1:], S.D)
    if alpha != 1.0:
        x = x / alpha
    rr = smw.relres(A, x, b_in)
    return dict(x=x, Y=X, z=z, c=c, rr=rr, iters=its, statuses=sts, alpha=alpha)


def run(A, b, kind="A2", drop="none", tau=1e-3, eps=1e-8, method="bicgstab",
        restart=30, maxit=500, equilibrate=False, **spai_kw):
    S = split_mod.split(A)
    M, info = build_M(S, kind, drop, tau, **spai_kw)
    out = solve(A, b, S, M, eps, method, restart, maxit, equilibrate)
    out.update(split=S, M=M, build=info)
    return out
