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


def solve(A, b, S, M, eps=1e-8, method="bicgstab", restart=30, maxit=500):
    """Solve the s+1 systems and recover x_hat; returns dict with x, rr, c, iters."""
    n = A.shape[0]
    s = S.s
    R = np.zeros((n, s + 1))
    R[:, 0] = b
    if s:
        R[:, 1:] = S.U.toarray()
    thr = krylov.thresholds(float(np.linalg.norm(b)), s, eps)
    At = sp.csr_matrix(S.At)
    Mr = sp.csr_matrix(M)
    X, its, sts = krylov.solve_block(At, Mr, R, thr, method, restart, maxit)
    x, z, c = smw.recover(X[:, 0], X[:, 1:], S.D)
    rr = smw.relres(A, x, b)
    return dict(x=x, Y=X, z=z, c=c, rr=rr, iters=its, statuses=sts)


def run(A, b, kind="A2", drop="none", tau=1e-3, eps=1e-8, method="bicgstab",
        restart=30, maxit=500, **spai_kw):
    S = split_mod.split(A)
    M, info = build_M(S, kind, drop, tau, **spai_kw)
    out = solve(A, b, S, M, eps, method, restart, maxit)
    out.update(split=S, M=M, build=info)
    return out
