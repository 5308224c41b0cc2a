"""Oracle: gradients of a scalar loss through x = A^{-1} b, via the split of A^T.

Test infrastructure only (see the package docstring).

The paper solves Ax = b only; the gradient is derived here from its Theorem
3.1 applied to the transpose.  With A = A~ + U V^T we have
A^T = A~^T + V U^T, so for g = dL/dx the adjoint solution lambda = A^{-T} g is
    eta = A~^{-T} g,  Z = A~^{-T} V,  lambda = eta - Z (I + U^T Z)^{-1} (U^T eta),
i.e. s+1 systems with A~^T (right-preconditioned by M^T, which approximates
A~^{-T}) and an s x s solve.  Then dL/db = lambda and dL/dA_ij = -lambda_i x_j
for every stored nonzero (i, j) of A (the derivative of A^{-1} b with respect
to A_ij is -A^{-1} e_i x_j).  Stopping rules are the Section 4 theorem's with
the roles of U and V exchanged: column 0 stops at (eps/2)||g||, the columns
with right-hand side e_{j_d} (norm 1) at eps ||g|| / (2 sqrt(s)).

When the forward solve's W = A~^{-1} U is at hand, the transpose of Theorem
3.1's formula, A^{-T} = A~^{-T} (I - V K^{-T} W^T) with K = I + V^T W, needs
one system with A~^T instead of s+1 (adjoint_from_forward), with the true
adjoint residual checked and corrected while it exceeds eps ||g||.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .krylov import solve_block, thresholds


def adjoint(S, M, x, g, eps=1e-8, method="bicgstab", restart=30, maxit=500):
    """Return dict(lam, grad_b, eta, Z, iters, statuses)."""
    n = S.At.shape[0]
    s = S.s
    AtT = sp.csr_matrix(S.At.T)
    MT = sp.csr_matrix(sp.csc_matrix(M).T)
    R = np.zeros((n, s + 1))
    R[:, 0] = g
    for d, j in enumerate(S.D.tolist()):
        R[j, d + 1] = 1.0
    thr = thresholds(float(np.linalg.norm(g)), s, eps)
    X, its, sts = solve_block(AtT, MT, R, thr, method, restart, maxit)
    eta = X[:, 0]
    Z = X[:, 1:]
    if s:
        Ud = S.U.toarray()
        K = np.eye(s) + Ud.T @ Z
        w = np.linalg.solve(K, Ud.T @ eta)
        lam = eta - Z @ w
    else:
        lam = eta.copy()
    return dict(lam=lam, grad_b=lam, eta=eta, Z=Z, iters=its, statuses=sts)


def grad_A_values(A, lam, x):
    """dL/dA_ij = -lambda_i x_j for the stored entries of A, in A's CSR order."""
    A = sp.csr_matrix(A)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    return -lam[rows] * x[A.indices]


def forward_correction(W, D, v):
    """v - V K^{-T} W^T v with K = I + V^T W (V = (e_{j_1} .. e_{j_s}), D = j).

    Theorem 3.1 gives A^{-1} = A~^{-1} - W K^{-1} V^T A~^{-1} with W = A~^{-1} U;
    its transpose is A^{-T} = A~^{-T} (I - V K^{-T} W^T).  So A^{-T} v is one
    solve with A~^T on this corrected right-hand side.  Returns (rhs, z)."""
    rhs = np.array(v, dtype=np.float64, copy=True)
    s = len(D)
    if s == 0:
        return rhs, np.zeros(0)
    K = np.eye(s) + W[D, :]
    z = np.linalg.solve(K.T, W.T @ v)
    rhs[D] -= z
    return rhs, z


def adjoint_from_forward(S, M, W, g, eps=1e-8, method="bicgstab", restart=30, maxit=500, passes=4):
    """lambda = A^{-T} g from the forward solve's W (n x s, approximately A~^{-1} U).

    Each pass solves A~^T d = forward_correction(W, D, res) for one column (M^T
    as right preconditioner) and adds d to lambda; res starts as g and is then
    the true residual g - A^T lambda = g - A~^T lambda - V (U^T lambda).  The
    passes stop once ||g - A^T lambda|| < eps ||g||.  After a pass the true
    residual is (I + V W^T) r_s - V R^T d (r_s = the solve's residual, R = U -
    A~ W the forward's auxiliary residuals, d the pass's solution): the second
    term, W's own error, usually keeps the first pass above eps and the next
    pass removes it.  The first solve stops at (eps/2) ||g||, each later one at
    (eps/2) ||g|| / a with a = max(1, ||(I + V W^T) r_s|| / ||r_s||) of the pass
    before, so that the next pass's (I + V W^T) r_s stays below (eps/2) ||g||.
    Returns dict(lam, grad_b, iters, passes, rr, status)."""
    n = S.At.shape[0]
    D = np.asarray(S.D, dtype=np.int64)
    AtT = sp.csr_matrix(S.At.T)
    MT = sp.csr_matrix(sp.csc_matrix(M).T)
    U = sp.csc_matrix(S.U)
    gnorm = float(np.linalg.norm(g))
    lam = np.zeros(n)
    if gnorm == 0.0:
        return dict(lam=lam, grad_b=lam, iters=0, passes=0, rr=0.0, status="converged")
    res = np.array(g, dtype=np.float64, copy=True)
    thr = 0.5 * eps * gnorm
    iters = 0
    rr = np.inf
    p = 0
    for p in range(1, passes + 1):
        rhs, _ = forward_correction(W, D, res)
        X, its, sts = solve_block(AtT, MT, rhs[:, None], [thr], method, restart, maxit)
        iters += int(its[0])
        lam = lam + X[:, 0]
        rho = g - AtT @ lam
        if len(D):
            rho[D] -= U.T @ lam
        rnorm = float(np.linalg.norm(rho))
        rr = rnorm / gnorm
        if rr < eps:
            break
        rs = rhs - AtT @ X[:, 0]
        ars = rs.copy()
        if len(D):
            ars[D] += W.T @ rs
        nrs = float(np.linalg.norm(rs))
        amp = max(1.0, float(np.linalg.norm(ars)) / nrs) if nrs > 0.0 else 1.0
        thr = 0.5 * eps * gnorm / amp
        res = rho
    return dict(lam=lam, grad_b=lam, iters=iters, passes=p, rr=rr,
                status="converged" if rr < eps else "maxit")
