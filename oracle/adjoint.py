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
