"""Oracle: right-preconditioned Krylov solves of the s+1 systems with A~.

Test infrastructure only (see the package docstring).

Section 3 (regprob), (auxi): A~ y = b and A~ w_j = u_j.  Section 5 solves them
with BiCGStab, right preconditioning (A~ M u = rhs, x = M u), x_0 = 0, at
most 500 iterations (also GMRES(20) is mentioned there).  Stopping rules are
those of the Section 4 theorem with c = 1:
    column 0 (rhs b):   ||b - A~ y|| < (eps/2) ||b||                 (stopb)
    column j (rhs u_j): ||u_j - A~ w_j|| < eps ||b|| / (2 sqrt(s))    (stopU2, c = 1)
The thresholds are computed by ``thresholds`` and passed in as absolute
numbers; every solve below handles one right-hand side.

Readings fixed here (the paper names the solvers but not their variants):
* BiCGStab is van der Vorst's algorithm with r_hat = r_0.  Convergence is
  declared only on the true residual rhs - A~ x, which is computed whenever
  the recursively updated residual (s at the half step, r at the full step)
  falls below the threshold; if the true residual at the full step does not
  pass, it replaces the recursive one.  A breakdown (|rho| or |r_hat^T v| or
  |omega| below 1e-300, or t = 0) restarts once with r_hat = r; a second one
  ends the solve with status "breakdown".
* GMRES(m) uses modified Gram-Schmidt Arnoldi and Givens rotations; the
  solution is formed at the end of each cycle or when the rotated residual
  estimate falls below the threshold, and convergence is again declared on
  the true residual.
Iteration counts: one BiCGStab iteration = two preconditioned products; one
GMRES iteration = one Arnoldi step.
"""
from __future__ import annotations

import math

import numpy as np

TINY = 1e-300


def thresholds(b_norm: float, s: int, eps: float, u_norms=None, c: float = 1.0):
    """Absolute residual thresholds for the s+1 columns [b, u_1..u_s] (stopb, stopU2)."""
    t = [0.5 * eps * b_norm]
    for _ in range(s):
        t.append(eps * b_norm / (2.0 * math.sqrt(s) * c))
    return np.asarray(t)


def bicgstab(A, M, rhs, thr, maxit=500, force_restart_at=(), trace=None):
    """Return (x, iterations, status) with status in {"converged", "maxit", "breakdown"}.

    Two test hooks leave the arithmetic unchanged: ``force_restart_at`` lists
    iterations at whose end the solver restarts exactly as after a breakdown of
    omega (so that the restart can be exercised on well-conditioned systems),
    and ``trace``, a list, receives ``(event, iteration, state)`` tuples for
    every restart ("restart") and residual replacement ("replace"), where state
    holds copies of x, r, r_hat, p and v right after the event (and, for a
    replacement, the recursive residual it replaced as r_rec).
    """
    force = set(int(i) for i in force_restart_at)
    rhs = np.asarray(rhs, dtype=np.float64)
    n = rhs.size
    x = np.zeros(n)
    r = rhs.copy()
    if np.linalg.norm(r) < thr:
        return x, 0, "converged"
    rhat = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros(n)
    p = np.zeros(n)
    restarts = 0
    it = 0

    def note(event, **extra):
        if trace is not None:
            state = dict(x=x.copy(), r=r.copy(), rhat=rhat.copy(), p=p.copy(), v=v.copy())
            state.update(extra)
            trace.append((event, it, state))

    def restart():
        nonlocal rhat, rho_old, alpha, omega, v, p, restarts
        restarts += 1
        rhat = r.copy()
        rho_old = alpha = omega = 1.0
        v = np.zeros(n)
        p = np.zeros(n)
        note("restart")
        return restarts <= 1

    while it < maxit:
        it += 1
        rho = float(rhat @ r)
        if abs(rho) < TINY:
            if not restart():
                return x, it, "breakdown"
            continue
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = M @ p
        v = A @ ph
        sigma = float(rhat @ v)
        if abs(sigma) < TINY:
            if not restart():
                return x, it, "breakdown"
            continue
        alpha = rho / sigma
        s = r - alpha * v
        if np.linalg.norm(s) < thr:
            xh = x + alpha * ph
            if np.linalg.norm(rhs - A @ xh) < thr:
                return xh, it, "converged"
        sh = M @ s
        t = A @ sh
        tt = float(t @ t)
        if tt < TINY:
            if not restart():
                return x, it, "breakdown"
            continue
        omega = float(t @ s) / tt
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho_old = rho
        if np.linalg.norm(r) < thr:
            rt = rhs - A @ x
            if np.linalg.norm(rt) < thr:
                return x, it, "converged"
            r_rec, r = r, rt
            note("replace", r_rec=r_rec)
        if abs(omega) < TINY or it in force:
            if not restart():
                return x, it, "breakdown"
    return x, it, "maxit"


def _givens(a: float, b: float):
    if b == 0.0:
        return 1.0, 0.0
    h = math.hypot(a, b)
    return a / h, b / h


def gmres(A, M, rhs, thr, restart=30, maxit=500):
    """Right-preconditioned GMRES(restart); returns (x, iterations, status)."""
    rhs = np.asarray(rhs, dtype=np.float64)
    n = rhs.size
    x = np.zeros(n)
    r = rhs.copy()
    beta = float(np.linalg.norm(r))
    if beta < thr:
        return x, 0, "converged"
    it = 0
    while it < maxit:
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        g = np.zeros(restart + 1)
        g[0] = beta
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        k = 0
        for j in range(restart):
            it += 1
            w = A @ (M @ V[j])
            for i in range(j + 1):
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            hnext = float(np.linalg.norm(w))
            H[j + 1, j] = hnext
            for i in range(j):
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            if hnext == 0.0 or abs(g[j + 1]) < thr or it >= maxit:
                break
            V.append(w / hnext)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        upd = np.zeros(n)
        for i in range(k):
            upd += y[i] * V[i]
        x = x + M @ upd
        r = rhs - A @ x
        beta = float(np.linalg.norm(r))
        if beta < thr:
            return x, it, "converged"
    return x, it, "maxit"


def solve_block(A, M, R, thr, method="bicgstab", restart=30, maxit=500, force_restart_at=()):
    """Solve A~ X = R column by column; returns (X, iterations list, statuses list).

    ``force_restart_at`` is passed to every BiCGStab solve (a test hook, see
    ``bicgstab``)."""
    R = np.asarray(R, dtype=np.float64)
    if R.ndim == 1:
        R = R[:, None]
    X = np.zeros_like(R)
    its, sts = [], []
    for c in range(R.shape[1]):
        if method == "bicgstab":
            X[:, c], it, st = bicgstab(A, M, R[:, c], thr[c], maxit, force_restart_at)
        elif method == "gmres":
            X[:, c], it, st = gmres(A, M, R[:, c], thr[c], restart, maxit)
        else:
            raise ValueError(method)
        its.append(it)
        sts.append(st)
    return X, its, sts
