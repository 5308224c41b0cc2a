"""Checks that pin the oracle to facts fixed by the paper or by mathematics.

Each check takes the function under test as an argument, so the same check
runs against the oracle (tests/test_oracle_*.py) and against deliberately
broken copies of it (tests/test_pins_catch_mistakes.py), which must fail.
Every check raises AssertionError on a mismatch.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------- split -----

def check_split_bruteforce(split_fn, A, keep=None, dense_factor=10.0):
    """Independent formulation of the Section 4 split.

    p = floor(nnz/n); a column is irregular iff count > 10p; in an irregular
    column an off-diagonal entry (i, j) is kept iff fewer than keep-1 other
    off-diagonal entries are strictly nearer (|i'-j| < |i-j|, or equal
    distance and i' < i).  Also A == A~ + U V^T exactly, entry by entry.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    Ad = A.toarray()
    nz = Ad != 0
    p = A.nnz // n
    counts = nz.sum(axis=0)
    D = [j for j in range(n) if counts[j] > dense_factor * p]
    S = split_fn(A) if keep is None else split_fn(A, keep=keep)
    kk = p if keep is None else keep
    assert S.p == p, (S.p, p)
    assert list(S.D) == D, (list(S.D), D)
    At = S.At.toarray()
    Ud = S.U.toarray()
    expect_At = Ad.copy()
    for d, j in enumerate(D):
        rows = [i for i in range(n) if nz[i, j] and i != j]
        for i in rows:
            nearer = sum(1 for i2 in rows if i2 != i and
                         (abs(i2 - j) < abs(i - j) or (abs(i2 - j) == abs(i - j) and i2 < i)))
            if nearer >= kk - 1:
                expect_At[i, j] = 0.0
                assert Ud[i, d] == Ad[i, j], (i, j)
            else:
                assert Ud[i, d] == 0.0
    assert np.array_equal(At, expect_At)
    recon = At.copy()
    for d, j in enumerate(D):
        recon[:, j] += Ud[:, d]
    assert np.array_equal(recon, Ad)
    assert S.At.nnz + S.U.nnz == A.nnz
    for j in D:
        assert At[j, j] != 0.0
        assert np.count_nonzero(At[:, j]) == min(kk, counts[j])


# -------------------------------------------------------------- pattern -----

def check_pattern_A2_bruteforce(pattern_fn, At):
    """J_k of P(|A~|^2) equals column k of the boolean product B B, B = (A~ != 0)."""
    B = (sp.csr_matrix(At).toarray() != 0).astype(np.int64)
    P = (B @ B) != 0
    C = sp.csc_matrix(At)
    C.sort_indices()
    for k in range(At.shape[0]):
        J = pattern_fn(C, k)
        assert list(J) == list(np.flatnonzero(P[:, k])), k


def check_rows_of_bruteforce(rows_fn, At, Js):
    """I_k = nonzero rows of A~(:, J_k), from the dense matrix."""
    Ad = sp.csr_matrix(At).toarray()
    C = sp.csc_matrix(At)
    C.sort_indices()
    for J in Js:
        I = rows_fn(C, J)
        expect = np.flatnonzero(np.any(Ad[:, np.asarray(J)] != 0, axis=1))
        assert list(I) == list(expect)


# ------------------------------------------------------------------ lsq -----

def check_ls_optimality(solve_fn, At, J, k, rtol=1e-9):
    """The LS solution satisfies the full-length normal equations and Pythagoras.

    With a = A~(:, J) (all n rows, from the sparse matrix) and r = a m - e_k:
    a^T r = 0 (to rounding) and ||r||^2 = 1 - (a m)_k, and res equals ||r||.
    """
    C = sp.csc_matrix(At)
    C.sort_indices()
    I, m, res = solve_fn(C, J, k)
    a = sp.csc_matrix(At)[:, np.asarray(J)].toarray()
    e = np.zeros(At.shape[0])
    e[k] = 1.0
    r = a @ m - e
    scale = np.linalg.norm(a, 2) * max(np.linalg.norm(r), 1e-300) + 1e-300
    assert np.linalg.norm(a.T @ r) <= rtol * max(scale, np.linalg.norm(a, 2)), k
    assert abs(np.dot(r, r) - (1.0 - (a @ m)[k])) <= rtol, k
    assert abs(res - np.linalg.norm(r)) <= rtol, k
    # the same minimiser from the SVD-based least-squares routine
    m2 = np.linalg.lstsq(a, e, rcond=None)[0]
    assert np.linalg.norm(m - m2) <= 1e-7 * max(1.0, np.linalg.norm(m2)), k


def check_full_pattern_inverse(solve_fn, At, tol=1e-10):
    """With J_k = {0..n-1} the column problems give exactly M = A~^{-1}."""
    n = At.shape[0]
    C = sp.csc_matrix(At)
    C.sort_indices()
    inv = np.linalg.inv(sp.csr_matrix(At).toarray())
    for k in range(n):
        I, m, res = solve_fn(C, np.arange(n), k)
        assert np.allclose(m, inv[:, k], atol=tol, rtol=0), k
        assert res < 1e-9


# ----------------------------------------------------------------- spai -----

def check_spai_gains(gain_fn, At, J, I, r):
    """rho_j^2 from (rhoj) equals the brute-force 1-D minimum of ||r + mu A~ e_j||."""
    C = sp.csc_matrix(At)
    C.sort_indices()
    R = sp.csr_matrix(At)
    R.sort_indices()
    cn2 = np.asarray(C.multiply(C).sum(axis=0)).ravel()
    cand, tau, g, rho2 = gain_fn(C, R, cn2, J, I, r)
    Ad = R.toarray()
    full_r = np.zeros(At.shape[0])
    full_r[np.asarray(I)] = r
    # candidate set J~ = N \ J with N = nonzero columns of A~(I, :)
    N = np.flatnonzero(np.any(Ad[np.asarray(I), :] != 0, axis=0))
    expect = sorted(set(N.tolist()) - set(np.asarray(J).tolist()))
    assert list(cand) == expect
    for t, j in enumerate(cand):
        col = Ad[:, j]
        mu = np.linalg.lstsq(col[:, None], -full_r, rcond=None)[0][0]
        best = np.linalg.norm(full_r + mu * col) ** 2
        assert abs(best - rho2[t]) <= 1e-10 * max(1.0, np.dot(r, r)), (j, best, rho2[t])


# ----------------------------------------------------------------- drop -----

def check_drop_bound(assemble_fn, At, patterns, values, res, delta):
    """PSAI(tol) bound: ||A~ m_drop - e_k|| <= res_k + ||A~||_1 sum_dropped|m| <= res_k + delta."""
    n = At.shape[0]
    M = assemble_fn(n, patterns, values, "tolk", delta=delta, At=At)
    A1 = np.max(np.asarray(abs(sp.csc_matrix(At)).sum(axis=0)).ravel())
    Md = sp.csc_matrix(M)
    for k in range(n):
        mk = np.zeros(n)
        mk[patterns[k]] = values[k]
        kept = Md[:, k].toarray().ravel()
        dropped = mk - kept
        e = np.zeros(n)
        e[k] = 1.0
        rd = np.linalg.norm(At @ kept - e)
        assert rd <= res[k] + A1 * np.abs(dropped).sum() + 1e-12
        assert rd <= res[k] + delta + 1e-12
        assert np.count_nonzero(kept) >= 1
        tol_k = delta / (len(patterns[k]) * A1)
        big = np.abs(mk) > tol_k
        assert np.all(kept[big] == mk[big])


# ------------------------------------------------------------------ smw -----

def check_smw_exact(recover_fn, A, At, U, D, b):
    """With exact y = A~^{-1} b and W = A~^{-1} U, recovery gives A^{-1} b."""
    Ad = sp.csr_matrix(A).toarray()
    Atd = sp.csr_matrix(At).toarray()
    y = np.linalg.solve(Atd, b)
    W = np.linalg.solve(Atd, U)
    x, z, c = recover_fn(y, W, D)
    xd = np.linalg.solve(Ad, b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def check_residual_identity(recover_fn, A, At, U, D, b, rng):
    """For arbitrary y, W: b - A x = r_y - R_W (I + V^T W)^{-1} V^T y and (rry)."""
    n = A.shape[0]
    s = len(D)
    y = rng.standard_normal(n)
    W = 0.1 * rng.standard_normal((n, s))
    x, z, c = recover_fn(y, W, D)
    r = b - A @ x
    ry = b - At @ y
    RW = U - At @ W
    rhs = ry - RW @ z
    assert np.linalg.norm(r - rhs) <= 1e-10 * (np.linalg.norm(r) + 1)
    assert np.linalg.norm(r) <= np.linalg.norm(ry) + c * np.linalg.norm(RW, "fro") + 1e-10


# --------------------------------------------------------------- krylov -----

def check_bicgstab_restart_is_fresh_start(bicgstab_fn, A, M, b, thr, at):
    """A restart (r_hat = r, p = v = 0, rho_old = alpha = omega = 1; Section 5
    BiCGStab with the breakdown reading) at the end of iteration `at` makes the
    rest of the solve a fresh BiCGStab on the residual system A e = b - A x_at
    started from e = 0.  So the restarted run must equal: `at` iterations,
    then a new solve of the residual system, added on.  Compared to 1e-12
    relative, with equal iteration counts; the state right after the restart
    is also checked (r_hat equal to r, p and v zero)."""
    trace = []
    xr, itr, str_ = bicgstab_fn(A, M, b, thr, force_restart_at=[at], trace=trace)
    xa, ita, sta = bicgstab_fn(A, M, b, 0.0, maxit=at)
    assert sta == "maxit" and ita == at
    e, ite, ste = bicgstab_fn(A, M, b - A @ xa, thr)
    xc = xa + e
    assert str_ == ste == "converged", (str_, ste)
    assert itr == at + ite, (itr, at, ite)
    assert np.linalg.norm(xr - xc) <= 1e-12 * np.linalg.norm(xc), np.linalg.norm(xr - xc)
    rs = [st for ev, it, st in trace if ev == "restart"]
    assert len(rs) == 1 and [it for ev, it, _ in trace if ev == "restart"] == [at]
    st = rs[0]
    assert np.array_equal(st["rhat"], st["r"]) and not st["p"].any() and not st["v"].any()


def check_bicgstab_second_breakdown(bicgstab_fn, A, M, b, thr, at, gap):
    """A second breakdown ends the solve with status "breakdown" at that
    iteration; the returned x is the iterate reached by then, i.e. x_at plus
    `gap` iterations of a fresh solve of the residual system."""
    xr, itr, str_ = bicgstab_fn(A, M, b, thr, force_restart_at=[at, at + gap])
    assert str_ == "breakdown" and itr == at + gap, (str_, itr)
    xa, _, _ = bicgstab_fn(A, M, b, 0.0, maxit=at)
    e, ite, ste = bicgstab_fn(A, M, b - A @ xa, 0.0, maxit=gap)
    assert ste == "maxit" and ite == gap
    assert np.linalg.norm(xr - (xa + e)) <= 1e-12 * np.linalg.norm(xa + e)


def check_bicgstab_replacement(bicgstab_fn, A, M, b, thr):
    """Convergence is declared on the true residual only; when the recursive
    residual passes and the true one does not, the true residual replaces the
    recursive one and the iteration continues.  On a system where that branch
    is reached: the recursive residual had passed (its norm < thr) while
    b - A x had not, r equals b - A x afterwards, and the solve still ends with
    a true residual below thr and x within kappa * thr / ||b|| of the dense
    solution."""
    trace = []
    x, it, st = bicgstab_fn(A, M, b, thr, trace=trace)
    reps = [(i, s) for ev, i, s in trace if ev == "replace"]
    assert reps, "the residual replacement branch was not reached"
    for i, s in reps:
        rt = b - A @ s["x"]
        assert np.linalg.norm(s["r_rec"]) < thr <= np.linalg.norm(rt), i
        assert np.array_equal(s["r"], rt), i
    assert st == "converged", st
    assert np.linalg.norm(b - A @ x) < thr
    Ad = A.toarray()
    xd = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(x - xd) <= 2.0 * kappa * thr / np.linalg.norm(b) * np.linalg.norm(xd)


def _krylov_minres(AM, r, m):
    """argmin ||r - AM z|| over z in K_m(AM, r), from an orthonormal basis of
    the explicit Krylov vectors r, AM r, ..., (AM)^(m-1) r (numpy QR) and a dense
    least-squares solve: a formulation independent of Arnoldi and Givens."""
    K = np.empty((r.size, m))
    v = r / np.linalg.norm(r)
    for j in range(m):
        K[:, j] = v
        v = AM @ v
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(AM @ Q, r, rcond=None)
    return Q @ y


def check_gmres_cycles_minimise(gmres_fn, A, M, b, m, cycles=2):
    """GMRES(m) (Section 5's setting, right preconditioning): each full cycle
    takes x_{c+1} = x_c + M z with z minimising ||r_c - A M z|| over the Krylov
    space K_m(A M, r_c) of the current true residual r_c = b - A x_c.  Run for
    exactly `cycles` full cycles (threshold 0, maxit = cycles m) and compare with
    those minimisers built without Arnoldi (to 1e-8 relative)."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    Md = M.toarray() if sp.issparse(M) else np.asarray(M)
    AM = Ad @ Md
    x, it, st = gmres_fn(A, M, b, 0.0, restart=m, maxit=cycles * m)
    assert st == "maxit" and it == cycles * m, (st, it)
    xe = np.zeros(b.size)
    for _ in range(cycles):
        r = b - Ad @ xe
        xe = xe + Md @ _krylov_minres(AM, r, m)
    assert np.linalg.norm(x - xe) <= 1e-8 * np.linalg.norm(xe), np.linalg.norm(x - xe) / np.linalg.norm(xe)


def check_forward_correction_exact(correction_fn, A, At, U, D, v):
    """With exact W = A~^{-1} U, solving A~^T lam = correction_fn(W, D, v) gives
    A^{-T} v (Theorem 3.1's A^{-1} transposed)."""
    Ad = sp.csr_matrix(A).toarray()
    Atd = sp.csr_matrix(At).toarray()
    W = np.linalg.solve(Atd, sp.csc_matrix(U).toarray())
    rhs, _ = correction_fn(W, np.asarray(D, dtype=np.int64), v)
    lam = np.linalg.solve(Atd.T, rhs)
    lam_d = np.linalg.solve(Ad.T, v)
    assert np.linalg.norm(lam - lam_d) <= 1e-10 * np.linalg.norm(lam_d)


def check_adjoint_reported_residual(adjoint_fn, A, S, M, W, g, eps):
    """The adjoint's reported rr is the true ||g - A^T lam|| / ||g|| (to 1e-3 of
    itself: the two ways of forming A^T lam round differently), below eps."""
    out = adjoint_fn(S, M, W, g, eps=eps)
    rr = np.linalg.norm(g - sp.csr_matrix(A).T @ out["lam"]) / np.linalg.norm(g)
    assert abs(rr - out["rr"]) <= 1e-3 * rr + 1e-15
    assert rr < eps
