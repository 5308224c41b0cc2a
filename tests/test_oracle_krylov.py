"""Oracle Krylov solves and the Section 4 stopping rules."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import krylov, smw, split as osplit


def _small(seed=0, n=120):
    return W.random_sparse(n, 0.04, seed, diag=3.0)


def test_exact_preconditioner_one_iteration():
    A = _small()
    Minv = sp.csr_matrix(np.linalg.inv(A.toarray()))
    b = A @ np.ones(A.shape[0])
    x, it, st = krylov.bicgstab(A, Minv, b, 1e-10 * np.linalg.norm(b))
    assert st == "converged" and it == 1
    assert np.allclose(x, 1.0, atol=1e-10)
    x, it, st = krylov.gmres(A, Minv, b, 1e-10 * np.linalg.norm(b))
    assert st == "converged" and it == 1


def test_unpreconditioned_gmres_exact_in_n_steps():
    A = _small(1, n=40)
    I = sp.identity(40, format="csr")
    b = np.random.default_rng(1).standard_normal(40)
    x, it, st = krylov.gmres(A, I, b, 1e-11 * np.linalg.norm(b), restart=40, maxit=40)
    assert st == "converged" and it <= 40
    assert np.allclose(x, np.linalg.solve(A.toarray(), b), atol=1e-9)


@pytest.mark.parametrize("m,cycles", [(5, 1), (5, 3), (12, 2)])
def test_gmres_cycles_minimise_residual(m, cycles):
    """GMRES(m) against the minimal residual over each cycle's Krylov space,
    with a sparse approximate inverse as M (its entries from a dense inverse)."""
    import pins
    A = _small(4, n=80)
    Ad = A.toarray()
    Minv = np.linalg.inv(Ad)
    Minv[np.abs(Minv) < 0.05 * np.abs(Minv).max()] = 0.0
    b = np.random.default_rng(4).standard_normal(80)
    pins.check_gmres_cycles_minimise(krylov.gmres, A, sp.csr_matrix(Minv), b, m, cycles)


def test_bicgstab_true_residual_and_dense_solution():
    A = _small(2, n=200)
    I = sp.identity(200, format="csr")
    b = np.random.default_rng(2).standard_normal(200)
    thr = 1e-9 * np.linalg.norm(b)
    x, it, st = krylov.bicgstab(A, I, b, thr)
    assert st == "converged"
    assert np.linalg.norm(b - A @ x) < thr
    xd = np.linalg.solve(A.toarray(), b)
    kappa = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - xd) <= kappa * 1e-9 * np.linalg.norm(xd)


def test_zero_rhs_and_maxit():
    A = _small(3)
    I = sp.identity(A.shape[0], format="csr")
    x, it, st = krylov.bicgstab(A, I, np.zeros(A.shape[0]), 1e-12)
    assert st == "converged" and it == 0 and not x.any()
    b = np.ones(A.shape[0])
    x, it, st = krylov.bicgstab(A, I, b, 1e-300, maxit=3)
    assert st == "maxit" and it == 3


def test_stopping_rules_imply_target():
    """Section 4 theorem: (stopb) and (stopU2) with the true c imply rr < eps."""
    rng = np.random.default_rng(4)
    w = W.make(1)
    S = osplit.split(w.A)
    A, At, b = w.A, S.At, w.b
    U = S.U.toarray()
    Atd = At.toarray()
    y = np.linalg.solve(Atd, b)
    Wx = np.linalg.solve(Atd, U)
    eps = 1e-6
    s = S.s
    _, z, c = smw.recover(y, Wx, S.D)
    thr = krylov.thresholds(np.linalg.norm(b), s, eps, c=c)
    # perturb the exact solutions so that each residual sits just under its threshold
    yh = y + np.linalg.solve(Atd, rng.standard_normal(b.size))
    ry = b - At @ yh
    yh = y + (yh - y) * (0.99 * thr[0] / np.linalg.norm(ry))
    Wh = Wx.copy()
    for j in range(s):
        d = np.linalg.solve(Atd, rng.standard_normal(b.size))
        rj = At @ d
        Wh[:, j] = Wx[:, j] + d * (0.99 * thr[j + 1] / np.linalg.norm(rj))
    assert np.linalg.norm(b - At @ yh) < thr[0]
    xh, z2, c2 = smw.recover(yh, Wh, S.D)
    # c of the perturbed solutions is close to the exact one; the bound uses c2
    thr2 = krylov.thresholds(np.linalg.norm(b), s, eps, c=max(c, c2) * 1.0001)
    assert all(np.linalg.norm(U[:, j] - At @ Wh[:, j]) < thr2[j + 1] * 1.0001 for j in range(s))
    assert smw.relres(A, xh, b) < eps
    assert math.isclose(thr[0], 0.5 * eps * np.linalg.norm(b))


def _sai_A(A):
    """The oracle's own M on the pattern of A (a real preconditioner for the restart pins)."""
    from oracle import lsq, pattern as opat
    C = opat.as_csc(A)
    n = A.shape[0]
    cols, rows, vals = [], [], []
    for k in range(n):
        J = opat.pattern_A(C, k)
        _, m, _ = lsq.solve_column(C, J, k)
        rows += list(J)
        cols += [k] * len(J)
        vals += list(m)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


@pytest.mark.parametrize("seed,at,prec", [(0, 2, False), (1, 4, False), (2, 7, False), (3, 3, True)])
def test_bicgstab_restart_is_fresh_start(seed, at, prec):
    from tests import pins
    A = W.random_sparse(150, 0.04, seed, diag=2.0 if not prec else 1.0)
    M = _sai_A(A) if prec else sp.identity(A.shape[0], format="csr")
    b = A @ np.ones(A.shape[0])
    pins.check_bicgstab_restart_is_fresh_start(krylov.bicgstab, A, M, b, 1e-11 * np.linalg.norm(b), at)


def test_bicgstab_second_breakdown():
    from tests import pins
    A = W.random_sparse(150, 0.04, 5, diag=2.0)
    b = A @ np.ones(A.shape[0])
    pins.check_bicgstab_second_breakdown(krylov.bicgstab, A, sp.identity(150, format="csr"), b,
                                         1e-11 * np.linalg.norm(b), 3, 4)


@pytest.mark.parametrize("seed,n,diag", [(13, 60, 0.5), (12, 120, 1.0)])
def test_bicgstab_residual_replacement(seed, n, diag):
    """Systems (found by a seed search) whose recursive residual passes 1e-14 ||b||
    before the true residual does."""
    from tests import pins
    A = W.random_sparse(n, 0.08, seed, diag=diag)
    b = A @ np.ones(n)
    pins.check_bicgstab_replacement(krylov.bicgstab, A, sp.identity(n, format="csr"), b,
                                    1e-14 * np.linalg.norm(b))


def check_equilibration(run_fn, A, b):
    """Section 4's scaling of b: with equilibrate the solve of A x = lambda b is the
    solve of the same scaled right-hand side rho b / ||b|| for every lambda, so x
    scales exactly with lambda (to 1e-12) with the same iteration counts, meets
    rr < eps, and matches the dense solution within ||A^{-1}|| ||r||."""
    base = run_fn(A, b, equilibrate=True)
    Ad = A.toarray()
    smin = np.linalg.svd(Ad, compute_uv=False)[-1]
    xd = np.linalg.solve(Ad, b)
    assert base["rr"] < 1e-8
    assert np.linalg.norm(base["x"] - xd) <= np.linalg.norm(b - A @ base["x"]) / smin * (1 + 1e-6)
    for lam in (1e-10, 1e10):
        out = run_fn(A, lam * b, equilibrate=True)
        assert out["iters"] == base["iters"], (lam, out["iters"], base["iters"])
        assert np.linalg.norm(out["x"] - lam * base["x"]) <= 1e-12 * np.linalg.norm(lam * base["x"]), lam
        assert out["rr"] < 1e-8


def test_equilibration_scale_invariance():
    from oracle import pipeline as opipe
    w = W.make(2, dims=(12, 12, 12), s=4, density=0.2)
    check_equilibration(lambda A, b, **kw: opipe.run(A, b, kind="A2", drop="abs", tau=1e-3, maxit=300, **kw),
                        w.A, w.b)


def test_equilibration_rescues_large_b():
    """Without the scaling, b = 1e10 A 1 makes the auxiliary thresholds
    eps ||b|| / (2 sqrt(s)) far too loose for c = 1 and rr misses eps by far; with
    it the solve meets rr < eps."""
    from oracle import pipeline as opipe
    w = W.make(2, dims=(12, 12, 12), s=4, density=0.2)
    raw = opipe.run(w.A, 1e10 * w.b, kind="A2", drop="abs", tau=1e-3)
    eq = opipe.run(w.A, 1e10 * w.b, kind="A2", drop="abs", tau=1e-3, equilibrate=True)
    assert raw["rr"] > 1e-3 and eq["rr"] < 1e-8
