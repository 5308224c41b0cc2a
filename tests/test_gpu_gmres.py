"""Batched GMRES(m) on the GPU (sai_krylov / sai_solve with SAI_GMRES) vs the oracle.

The batched form (one lockstep run over the k columns, the BiCGStab sparse
products, classical Gram-Schmidt with one reorthogonalisation) is forced with
the GMRES_BATCH_NK knob at 0 on matrices small enough for a dense SVD.  The
oracle runs GMRES(m) column by column with modified Gram-Schmidt on the same
right-hand sides with its own FP64 M (equal to the library's FP64 build to
1e-12).  Bars: every column's true residual, recomputed on the host in FP64,
below its threshold; iteration counts equal up to 2 (the two orthogonalisations
round differently, so a column that meets its threshold within rounding may
take one step more or less, and that can move a restart); x within
||A~^{-1}|| (sum of both true residuals) of the oracle's.  Stopped runs (maxit)
are compared value for value (same iterations, so the iterates agree to
rounding).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import krylov as okry
from oracle import pipeline as opipe
from oracle import split as osplit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1211_6866_amd as P  # noqa: E402

CASES = {
    "c1": (1, {}, "A"),
    "c2_12": (2, dict(dims=(12, 12, 12), s=4, density=0.2), "A2"),
    "c4_40": (4, dict(dims=(40, 37), s=3, density=0.15), "A2"),
    "c3_3000": (3, dict(n=3000, s=4, density=0.05), "A"),
}
_CACHE = {}


def _setup(name):
    """Workload, split, FP64 preconditioner (library and oracle), [b, U], sigma_min(A~)."""
    if name not in _CACHE:
        idx, kw, kind = CASES[name]
        w = W.make(idx, **kw)
        S = osplit.split(w.A)
        rp, ci, va = P.csr_to_device(w.A)
        g = P.Split(rp, ci, va)
        drop = "none" if kind == "A" else "abs"
        pc = P.Precond(g, pattern=P.PAT_A if kind == "A" else P.PAT_A2,
                       drop=P.DROP_NONE if kind == "A" else P.DROP_ABS, tau=1e-3, precision=P.FP64)
        Mo, _ = opipe.build_M(S, kind, drop, 1e-3)
        n, s = w.A.shape[0], S.s
        R = np.zeros((n, s + 1))
        R[:, 0] = w.b
        R[:, 1:] = S.U.toarray()
        At = sp.csr_matrix(S.At)
        smin = float(np.linalg.svd(S.At.toarray(), compute_uv=False)[-1])
        _CACHE[name] = (w, S, g, pc, sp.csr_matrix(Mo), R, At, smin)
    return _CACHE[name]


def _krylov(g, pc, R, thr, batch_n=0, **kw):
    try:
        P.tune_set("GMRES_BATCH_NK", batch_n)
        X, its, sts, code = P.krylov(g, pc, torch.from_numpy(np.ascontiguousarray(R)).cuda(), thr,
                                     method=P.GMRES, **kw)
    finally:
        P.tune_set("GMRES_BATCH_NK", 32768)
    return X.cpu().numpy(), its, sts, code


def _check_vs_oracle(At, R, thr, smin, Xh, its, Xo, itso, tag):
    for c in range(R.shape[1]):
        rg = np.linalg.norm(R[:, c] - At @ Xh[:, c])
        ro = np.linalg.norm(R[:, c] - At @ Xo[:, c])
        assert rg < thr[c], (tag, c, rg, thr[c])
        assert abs(its[c] - itso[c]) <= 2, (tag, c, its, itso)
        assert np.linalg.norm(Xh[:, c] - Xo[:, c]) <= (rg + ro) / smin, (tag, c)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("restart", [5, 20, 40])
def test_gmres_batched_vs_oracle(name, restart):
    """[b, U] of each case to eps 1e-10 (thresholds of the auxiliary systems with
    c = 1); restart 5 runs many cycles, 40 runs cycles longer than the 32-vector
    projection chunk (c1, c4_40)."""
    w, S, g, pc, Mo, R, At, smin = _setup(name)
    thr = okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)
    Xh, its, sts, code = _krylov(g, pc, R, thr, restart=restart)
    assert code == P.OK and all(v == 0 for v in sts), (its, sts)
    Xo, itso, stso = okry.solve_block(At, Mo, R, thr, method="gmres", restart=restart)
    assert all(v == "converged" for v in stso)
    _check_vs_oracle(At, R, thr, smin, Xh, its, Xo, itso, (name, restart))
    print(f"{name} GMRES({restart}): gpu iterations {its}, oracle {itso}")


def test_gmres_batched_matches_per_column_form():
    """The batched and the per-column (one workgroup per column) forms on the
    same systems: the same iteration counts up to 2, and x within the forward
    bound of each other."""
    w, S, g, pc, Mo, R, At, smin = _setup("c4_40")
    thr = okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)
    Xb, itb, stb, cb = _krylov(g, pc, R, thr, batch_n=0, restart=20)
    Xc, itc, stc, cc = _krylov(g, pc, R, thr, batch_n=1 << 30, restart=20)
    assert cb == cc == P.OK
    _check_vs_oracle(At, R, thr, smin, Xb, itb, Xc, itc, "batched vs per-column")


@pytest.mark.parametrize("k", [1, 13, 64])
def test_gmres_batched_column_counts(k):
    """k = 1 (one column pair with a pad column), 13 (odd, several lane
    classes) and 64 (the most columns): random right-hand sides (seeded),
    restart 20, against the oracle column by column."""
    w, S, g, pc, Mo, R, At, smin = _setup("c2_12")
    rng = np.random.default_rng(1000 + k)
    Rk = rng.standard_normal((At.shape[0], k))
    thr = [1e-10 * np.linalg.norm(Rk[:, c]) for c in range(k)]
    Xh, its, sts, code = _krylov(g, pc, Rk, thr, restart=20)
    assert code == P.OK and all(v == 0 for v in sts), (its, sts)
    Xo, itso, stso = okry.solve_block(At, Mo, Rk, thr, method="gmres", restart=20)
    _check_vs_oracle(At, Rk, thr, smin, Xh, its, Xo, itso, ("k", k))


def test_gmres_batched_maxit_stops_like_oracle():
    """maxit = 7 with restart 5: one full cycle and a partial one of two steps;
    every column stops with status 1 (SAI_ENOCONV overall) after 7 iterations,
    and its iterate equals the oracle's after the same 7 steps to rounding."""
    w, S, g, pc, Mo, R, At, smin = _setup("c1")
    thr = okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)
    Xh, its, sts, code = _krylov(g, pc, R, thr, restart=5, maxit=7)
    assert code == P.ENOCONV and all(v == 1 for v in sts) and all(v == 7 for v in its), (its, sts)
    Xo, itso, stso = okry.solve_block(At, Mo, R, thr, method="gmres", restart=5, maxit=7)
    assert all(v == "maxit" for v in stso) and all(v == 7 for v in itso)
    for c in range(R.shape[1]):
        assert np.linalg.norm(Xh[:, c] - Xo[:, c]) <= 1e-8 * np.linalg.norm(Xo[:, c]), c


def test_gmres_batched_degenerate_columns():
    """A zero right-hand side converges at once (x = 0, no iteration) next to
    ordinary columns; maxit = 0 stops every nonzero column at x = 0 with status 1."""
    w, S, g, pc, Mo, R, At, smin = _setup("c2_12")
    R2 = R.copy()
    R2[:, 2] = 0.0
    thr = okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)
    Xh, its, sts, code = _krylov(g, pc, R2, thr, restart=20)
    assert code == P.OK and sts[2] == 0 and its[2] == 0 and not Xh[:, 2].any()
    for c in (0, 1, 3, 4):
        assert np.linalg.norm(R2[:, c] - At @ Xh[:, c]) < thr[c]
    X0, its0, sts0, code0 = _krylov(g, pc, R2, thr, restart=20, maxit=0)
    assert code0 == P.ENOCONV and not X0.any()
    assert [v for c, v in enumerate(sts0) if c != 2] == [1, 1, 1, 1] and sts0[2] == 0
    assert all(v == 0 for v in its0)


def test_gmres_solve_default_batched():
    """sai_solve with GMRES(20) on a 27,000-row 3-D matrix (the batched form by
    default): the final residual, recomputed on the host, within the theorem's
    bound (eps/2)(1 + c) for c = 1 thresholds."""
    w = W.make(2, dims=(30, 30, 30), s=6, density=0.05)
    rp, ci, va = P.csr_to_device(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP32)
    b = torch.from_numpy(w.b).cuda()
    x, st = P.solve(g, pc, b, method=P.GMRES, restart=20, eps=1e-8)
    xs = x.cpu().numpy()
    rr = np.linalg.norm(w.b - w.A @ xs) / np.linalg.norm(w.b)
    assert st["status"] == P.OK and rr < 1e-8 * (1.0 + st["c"]) / 2.0 * (1.0 + 1e-6), (rr, st)
    print(f"GMRES(20) on 30^3: iterations {st['iters']}, rr {rr:.2e}")
