"""GPU path at the full workload sizes, in the configuration bench.py times.

The oracle cannot build M or run the Krylov solves at these sizes in seconds,
so the checks are: the split against the oracle's split (bit-exact, full);
J_k, I_k (bit-exact) and m_k (rel. 1e-4, FP32 build) on a seeded sample of
columns that includes the dense columns and the first/last columns; the
dropped pattern of the sampled columns; rr < 1e-8 recomputed on the host in
FP64; and, for the loss workloads, properties of the gradient that hold at any
size (A^T lambda = g to solve tolerance, sum_ij A_ij G_ij = -lambda^T b) plus,
for the 500x500 workload, central differences of the exact loss (rank-one
updates of a sparse LU of A) on 16 seeded entries.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import drop as odrop
from oracle import lsq as olsq
from oracle import pattern as opat
from oracle import psai as opsai
from oracle import spai as ospai
from oracle import split as osplit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1211_6866_amd as P  # noqa: E402

SETTINGS = {
    2: dict(pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3),
    3: dict(pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=0.4, spai_steps=3, spai_per_step=5),
    4: dict(pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3),
    5: dict(pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3),
}


def _np(t):
    return t.detach().cpu().numpy()


def _sample(n, dense, seed, count=48):
    rng = np.random.default_rng(seed)
    cols = set(rng.choice(n, size=count, replace=False).tolist())
    cols.update(int(j) for j in dense)
    cols.update([0, 1, n - 2, n - 1])
    return sorted(cols)


@pytest.mark.parametrize("idx,prec", [(2, P.FP32), (3, P.FP32), (4, P.FP32), (5, P.FP32), (2, P.FP64),
                                      (5, P.FP64)])
def test_fullsize_workload(idx, prec):
    """prec: the mixed build (FP32 M) of every workload, and the plain FP64 build
    of the two 3D workloads (the bench times both)."""
    print(f"\nworkload {idx} ({'FP32' if prec == P.FP32 else 'FP64'} M): generating", flush=True)
    w = W.make(idx)
    n = w.A.shape[0]
    S = osplit.split(w.A)
    rp, ci, va = P.csr_to_device(w.A)
    g = P.Split(rp, ci, va)
    # ---- split: bit-exact, whole matrix
    arr = g.arrays()
    assert (g.s, g.p) == (S.s, S.p)
    assert np.array_equal(_np(arr["dense_cols"]), S.D)
    assert np.array_equal(_np(arr["t_row_ptr"]), S.At.indptr)
    assert np.array_equal(_np(arr["t_col_idx"]), S.At.indices)
    assert np.array_equal(_np(arr["t_val"]), S.At.data)
    del arr
    print(f"workload {idx}: split ok (s={S.s}, p={S.p})", flush=True)
    # ---- build with the lists kept
    bkw = SETTINGS[idx]
    pc = P.Precond(g, precision=prec, keep_lists=True, **bkw)
    assert (pc.stats.s, pc.stats.p) == (S.s, S.p)
    pa = pc.arrays()
    jp, ji, ip, ii = (_np(pa[k]) for k in ("j_ptr", "j_idx", "i_ptr", "i_idx"))
    mf = _np(pa["m_full"]).astype(np.float64)
    cp_, ri_, cv_ = _np(pa["col_ptr"]), _np(pa["row_idx"]), _np(pa["cval"]).astype(np.float64)
    del pa
    C = opat.as_csc(S.At)
    R = sp.csr_matrix(S.At)
    R.sort_indices()
    cn2 = ospai.column_norms2(C) if idx == 3 else None
    flips = 0
    worst = 0.0
    tol = 1e-12 if prec == P.FP64 else 1e-4
    for k in _sample(n, S.D, w.seed):
        if idx == 3:
            J, I, m, res, _ = ospai.spai_column(C, R, cn2, k, 3, 5, 0.4, "A")
        else:
            J = opat.pattern_A2(C, k)
            I, m, res = olsq.solve_column(C, J, k)
        assert np.array_equal(ji[jp[k]:jp[k + 1]], J), k
        assert np.array_equal(ii[ip[k]:ip[k + 1]], I), k
        e = np.linalg.norm(mf[jp[k]:jp[k + 1]] - m) / np.linalg.norm(m)
        worst = max(worst, e)
        assert e <= tol, (k, e)
        # dropped column: the same kept rows, except (FP32) entries within the
        # build's tolerance of tau; in FP64 bit-exact
        if bkw["drop"] == P.DROP_ABS:
            keep = odrop.drop_column(m, bkw["tau"])
            rows_o = set(J[keep].tolist())
            rows_g = set(ri_[cp_[k]:cp_[k + 1]].tolist())
            if prec == P.FP64:
                assert rows_o == rows_g, k
                vals_g = cv_[cp_[k]:cp_[k + 1]]
                assert np.linalg.norm(vals_g - m[keep]) <= 1e-12 * np.linalg.norm(m[keep]), k
            for r_ in rows_o ^ rows_g:
                pos = int(np.searchsorted(J, r_))
                assert abs(abs(m[pos]) - bkw["tau"]) <= 1e-4 * np.linalg.norm(m), (k, r_)
                flips += 1
    assert flips <= pc.stats.drop_flips
    if idx == 2 and prec == P.FP32:
        # the standalone gather at full size, sampled columns bit-exact (float32 copies)
        off, blocks = P.gather(g, pc, precision=P.FP32)
        off = _np(off)
        for k in _sample(n, S.D, w.seed + 2):
            J, I = ji[jp[k]:jp[k + 1]], ii[ip[k]:ip[k + 1]]
            got = _np(blocks[off[k]:off[k + 1]]).reshape(len(J), len(I)).T
            assert np.array_equal(got, olsq.dense_block(C, I, J).astype(np.float32)), k
        del blocks
    print(f"workload {idx}: sampled columns ok (worst rel err {worst:.2e}, {flips} threshold flips; "
          f"{pc.stats.drop_flips} undecidable entries in M)", flush=True)
    # ---- solve: rr < 1e-8 recomputed in FP64 on the host
    b = torch.from_numpy(w.b).cuda()
    x, st = P.solve(g, pc, b, eps=1e-8)
    xs = _np(x)
    rr = np.linalg.norm(w.b - w.A @ xs) / np.linalg.norm(w.b)
    print(f"workload {idx}: rr = {rr:.3e}, iters = {st['iters']}", flush=True)
    assert rr < 1e-8 and abs(rr - st["rr"]) <= 1e-6 * rr
    if idx not in (4, 5):
        return
    # ---- adjoint: properties at any size.  A 1e-8 forward tolerance leaves about
    # kappa * 1e-8 relative error in x and hence in -lambda_i x_j, so the gradient
    # run solves forward and adjoint to 1e-10.
    x, st = P.solve(g, pc, b, eps=1e-10)
    xs = _np(x)
    xstar = W.x_star(n, w.seed)
    gx = x - torch.from_numpy(xstar).cuda()
    gb, ga, bst = P.backward(g, pc, x, gx, eps=1e-10)
    lam, G = _np(gb), _np(ga)
    gv = xs - xstar
    res_adj = np.linalg.norm(w.A.T @ lam - gv) / np.linalg.norm(gv)
    trace = float(np.dot(w.A.data, G))
    print(f"workload {idx}: ||A^T lam - g||/||g|| = {res_adj:.2e}", flush=True)
    assert res_adj < 1e-9
    assert abs(trace + lam @ w.b) <= 1e-8 * abs(lam @ w.b)
    rows = np.repeat(np.arange(n), np.diff(w.A.indptr))
    assert np.array_equal(G, -lam[rows] * xs[w.A.indices])
    # the same from the forward solve's W (sai_solve_y, sai_backward_y): one system
    # with A~^T per correction pass, its true residual checked below eps
    x2, Y2, st2 = P.solve_y(g, pc, b, eps=1e-10)
    xs2 = _np(x2)
    gv2 = xs2 - xstar
    gb2, ga2, bst2 = P.backward_y(g, pc, x2, Y2, torch.from_numpy(gv2).cuda(), eps=1e-10)
    lam2, G2 = _np(gb2), _np(ga2)
    res2 = np.linalg.norm(w.A.T @ lam2 - gv2) / np.linalg.norm(gv2)
    print(f"workload {idx}: from the forward's W ||A^T lam - g||/||g|| = {res2:.2e} "
          f"({bst2['iters'][0]} iterations against {sum(bst['iters'])})", flush=True)
    assert bst2["status"] == P.OK and res2 < 1e-10 * (1 + 1e-3)
    # the GPU's residual (A~^T lam + V U^T lam) and the host's round differently:
    # 1e-3 of themselves plus 64 unit roundoffs of || |A|^T |lam| || + ||g|| over ||g||
    gn2 = np.linalg.norm(gv2)
    rnd = 64 * np.finfo(np.float64).eps * (np.linalg.norm(abs(w.A).T @ np.abs(lam2)) + gn2) / gn2
    assert abs(res2 - bst2["rr"]) <= 1e-3 * res2 + rnd
    assert np.array_equal(G2, -lam2[rows] * xs2[w.A.indices])
    if idx != 4:
        return
    # ---- central differences of the exact loss (workload 4)
    import scipy.sparse.linalg as spla
    lu = spla.splu(sp.csc_matrix(w.A))
    x0 = lu.solve(w.b)
    h = 1e-6
    for q in W.fd_entries(w.A, w.dense_cols, w.seed, 16):
        i, j = int(rows[q]), int(w.A.indices[q])
        ei = np.zeros(n)
        ei[i] = 1.0
        z = lu.solve(ei)                      # A^{-1} e_i
        # (A + t e_i e_j^T)^{-1} b = x0 - t z x0_j / (1 + t z_j)
        dp = -h * z * x0[j] / (1.0 + h * z[j])
        dm = h * z * x0[j] / (1.0 - h * z[j])
        # L+ - L- = 0.5 (x+ - x-)^T (x+ + x- - 2 x*)
        dl = 0.5 * np.dot(dp - dm, 2.0 * (x0 - xstar) + dp + dm)
        fd = dl / (2.0 * h)
        assert abs(fd - G[q]) <= 1e-5 * max(abs(G[q]), 1e-6 * np.abs(G).max()), (q, fd, G[q])
        assert abs(fd - G2[q]) <= 1e-5 * max(abs(G2[q]), 1e-6 * np.abs(G2).max()), (q, fd, G2[q])
    print("workload 4: 16 finite differences ok (both adjoint forms)", flush=True)


@pytest.mark.parametrize("idx,delta,lmax", [(2, 0.2, 10), (4, 0.2, 10)])
def test_fullsize_psai_tol(idx, delta, lmax):
    """PSAI(tol) at the full sizes: sampled columns against the oracle's loop
    (final pattern bit-exact, values to FP32 rounding, residual of the last solve)."""
    print(f"\nworkload {idx}: PSAI(tol) delta={delta} lmax={lmax}", flush=True)
    w = W.make(idx)
    n = w.A.shape[0]
    S = osplit.split(w.A)
    rp, ci, va = P.csr_to_device(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_PSAI_TOL, delta=delta, psai_lmax=lmax, precision=P.FP32,
                   keep_lists=True)
    pa = pc.arrays()
    jp, ji = _np(pa["j_ptr"]), _np(pa["j_idx"])
    mf, res = _np(pa["m_full"]).astype(np.float64), _np(pa["res"])
    del pa
    C = opat.as_csc(S.At)
    a1 = odrop.norm1(C)
    for k in _sample(n, S.D, w.seed + 1):
        Sk, mk, rk, _ = opsai.psai_tol_column(C, k, delta, lmax, a1)
        assert np.array_equal(ji[jp[k]:jp[k + 1]], Sk), k
        e = np.linalg.norm(mf[jp[k]:jp[k + 1]] - mk) / np.linalg.norm(mk)
        assert e <= 1e-7, (k, e)
        assert abs(res[k] - rk) <= 1e-12, (k, res[k], rk)
    print(f"workload {idx}: PSAI(tol) sampled columns ok, mean nnz/col {jp[-1] / n:.2f}", flush=True)
    b = torch.from_numpy(w.b).cuda()
    x, st = P.solve(g, pc, b, eps=1e-8)
    rr = np.linalg.norm(w.b - w.A @ _np(x)) / np.linalg.norm(w.b)
    print(f"workload {idx}: PSAI(tol) rr = {rr:.3e}, iters = {st['iters']}", flush=True)
    assert rr < 1e-8 * (1.0 + st["c"]) / 2.0 * (1.0 + 1e-6), (rr, st["c"])  # the theorem with c = 1


@pytest.mark.parametrize("idx", [2, 5])
def test_fullsize_gmres20(idx):
    """GMRES(20) on the s+1 systems at full size (the batched form, run by
    `bench.py --method gmres --restart 20`): every column meets its (stopb) /
    (stopU2) threshold, so rr recomputed on the host in FP64 is within the
    theorem's (eps/2)(1 + c), as is BiCGStab's.  The two x differ by at most
    ||A^{-1}|| times the sum of their residuals; kappa(A) of these stencil
    matrices is of order 1e4, so they must agree to 1e-3 relative."""
    print(f"\nworkload {idx}: GMRES(20)", flush=True)
    w = W.make(idx)
    rp, ci, va = P.csr_to_device(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, precision=P.FP32, **SETTINGS[idx])
    b = torch.from_numpy(w.b).cuda()
    xg, sg = P.solve(g, pc, b, method=P.GMRES, restart=20, eps=1e-8)
    xb, sb = P.solve(g, pc, b, method=P.BICGSTAB, eps=1e-8)
    bn = np.linalg.norm(w.b)
    for x, st in ((xg, sg), (xb, sb)):
        rr = np.linalg.norm(w.b - w.A @ _np(x)) / bn
        assert st["status"] == P.OK and rr < 1e-8 * (1.0 + st["c"]) / 2.0 * (1.0 + 1e-6), (rr, st["c"])
    e = np.linalg.norm(_np(xg) - _np(xb)) / np.linalg.norm(_np(xb))
    print(f"workload {idx}: GMRES(20) iterations max {max(sg['iters'])}, BiCGStab {max(sb['iters'])}, "
          f"|x_g - x_b| / |x_b| = {e:.2e}", flush=True)
    assert e <= 1e-3
