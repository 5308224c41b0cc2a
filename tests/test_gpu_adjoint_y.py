"""The adjoint from the forward solve's W (sai_solve_y + sai_backward_y) on the GPU.

A^{-T} = A~^{-T} (I - V K^{-T} W^T) with K = I + V^T W (Theorem 3.1's inverse,
transposed) needs one system with A~^T per correction pass.  Bars: the reported
adjoint residual is the true ||g - A^T lambda|| / ||g|| (recomputed on the host
in FP64, to 1e-3 of itself) and below eps; lambda within the forward-error bound
of the dense A^{-T} g and of the oracle's lambda (the sum of both residuals over
sigma_min(A)); gradients rel. 1e-5 at eps = 1e-12 as for sai_backward.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import adjoint as oadj
from oracle import pipeline as opipe

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


def _np(t):
    return t.detach().cpu().numpy()


def _setup(name, precision=None):
    idx, kw, kind = CASES[name]
    w = W.make(idx, **kw)
    rp, ci, va = P.csr_to_device(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A if kind == "A" else P.PAT_A2,
                   drop=P.DROP_NONE if kind == "A" else P.DROP_ABS, tau=1e-3,
                   precision=precision if precision is not None else P.FP32)
    return w, g, pc, kind


def _true_rr(A, lam, gv):
    return np.linalg.norm(gv - sp.csr_matrix(A).T @ lam) / np.linalg.norm(gv)


def _rr_agrees(A, lam, gv, rr_host, rr_gpu):
    """The GPU's residual (A~^T lam + V U^T lam, its own summation order) and the
    host's (A^T lam) agree to 1e-3 of themselves plus the rounding of forming them:
    64 unit roundoffs of || |A|^T |lam| || + ||g||, over ||g||."""
    gn = np.linalg.norm(gv)
    rnd = 64 * np.finfo(np.float64).eps * (np.linalg.norm(abs(sp.csr_matrix(A)).T @ np.abs(lam)) + gn) / gn
    return abs(rr_host - rr_gpu) <= 1e-3 * rr_host + rnd


@pytest.mark.parametrize("name", ["c1", "c2_12", "c4_40"])
def test_backward_y_vs_dense(name):
    """eps = 1e-12 forward and adjoint: lambda and the gradients against the dense
    solve to 1e-5 (the bar of sai_backward's test), the reported residual true."""
    w, g, pc, _ = _setup(name)
    b = torch.from_numpy(w.b).cuda()
    x, Y, st = P.solve_y(g, pc, b, eps=1e-12)
    assert tuple(Y.shape) == (w.A.shape[0], g.s + 1)
    xs = W.x_star(w.A.shape[0], w.seed)
    gx = x - torch.from_numpy(xs).cuda()
    gb, ga, bst = P.backward_y(g, pc, x, Y, gx, eps=1e-12)
    assert bst["status"] == P.OK and bst["iters"][1:] == [0] * g.s
    Ad = w.A.toarray()
    xd = np.linalg.solve(Ad, w.b)
    lam = np.linalg.solve(Ad.T, xd - xs)
    Gd = oadj.grad_A_values(w.A, lam, xd)
    assert np.linalg.norm(_np(gb) - lam) <= 1e-5 * np.linalg.norm(lam)
    assert np.linalg.norm(_np(ga) - Gd) <= 1e-5 * np.linalg.norm(Gd)
    rr = _true_rr(w.A, _np(gb), _np(gx))
    assert bst["rr"] < 1e-12 and _rr_agrees(w.A, _np(gb), _np(gx), rr, bst["rr"]), (rr, bst["rr"])
    print(f"{name}: adjoint iterations {bst['iters'][0]}, rr {rr:.2e}")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("method", ["bicgstab", "gmres"])
def test_backward_y_vs_oracle_at_1e8(name, method):
    """The benchmark's setting (forward and adjoint to eps = 1e-8, FP32 M): the
    correction passes bring the true adjoint residual below 1e-8; lambda against
    the oracle's adjoint_from_forward (its own forward W, FP64 M) within the sum
    of both residuals over sigma_min(A)."""
    w, g, pc, kind = _setup(name)
    mk = dict(method=P.GMRES, restart=20) if method == "gmres" else {}
    b = torch.from_numpy(w.b).cuda()
    x, Y, st = P.solve_y(g, pc, b, eps=1e-8, **mk)
    gv = _np(x) - W.x_star(w.A.shape[0], w.seed)
    gx = torch.from_numpy(gv).cuda()
    gb, ga, bst = P.backward_y(g, pc, x, Y, gx, eps=1e-8, **mk)
    lam = _np(gb)
    rr = _true_rr(w.A, lam, gv)
    assert bst["status"] == P.OK and rr < 1e-8 and _rr_agrees(w.A, lam, gv, rr, bst["rr"]), (rr, bst)
    out = opipe.run(w.A, w.b, kind=kind, drop="none" if kind == "A" else "abs", eps=1e-8, method=method,
                    restart=20)
    ro = oadj.adjoint_from_forward(out["split"], out["M"], out["Y"][:, 1:], gv, eps=1e-8, method=method,
                                   restart=20)
    assert ro["status"] == "converged"
    smin = float(np.linalg.svd(w.A.toarray(), compute_uv=False)[-1])
    bound = (rr + _true_rr(w.A, ro["lam"], gv)) * np.linalg.norm(gv) / smin
    assert np.linalg.norm(lam - ro["lam"]) <= bound
    print(f"{name} {method}: adjoint iterations {bst['iters'][0]} (oracle {ro['iters']}), rr {rr:.2e}")


def test_backward_y_matches_transposed_split_form():
    """sai_backward_y and sai_backward (s + 1 transposed systems) on the same
    forward solution: lambda within the forward-error bound of each other."""
    w, g, pc, _ = _setup("c4_40")
    b = torch.from_numpy(w.b).cuda()
    x, Y, st = P.solve_y(g, pc, b, eps=1e-10)
    gv = _np(x) - W.x_star(w.A.shape[0], w.seed)
    gx = torch.from_numpy(gv).cuda()
    gy, _, sty = P.backward_y(g, pc, x, Y, gx, eps=1e-10, want_a=False)
    gs, _, sts = P.backward(g, pc, x, gx, eps=1e-10, want_a=False)
    ry, rs = _true_rr(w.A, _np(gy), gv), _true_rr(w.A, _np(gs), gv)
    smin = float(np.linalg.svd(w.A.toarray(), compute_uv=False)[-1])
    assert np.linalg.norm(_np(gy) - _np(gs)) <= (ry + rs) * np.linalg.norm(gv) / smin
    assert ry < 1e-10
    print(f"one transposed system: {sty['iters'][0]} iterations; s + 1 systems: {sum(sts['iters'])}")


def test_solve_y_same_x_as_solve():
    """Keeping Y changes nothing in the forward solve: x and the statistics equal
    sai_solve's bit for bit, and Y's columns solve A~ [y, W] = [b, U]."""
    w, g, pc, _ = _setup("c2_12")
    b = torch.from_numpy(w.b).cuda()
    x1, st1 = P.solve(g, pc, b, eps=1e-8)
    x2, Y, st2 = P.solve_y(g, pc, b, eps=1e-8)
    assert torch.equal(x1, x2) and st1["iters"] == st2["iters"] and st1["rr"] == st2["rr"]
    from oracle import split as osplit
    S = osplit.split(w.A)
    Yh = _np(Y)
    At = sp.csr_matrix(S.At)
    # the thresholds (stopb), (stopU2) with c = 1, with room for the host's rounding
    assert np.linalg.norm(w.b - At @ Yh[:, 0]) < 0.5e-8 * np.linalg.norm(w.b) * (1 + 1e-6)
    U = S.U.toarray()
    for d in range(S.s):
        assert (np.linalg.norm(U[:, d] - At @ Yh[:, 1 + d])
                < 1e-8 * np.linalg.norm(w.b) / (2 * np.sqrt(S.s)) * (1 + 1e-6))


def test_backward_y_without_dense_columns_and_zero_gradient():
    """s = 0 (no irregular column: Y may be NULL, plain A^T lambda = g with the
    residual passes) and g = 0 (lambda = 0, no iteration)."""
    r, c, v, nn = W.stencil((30, 30), 7)
    A = sp.csr_matrix(sp.coo_matrix((v, (r, c)), shape=(nn, nn)))
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    rp, ci, va = P.csr_to_device(A)
    g = P.Split(rp, ci, va)
    assert g.s == 0
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, precision=P.FP32)
    rng = np.random.default_rng(6)
    gv = rng.standard_normal(A.shape[0])
    x = torch.from_numpy(rng.standard_normal(A.shape[0])).cuda()
    gb, ga, st = P.backward_y(g, pc, x, None, torch.from_numpy(gv).cuda(), eps=1e-8)
    rr = _true_rr(A, _np(gb), gv)
    assert st["status"] == P.OK and rr < 1e-8
    w, g2, pc2, _ = _setup("c2_12")
    x2, Y2, _ = P.solve_y(g2, pc2, torch.from_numpy(w.b).cuda(), eps=1e-8)
    z = torch.zeros(w.A.shape[0], dtype=torch.float64, device="cuda")
    gb2, ga2, st2 = P.backward_y(g2, pc2, x2, Y2, z, eps=1e-8)
    assert st2["status"] == P.OK and st2["iters"][0] == 0 and not _np(gb2).any() and not _np(ga2).any()


def test_backward_y_many_dense_columns():
    """s = 100 (W^T r reduced over 100 columns, K^T of order 100) against the dense
    solve."""
    w = W.make(4, dims=(60, 60), s=100, density=0.15)
    rp, ci, va = P.csr_to_device(w.A)
    g = P.Split(rp, ci, va)
    assert g.s == 100
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP64)
    b = torch.from_numpy(w.b).cuda()
    x, Y, st = P.solve_y(g, pc, b, eps=1e-12)
    xs = _np(x)
    xst = W.x_star(w.A.shape[0], w.seed)
    gx = x - torch.from_numpy(xst).cuda()
    gb, ga, bst = P.backward_y(g, pc, x, Y, gx, eps=1e-12)
    lam = np.linalg.solve(w.A.toarray().T, xs - xst)
    assert bst["status"] == P.OK
    assert np.linalg.norm(_np(gb) - lam) <= 1e-5 * np.linalg.norm(lam)
    Gd = oadj.grad_A_values(w.A, lam, xs)
    assert np.linalg.norm(_np(ga) - Gd) <= 1e-5 * np.linalg.norm(Gd)


def test_backward_y_rejects_missing_y_and_non_finite_gradient():
    w, g, pc, _ = _setup("c2_12")
    x = torch.zeros(w.A.shape[0], dtype=torch.float64, device="cuda")
    with pytest.raises(P.SaiError) as e:
        P.backward_y(g, pc, x, None, x.clone())
    assert e.value.code == P.EINVAL
    x2, Y, _ = P.solve_y(g, pc, torch.from_numpy(w.b).cuda(), eps=1e-8)
    gx = torch.ones_like(x2)
    gx[5] = float("nan")
    with pytest.raises(P.SaiError) as e:
        P.backward_y(g, pc, x2, Y, gx)
    assert e.value.code == P.EINVAL


def test_backward_y_iteration_limit():
    """maxit = 3: the passes stop without reaching eps; SAI_ENOCONV with the
    gradients still written (finite) and the reported residual the true one."""
    w, g, pc, _ = _setup("c4_40")
    b = torch.from_numpy(w.b).cuda()
    x, Y, _ = P.solve_y(g, pc, b, eps=1e-8)
    gv = _np(x) - W.x_star(w.A.shape[0], w.seed)
    gb, ga, st = P.backward_y(g, pc, x, Y, torch.from_numpy(gv).cuda(), eps=1e-8, maxit=3,
                              raise_on_error=False)
    assert st["code"] == P.ENOCONV and st["status"] == P.ENOCONV
    lam = _np(gb)
    assert np.isfinite(lam).all() and np.isfinite(_np(ga)).all()
    rr = _true_rr(w.A, lam, gv)
    assert rr >= 1e-8 and _rr_agrees(w.A, lam, gv, rr, st["rr"])
    assert 0 < st["iters"][0] <= 4 * 3
