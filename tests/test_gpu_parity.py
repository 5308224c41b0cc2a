"""GPU path vs the FP64 oracle, through the C ABI (Python binding = marshalling only).

Bars: integer/index outputs bit-exact; M per column rel. 1e-12 (FP64 build) or
1e-4 (FP32 build); x to the residual tolerance 1e-8 (rr recomputed on the host
in FP64) and the forward error it implies; gradients rel. 1e-5 (normwise).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import adjoint as oadj
from oracle import drop as odrop
from oracle import krylov as okry
from oracle import lsq as olsq
from oracle import pattern as opat
from oracle import pipeline as opipe
from oracle import smw as osmw
from oracle import split as osplit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1211_6866_amd as P  # noqa: E402

CASES = {
    "c1": (1, {}),
    "c2_12": (2, dict(dims=(12, 12, 12), s=4, density=0.2)),
    "c2_13x9x7": (2, dict(dims=(13, 9, 7), s=3, density=0.3)),
    "c4_40": (4, dict(dims=(40, 37), s=3, density=0.15)),
    "c3_3000": (3, dict(n=3000, s=4, density=0.05)),
}


def _np(t):
    return t.detach().cpu().numpy()


def _load(name):
    idx, kw = CASES[name]
    w = W.make(idx, **kw)
    return w, P.csr_to_device(w.A)


@pytest.mark.parametrize("name", list(CASES))
def test_split_bit_exact(name):
    w, (rp, ci, va) = _load(name)
    S = osplit.split(w.A)
    g = P.Split(rp, ci, va)
    assert (g.s, g.p) == (S.s, S.p)
    arr = g.arrays()
    assert np.array_equal(_np(arr["dense_cols"]), S.D)
    At = S.At
    assert np.array_equal(_np(arr["t_row_ptr"]), At.indptr)
    assert np.array_equal(_np(arr["t_col_idx"]), At.indices)
    assert np.array_equal(_np(arr["t_val"]), At.data)           # copies: bit-exact
    Ct = sp.csc_matrix(At)
    Ct.sort_indices()
    assert np.array_equal(_np(arr["t_col_ptr"]), Ct.indptr)
    assert np.array_equal(_np(arr["t_row_idx"]), Ct.indices)
    assert np.array_equal(_np(arr["t_cval"]), Ct.data)
    Ur = sp.csr_matrix(S.U)
    Ur.sort_indices()
    assert np.array_equal(_np(arr["u_row_ptr"]), Ur.indptr)
    assert np.array_equal(_np(arr["u_col"]), Ur.indices)
    assert np.array_equal(_np(arr["u_val"]), Ur.data)


def test_split_keep_and_largest_rule():
    w, (rp, ci, va) = _load("c2_12")
    # keep - 1 <= 16 candidates per thread in registers; 18 and 30 take the
    # multi-pass selection
    for keep, rule, orule in [(1, P.KEEP_NEAREST, "nearest"), (4, P.KEEP_LARGEST, "largest"),
                              (17, P.KEEP_LARGEST, "largest"), (17, P.KEEP_NEAREST, "nearest"),
                              (18, P.KEEP_NEAREST, "nearest"), (30, P.KEEP_LARGEST, "largest")]:
        S = osplit.split(w.A, keep=keep, rule=orule)
        g = P.Split(rp, ci, va, keep=keep, rule=rule)
        arr = g.arrays()
        assert np.array_equal(_np(arr["t_col_idx"]), S.At.indices)
        assert np.array_equal(_np(arr["t_val"]), S.At.data)


@pytest.mark.parametrize("name,kind", [("c1", P.PAT_A), ("c1", P.PAT_A2), ("c2_12", P.PAT_A2),
                                       ("c2_13x9x7", P.PAT_A2), ("c4_40", P.PAT_A2),
                                       ("c3_3000", P.PAT_A)])
@pytest.mark.parametrize("prec", [P.FP64, P.FP32])
def test_patterns_and_columns(name, kind, prec):
    w, dev = _load(name)
    _check_patterns(w.A, dev, kind, prec)


@pytest.mark.parametrize("prec", [P.FP64, P.FP32])
def test_patterns_long_candidate_lists(prec):
    """Band of half-width 8: P(|A~|^2 e_k) has 33 entries and 33 * 17 = 561
    candidates for I_k at interior columns, more than the small pattern kernel
    holds, so those columns go through the large kernel's redo list."""
    A = W.banded(600, 8, 2, 0.5, 7)
    _check_patterns(A, P.csr_to_device(A), P.PAT_A2, prec)


def _check_patterns(A, dev, kind, prec):
    rp, ci, va = dev
    S = osplit.split(A)
    C = opat.as_csc(S.At)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=kind, drop=P.DROP_NONE, precision=prec, keep_lists=True)
    arr = pc.arrays()
    jp, ji, ip, ii = (_np(arr[k]) for k in ("j_ptr", "j_idx", "i_ptr", "i_idx"))
    mf, res = _np(arr["m_full"]).astype(np.float64), _np(arr["res"])
    n = A.shape[0]
    f = opat.pattern_A if kind == P.PAT_A else opat.pattern_A2
    tol = 1e-12 if prec == P.FP64 else 1e-4
    worst = 0.0
    for k in range(n):
        J = f(C, k)
        assert np.array_equal(ji[jp[k]:jp[k + 1]], J), k
        I, m, r = olsq.solve_column(C, J, k)
        assert np.array_equal(ii[ip[k]:ip[k + 1]], I), k
        e = np.linalg.norm(mf[jp[k]:jp[k + 1]] - m) / np.linalg.norm(m)
        worst = max(worst, e)
        assert e <= tol, (k, e)
        assert abs(res[k] - r) <= (1e-12 if prec == P.FP64 else 1e-5), (k, res[k], r)
    print(f"worst column rel err {worst:.2e}")


# c1: every column stops after the first loop; c2_12: one or two loops; c4_40:
# up to eight; c3_3000: l_max = 0; c2_13x9x7: no column reaches delta, all run
# out of loops.  (All within |S| <= 128 before the drop.)
@pytest.mark.parametrize("name,delta,lmax", [("c1", 0.4, 10), ("c2_12", 0.2, 10), ("c4_40", 0.15, 10),
                                              ("c3_3000", 0.4, 0), ("c2_13x9x7", 1e-3, 1)])
@pytest.mark.parametrize("prec", [P.FP64, P.FP32])
def test_psai_tol_vs_oracle(name, delta, lmax, prec):
    """PSAI(tol): final patterns bit-exact, values to the build precision,
    residuals of the last solve, against the oracle's loop."""
    from oracle import psai as opsai
    w, (rp, ci, va) = _load(name)
    S = osplit.split(w.A)
    n = w.A.shape[0]
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_PSAI_TOL, delta=delta, psai_lmax=lmax, precision=prec,
                   keep_lists=True)
    arr = pc.arrays()
    jp, ji = _np(arr["j_ptr"]), _np(arr["j_idx"])
    mf, res = _np(arr["m_full"]).astype(np.float64), _np(arr["res"])
    Ss, ms, rs, ls = opsai.psai_tol(S.At, delta=delta, lmax=lmax)
    assert pc.stats.l_m == int(np.max(ls)), (pc.stats.l_m, int(np.max(ls)))
    tol = 1e-12 if prec == P.FP64 else 1e-7
    worst = 0.0
    for k in range(n):
        assert np.array_equal(ji[jp[k]:jp[k + 1]], Ss[k]), (k, ji[jp[k]:jp[k + 1]], Ss[k])
        e = np.linalg.norm(mf[jp[k]:jp[k + 1]] - ms[k]) / np.linalg.norm(ms[k])
        worst = max(worst, e)
        assert e <= tol, (k, e)
        assert abs(res[k] - rs[k]) <= 1e-12, (k, res[k], rs[k])
    # M itself (CSC) holds exactly those columns
    cp, ri = _np(arr["col_ptr"]), _np(arr["row_idx"])
    assert np.array_equal(cp.astype(np.int64), jp) and np.array_equal(ri, ji)
    print(f"{name}: loops {np.bincount(ls)}, worst column rel err {worst:.2e}")


@pytest.mark.parametrize("prec", [P.FP64, P.FP32])
def test_psai_tol_large_patterns(prec):
    """PSAI(tol) with a small delta on a 20 x 20 grid: most columns run all 11
    loops and their power patterns reach 200-400 indices, past the fast
    search's 128, so they are searched again with the large limits; against the
    oracle's loop for every column."""
    from oracle import psai as opsai
    w = W.make(4, dims=(20, 20), s=2, density=0.15)
    S = osplit.split(w.A)
    n = w.A.shape[0]
    g = P.Split(*P.csr_to_device(w.A))
    pc = P.Precond(g, pattern=P.PAT_PSAI_TOL, delta=0.01, psai_lmax=10, precision=prec, keep_lists=True)
    arr = pc.arrays()
    jp, ji = _np(arr["j_ptr"]), _np(arr["j_idx"])
    mf, res = _np(arr["m_full"]).astype(np.float64), _np(arr["res"])
    Ss, ms, rs, ls = opsai.psai_tol(S.At, delta=0.01, lmax=10)
    assert max(len(x) for x in Ss) > 128
    assert pc.stats.l_m == int(np.max(ls))
    tol = 1e-12 if prec == P.FP64 else 1e-7
    for k in range(n):
        assert np.array_equal(ji[jp[k]:jp[k + 1]], Ss[k]), k
        assert np.linalg.norm(mf[jp[k]:jp[k + 1]] - ms[k]) <= tol * np.linalg.norm(ms[k]), k
        assert abs(res[k] - rs[k]) <= 1e-12, (k, res[k], rs[k])


def test_psai_tol_irregular_limits():
    """On the irregular matrix the power patterns grow about eightfold per loop:
    l_max = 1 (patterns up to a few hundred indices, through the large limits)
    matches the oracle on every column; l_max = 3 needs patterns beyond 512
    indices and is refused (SAI_ETOOBIG), as is a negative l_max (SAI_EINVAL)."""
    from oracle import psai as opsai
    w, (rp, ci, va) = _load("c3_3000")
    S = osplit.split(w.A)
    n = w.A.shape[0]
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_PSAI_TOL, delta=0.4, psai_lmax=1, precision=P.FP64, keep_lists=True)
    arr = pc.arrays()
    jp, ji, mf = _np(arr["j_ptr"]), _np(arr["j_idx"]), _np(arr["m_full"])
    Ss, ms, rs, ls = opsai.psai_tol(S.At, delta=0.4, lmax=1)
    for k in range(n):
        assert np.array_equal(ji[jp[k]:jp[k + 1]], Ss[k]), k
        assert np.linalg.norm(mf[jp[k]:jp[k + 1]] - ms[k]) <= 1e-12 * np.linalg.norm(ms[k]), k
    assert pc.stats.l_m == int(np.max(ls))
    print(f"l_max = 1: loops {np.bincount(ls)}, largest pattern {max(len(x) for x in Ss)}")
    with pytest.raises(P.SaiError) as e:
        P.Precond(g, pattern=P.PAT_PSAI_TOL, delta=0.4, psai_lmax=3)
    assert e.value.code == P.ETOOBIG
    with pytest.raises(P.SaiError) as e:
        P.Precond(g, pattern=P.PAT_PSAI_TOL, psai_lmax=-1)
    assert e.value.code == P.EINVAL


@pytest.mark.parametrize("kind", ["A", "spai"])
def test_standard_approach_vs_oracle(kind):
    """The standard approach (Section 5's S-SPAI; M built on A itself, no split):
    on the 45 x 45 workload the irregular columns give J_k of about 400 indices
    and I_k of about 1600 rows, past the fast kernels, so the large limits
    serve them.  Patterns bit-exact and values to 1e-12 against the oracle
    applied to A, and the solve of A x = b with M reaches (stopb)."""
    from oracle import spai as ospai
    w, (rp, ci, va) = _load("c1")
    n = w.A.shape[0]
    g = P.Split(rp, ci, va, dense_cols=[])
    assert g.s == 0
    kw = (dict(pattern=P.PAT_A, drop=P.DROP_NONE) if kind == "A" else
          dict(pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=0.4, spai_steps=3, spai_per_step=5))
    pc = P.Precond(g, precision=P.FP64, keep_lists=True, **kw)
    arr = pc.arrays()
    jp, ji, mf = _np(arr["j_ptr"]), _np(arr["j_idx"]), _np(arr["m_full"])
    C = opat.as_csc(w.A)
    out = ospai.spai(w.A, 3, 5, 0.4, "A") if kind == "spai" else None
    big = 0
    for k in range(n):
        if kind == "spai":
            J, I, m, res, _ = out[k]
        else:
            J = opat.pattern_A(C, k)
            I, m, res = olsq.solve_column(C, J, k)
        big += len(J) > 128
        assert np.array_equal(ji[jp[k]:jp[k + 1]], J), k
        assert np.linalg.norm(mf[jp[k]:jp[k + 1]] - m) <= 1e-12 * np.linalg.norm(m), k
    assert big > 0
    x, st = P.solve(g, pc, torch.from_numpy(w.b).cuda(), eps=1e-8)
    rr = np.linalg.norm(w.b - w.A @ _np(x)) / np.linalg.norm(w.b)
    assert rr < 0.5e-8, rr
    print(f"standard approach ({kind}): {big} columns with |J| > 128, iterations {st['iters']}, rr {rr:.2e}")


def test_psai_tol_solve():
    """A PSAI(tol) preconditioner drives the whole SMW-split solve: with c = 1 in
    (stopU2) the theorem bounds rr by (eps/2)(1 + c) for the computed c; with the
    refinement (SAI_C_ONE_THEN_REFINE) rr < eps strictly."""
    w, (rp, ci, va) = _load("c2_12")
    b = torch.from_numpy(w.b).cuda()
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_PSAI_TOL, delta=0.2, psai_lmax=10, precision=P.FP32)
    x, st = P.solve(g, pc, b, method=P.BICGSTAB, eps=1e-8)
    rr = np.linalg.norm(w.b - w.A @ _np(x)) / np.linalg.norm(w.b)
    assert rr < 1e-8 * (1.0 + st["c"]) / 2.0 * (1.0 + 1e-6), (rr, st)
    x, st = P.solve(g, pc, b, method=P.BICGSTAB, eps=1e-8, c_mode=P.C_ONE_THEN_REFINE)
    rr = np.linalg.norm(w.b - w.A @ _np(x)) / np.linalg.norm(w.b)
    assert rr < 1e-8, (rr, st)


def test_spai_long_search_from_diagonal():
    """SPAI from J = {k} with 6 steps of 8 columns: most columns go through
    several factor updates (rows appended at each), against the oracle's
    from-scratch solves: patterns and I bit-exact, values to 1e-12."""
    from oracle import spai as ospai
    w, (rp, ci, va) = _load("c3_3000")
    S = osplit.split(w.A)
    n = w.A.shape[0]
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=0.05, spai_steps=6,
                   spai_per_step=8, spai_init=P.INIT_DIAG, precision=P.FP64, keep_lists=True)
    arr = pc.arrays()
    jp, ji, ip, ii = (_np(arr[k]) for k in ("j_ptr", "j_idx", "i_ptr", "i_idx"))
    mf = _np(arr["m_full"])
    out = ospai.spai(S.At, steps=6, per_step=8, delta=0.05, init="diag")
    taken = np.zeros(7, dtype=np.int64)
    for k in range(n):
        J, I, m, res, t = out[k]
        taken[t] += 1
        assert np.array_equal(ji[jp[k]:jp[k + 1]], J), k
        assert np.array_equal(ii[ip[k]:ip[k + 1]], I), k
        e = np.linalg.norm(mf[jp[k]:jp[k + 1]] - m) / np.linalg.norm(m)
        assert e <= 1e-12, (k, e)
    assert taken[3:].sum() > n // 4
    print(f"augmentation steps taken per column: {taken.tolist()}")


@pytest.mark.parametrize("delta,init,prec", [(0.4, P.INIT_PATTERN_A, P.FP64),
                                              (0.05, P.INIT_PATTERN_A, P.FP64),
                                              (0.05, P.INIT_PATTERN_A, P.FP32),
                                              (0.2, P.INIT_DIAG, P.FP64)])
def test_spai_patterns_and_columns(delta, init, prec):
    from oracle import spai as ospai
    w, (rp, ci, va) = _load("c3_3000")
    S = osplit.split(w.A)
    n = w.A.shape[0]
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=delta, spai_steps=3,
                   spai_per_step=5, spai_init=init, precision=prec, keep_lists=True)
    arr = pc.arrays()
    jp, ji, ip, ii = (_np(arr[k]) for k in ("j_ptr", "j_idx", "i_ptr", "i_idx"))
    mf = _np(arr["m_full"]).astype(np.float64)
    out = ospai.spai(S.At, steps=3, per_step=5, delta=delta,
                     init="A" if init == P.INIT_PATTERN_A else "diag")
    tol = 1e-12 if prec == P.FP64 else 1e-4
    augmented = 0
    assert pc.stats.l_m == max(o[4] for o in out), (pc.stats.l_m, max(o[4] for o in out))
    for k in range(n):
        J, I, m, res, taken = out[k]
        augmented += taken > 0
        assert np.array_equal(ji[jp[k]:jp[k + 1]], J), k     # adaptive pattern: bit-exact
        assert np.array_equal(ii[ip[k]:ip[k + 1]], I), k
        e = np.linalg.norm(mf[jp[k]:jp[k + 1]] - m) / np.linalg.norm(m)
        assert e <= tol, (k, e)
    assert augmented > 0
    print(f"delta={delta}: {augmented} columns augmented")


@pytest.mark.parametrize("drop,prec", [(P.DROP_ABS, P.FP64), (P.DROP_TOLK, P.FP64),
                                       (P.DROP_ABS, P.FP32)])
def test_drop_and_assembly(drop, prec):
    w, (rp, ci, va) = _load("c2_12")
    S = osplit.split(w.A)
    n = w.A.shape[0]
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A2, drop=drop, tau=2e-3, delta=0.4, precision=prec,
                   keep_lists=True)
    arr = pc.arrays()
    jp, ji = _np(arr["j_ptr"]), _np(arr["j_idx"])
    Js = [ji[jp[k]:jp[k + 1]] for k in range(n)]
    _, ms, _ = olsq.build_columns(S.At, Js)
    mode = {P.DROP_ABS: "abs", P.DROP_TOLK: "tolk"}[drop]
    Mo = odrop.assemble(n, Js, ms, mode, tau=2e-3, delta=0.4, At=S.At)
    Mg = sp.csc_matrix((_np(arr["cval"]).astype(np.float64), _np(arr["row_idx"]),
                        _np(arr["col_ptr"])), shape=(n, n))
    flips = 0
    if prec == P.FP64:
        assert np.array_equal(Mg.indptr, Mo.indptr) and np.array_equal(Mg.indices, Mo.indices)
        assert abs(Mg - Mo).max() <= 1e-12 * abs(Mo).max()
    else:
        # entries within the FP32 build's tolerance of the threshold may flip: at
        # most the number the library reports as undecidable
        flips = abs((Mg != 0).astype(int) - (Mo != 0).astype(int)).sum()
        assert flips <= pc.stats.drop_flips, (flips, pc.stats.drop_flips)
    # the same count from the oracle's columns (FP64: the same entries)
    a1 = odrop.norm1(opat.as_csc(S.At))
    eta = 1e-4 if prec == P.FP32 else 1e-12
    near = 0
    for k in range(n):
        m = ms[k]
        tk = 2e-3 if drop == P.DROP_ABS else 0.4 / (len(m) * a1)
        big = int(np.argmax(np.abs(m)))
        band = eta * np.linalg.norm(m) / (1.0 - eta)
        near += sum(1 for q in range(len(m)) if q != big and abs(abs(m[q]) - tk) <= band)
    print(f"undecidable entries: library {pc.stats.drop_flips}, oracle {near}, flips seen "
          f"{flips if prec == P.FP32 else 0}")
    if prec == P.FP64:
        assert pc.stats.drop_flips == near
    assert (pc.stats.s, pc.stats.p) == (S.s, S.p)
    # CSR is the transpose of the CSC, bit for bit
    Mr = sp.csr_matrix((_np(arr["val"]).astype(np.float64), _np(arr["col_idx"]), _np(arr["row_ptr"])),
                       shape=(n, n))
    Mg.sort_indices()
    assert (Mr != sp.csr_matrix(Mg)).nnz == 0


_SIGMA_MIN = {}


def _sigma_min(name, A):
    """Smallest singular value of A (dense SVD, n <= 3000), cached per case."""
    if name not in _SIGMA_MIN:
        _SIGMA_MIN[name] = float(np.linalg.svd(A.toarray(), compute_uv=False)[-1])
    return _SIGMA_MIN[name]


def _forward_bound(name, A, b, x1, x2):
    """||x1 - x2|| <= ||A^{-1}|| (||b - A x1|| + ||b - A x2||): both residuals are
    recomputed here in float64, ||A^{-1}||_2 = 1 / sigma_min from a dense SVD."""
    return (np.linalg.norm(b - A @ x1) + np.linalg.norm(b - A @ x2)) / _sigma_min(name, A)


SOLVE_CASES = [("c1", P.GMRES), ("c1", P.BICGSTAB), ("c2_12", P.BICGSTAB), ("c2_13x9x7", P.BICGSTAB),
               ("c4_40", P.BICGSTAB), ("c3_3000", P.BICGSTAB)]


def _solve_both(name, method, c_mode):
    w, (rp, ci, va) = _load(name)
    b = torch.from_numpy(w.b).cuda()
    g = P.Split(rp, ci, va)
    kind = P.PAT_A if name in ("c1", "c3_3000") else P.PAT_A2
    drop = P.DROP_NONE if kind == P.PAT_A else P.DROP_ABS
    pc = P.Precond(g, pattern=kind, drop=drop, tau=1e-3, precision=P.FP32)
    x, st = P.solve(g, pc, b, method=method, restart=30, eps=1e-8, c_mode=c_mode)
    out = opipe.run(w.A, w.b, kind="A" if kind == P.PAT_A else "A2",
                    drop="none" if drop == P.DROP_NONE else "abs",
                    method="gmres" if method == P.GMRES else "bicgstab")
    return w, _np(x), st, out


@pytest.mark.parametrize("name,method", SOLVE_CASES)
def test_solve_c_one_vs_oracle(name, method):
    """The paper's setting, c = 1 in (stopU2): the theorem then bounds the final
    residual by (eps/2)(1 + c) (b - A x = r_y - R_W z, ||R_W z|| < eps ||b|| c / 2),
    which exceeds eps when c > 1.  x is compared with the oracle's x through
    ||A^{-1}|| times the sum of both true residuals."""
    w, xs, st, out = _solve_both(name, method, P.C_ONE)
    rr = np.linalg.norm(w.b - w.A @ xs) / np.linalg.norm(w.b)
    c = st["c"]
    assert rr < 1e-8 * (1.0 + c) / 2.0 * (1.0 + 1e-6), (rr, c, st)
    assert abs(rr - st["rr"]) <= 1e-3 * rr + 1e-15
    err = np.linalg.norm(xs - out["x"])
    bound = _forward_bound(name, w.A, w.b, xs, out["x"])
    assert err <= bound, (err, bound)
    print(f"{name}: gpu iters {st['iters']} oracle iters {out['iters']} rr {rr:.2e} / {out['rr']:.2e}, "
          f"|x - x_oracle| / |x_oracle| {err / np.linalg.norm(out['x']):.2e} "
          f"(bound {bound / np.linalg.norm(out['x']):.2e})")


@pytest.mark.parametrize("name,method", SOLVE_CASES)
def test_solve_refined_strict(name, method):
    """SAI_C_ONE_THEN_REFINE: the auxiliary solves are continued to the theorem's
    thresholds with the computed c, so rr < 1e-8 strictly, recomputed on the
    host; x against the oracle's as above."""
    w, xs, st, out = _solve_both(name, method, P.C_ONE_THEN_REFINE)
    rr = np.linalg.norm(w.b - w.A @ xs) / np.linalg.norm(w.b)
    assert st["status"] == P.OK and rr < 1e-8, (rr, st)
    err = np.linalg.norm(xs - out["x"])
    bound = _forward_bound(name, w.A, w.b, xs, out["x"])
    assert err <= bound, (err, bound)


def test_krylov_block_and_smw_vs_oracle():
    w, (rp, ci, va) = _load("c2_12")
    S = osplit.split(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, precision=P.FP64)
    n, s = w.A.shape[0], S.s
    R = np.zeros((n, s + 1))
    R[:, 0] = w.b
    R[:, 1:] = S.U.toarray()
    thr = okry.thresholds(np.linalg.norm(w.b), s, 1e-10)
    Rt = torch.from_numpy(R).cuda()
    X, its, sts, code = P.krylov(g, pc, Rt, thr)
    assert code == P.OK and all(v == 0 for v in sts)
    Xh = _np(X)
    for c in range(s + 1):
        assert np.linalg.norm(R[:, c] - S.At @ Xh[:, c]) < thr[c]
    # SMW recovery on the same Y, compared with the oracle's recovery
    x, cval = P.smw(g, X)
    xo, z, co = osmw.recover(Xh[:, 0], Xh[:, 1:], S.D)
    assert np.linalg.norm(_np(x) - xo) <= 1e-12 * np.linalg.norm(xo)
    assert abs(cval - co) <= 1e-12 * co
    rr = P.residual(g, torch.from_numpy(w.b).cuda(), x)
    assert abs(rr - osmw.relres(w.A, xo, w.b)) <= 1e-6 * rr + 1e-18
    # transposed solve
    Xt, its, sts, code = P.krylov(g, pc, Rt, thr, transpose=True)
    Xth = _np(Xt)
    AtT = sp.csr_matrix(S.At.T)
    for c in range(s + 1):
        assert np.linalg.norm(R[:, c] - AtT @ Xth[:, c]) < thr[c]


@pytest.mark.parametrize("name", ["c1", "c2_12", "c4_40"])
def test_adjoint_vs_oracle(name):
    w, (rp, ci, va) = _load(name)
    g = P.Split(rp, ci, va)
    kind = P.PAT_A if name == "c1" else P.PAT_A2
    pc = P.Precond(g, pattern=kind, drop=P.DROP_ABS if kind == P.PAT_A2 else P.DROP_NONE,
                   precision=P.FP32)
    b = torch.from_numpy(w.b).cuda()
    x, _ = P.solve(g, pc, b, eps=1e-12)
    xs = W.x_star(w.A.shape[0], w.seed)
    gx = x - torch.from_numpy(xs).cuda()
    gb, ga, st = P.backward(g, pc, x, gx, eps=1e-12)
    Ad = w.A.toarray()
    xd = np.linalg.solve(Ad, w.b)
    lam = np.linalg.solve(Ad.T, xd - xs)
    Gd = oadj.grad_A_values(w.A, lam, xd)
    assert np.linalg.norm(_np(gb) - lam) <= 1e-5 * np.linalg.norm(lam)
    assert np.linalg.norm(_np(ga) - Gd) <= 1e-5 * np.linalg.norm(Gd)


def test_more_than_64_right_hand_sides():
    """s = 100 irregular columns (101 right-hand sides, solved in groups of 64
    and 37): the forward solve against the oracle pipeline (rr within the
    theorem's (eps/2)(1 + c), x within ||A^{-1}|| times both residuals), the
    Krylov block against the oracle column by column, and the adjoint (U^T Z
    reduced in two column groups) against the dense solve."""
    w = W.make(4, dims=(60, 60), s=100, density=0.15)
    rp, ci, va = P.csr_to_device(w.A)
    g = P.Split(rp, ci, va)
    assert g.s == 100
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP64)
    b = torch.from_numpy(w.b).cuda()
    x, st = P.solve(g, pc, b)
    xs = _np(x)
    out = opipe.run(w.A, w.b, kind="A2", drop="abs")
    rr = np.linalg.norm(w.b - w.A @ xs) / np.linalg.norm(w.b)
    assert st["status"] == P.OK and rr < 1e-8 * (1.0 + st["c"]) / 2.0 * (1.0 + 1e-6), (rr, st["c"])
    assert len(st["iters"]) == 101 and all(abs(a - o) <= 1 for a, o in zip(st["iters"], out["iters"]))
    smin = float(np.linalg.svd(w.A.toarray(), compute_uv=False)[-1])
    bound = (np.linalg.norm(w.b - w.A @ xs) + np.linalg.norm(w.b - w.A @ out["x"])) / smin
    assert np.linalg.norm(xs - out["x"]) <= bound
    # the block through sai_krylov directly, against the oracle's solves
    S = osplit.split(w.A)
    R = np.zeros((w.A.shape[0], 101))
    R[:, 0] = w.b
    R[:, 1:] = S.U.toarray()
    thr = okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)
    X, its, sts, code = P.krylov(g, pc, torch.from_numpy(R).cuda(), thr)
    assert code == P.OK and all(v == 0 for v in sts)
    Xh = _np(X)
    At = sp.csr_matrix(S.At)
    for c in range(101):
        assert np.linalg.norm(R[:, c] - At @ Xh[:, c]) < thr[c], c
    # adjoint
    xst = W.x_star(w.A.shape[0], w.seed)
    gx = x - torch.from_numpy(xst).cuda()
    gb, ga, bst = P.backward(g, pc, x, gx, eps=1e-12)
    Ad = w.A.toarray()
    lam = np.linalg.solve(Ad.T, xs - xst)
    assert np.linalg.norm(_np(gb) - lam) <= 1e-5 * np.linalg.norm(lam)
    Gd = oadj.grad_A_values(w.A, lam, xs)
    assert np.linalg.norm(_np(ga) - Gd) <= 1e-5 * np.linalg.norm(Gd)


@pytest.mark.parametrize("width", ["narrow", "wide"])
def test_m_product_variants_bit_identical(width):
    """The sparse products' gather-batch variants (SPMM_M = 0 .. 4 and SPMM_A =
    0 .. 5, or SPMM_M_WIDE / SPMM_A_WIDE for blocks over 32 columns, chosen by
    the autotuner) change only how many loads are in flight: each row's
    products are added in the same order, so the whole Krylov solve is
    bit-identical.  So are the output blocks stored and the streamed ones read
    non-temporally (NT_STORE = NT_LOAD = 1; blocks this small use plain accesses
    by default).  narrow: [b, U] of a 12^3
    matrix (5 columns); wide: 40 seeded right-hand sides (the 32-lane class)."""
    w, (rp, ci, va) = _load("c2_12")
    S = osplit.split(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP32)
    if width == "narrow":
        R, _ = _oracle_rhs_and_M(w, S)
        thr = okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)
        km, ka, dm, da = "SPMM_M", "SPMM_A", 1, 0
    else:
        R = np.random.default_rng(40).standard_normal((w.A.shape[0], 40))
        thr = [1e-10 * np.linalg.norm(R[:, c]) for c in range(40)]
        km, ka, dm, da = "SPMM_M_WIDE", "SPMM_A_WIDE", 4, 5
    cases = [(dm, da, -1)] + [(v, da, -1) for v in range(5) if v != dm] + [(dm, v, -1) for v in range(6) if v != da]
    cases += [(dm, da, 1), (dm, da, 0)]
    out = []
    try:
        for m, a, nt in cases:
            P.tune_set(km, m)
            P.tune_set(ka, a)
            P.tune_set("NT_STORE", nt)
            P.tune_set("NT_LOAD", nt)
            X, its, sts, code = P.krylov(g, pc, torch.from_numpy(R).cuda(), thr)
            assert code == P.OK
            out.append((_np(X), its))
    finally:
        P.tune_set(km, dm)
        P.tune_set(ka, da)
        P.tune_set("NT_STORE", -1)
        P.tune_set("NT_LOAD", -1)
    for X, its in out[1:]:
        assert its == out[0][1] and np.array_equal(X, out[0][0])


def test_autograd_function():
    w, (rp, ci, va) = _load("c2_12")
    a = va.clone().requires_grad_(True)
    b = torch.from_numpy(w.b).cuda().requires_grad_(True)
    x = P.SAISolve.apply(a, b, rp, ci, dict(pattern=P.PAT_A2, drop=P.DROP_ABS, precision=P.FP32),
                         dict(eps=1e-12))
    xs = torch.from_numpy(W.x_star(w.A.shape[0], w.seed)).cuda()
    loss = 0.5 * ((x - xs) ** 2).sum()
    loss.backward()
    Ad = w.A.toarray()
    xd = np.linalg.solve(Ad, w.b)
    lam = np.linalg.solve(Ad.T, xd - _np(xs))
    assert np.linalg.norm(_np(b.grad) - lam) <= 1e-5 * np.linalg.norm(lam)
    Gd = oadj.grad_A_values(w.A, lam, xd)
    assert np.linalg.norm(_np(a.grad) - Gd) <= 1e-5 * np.linalg.norm(Gd)


def test_error_paths():
    # irregular column without a diagonal -> SAI_EZERODIAG
    n = 30
    A = sp.lil_matrix((n, n))
    for i in range(n):
        if i != 3:
            A[i, i] = 2.0
    for i in range(n):
        if i != 3:
            A[i, 3] = 0.5
    A = sp.csr_matrix(A)
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    rp, ci, va = P.csr_to_device(A)
    with pytest.raises(P.SaiError) as e:
        P.Split(rp, ci, va)
    assert e.value.code == P.EZERODIAG
    # unsorted columns -> SAI_EINVAL
    w, (rp, ci, va) = _load("c1")
    ci2 = ci.clone()
    ci2[[0, 1]] = ci2[[1, 0]]
    with pytest.raises(P.SaiError) as e:
        P.Split(rp, ci2, va)
    assert e.value.code == P.EINVAL
    # maxit = 1 -> SAI_ENOCONV with outputs written
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A, drop=P.DROP_NONE)
    x, st = P.solve(g, pc, torch.from_numpy(w.b).cuda(), maxit=1, raise_on_error=False)
    assert st["code"] == P.ENOCONV and np.isfinite(_np(x)).all()


@pytest.mark.parametrize("name", ["c2_12", "c3_3000", "c2_13x9x7"])
def test_krylov_block_widths(name):
    # BiCGStab on blocks of every width class (k = 1 .. 23 columns, odd and even,
    # so that every lanes-per-row variant and the pad column are exercised),
    # forward and transposed: every column meets its own true-residual threshold.
    w, (rp, ci, va) = _load(name)
    S = osplit.split(w.A)
    g = P.Split(rp, ci, va)
    kind = P.PAT_A if name == "c3_3000" else P.PAT_A2
    pc = P.Precond(g, pattern=kind, drop=P.DROP_ABS, tau=1e-3, precision=P.FP32)
    n = w.A.shape[0]
    rng = np.random.default_rng(5)
    ks = (1, 2, 3, 5, 8, 11, 13, 23, 29, 40) if name == "c2_12" else (1, 11, 23)
    for k in ks:
        R = rng.standard_normal((n, k))
        thr = [1e-10 * np.linalg.norm(R[:, c]) for c in range(k)]
        Rt = torch.from_numpy(R).cuda()
        for transpose in (False, True):
            Aop = S.At if not transpose else sp.csr_matrix(S.At.T)
            X, its, sts, code = P.krylov(g, pc, Rt, thr, transpose=transpose)
            assert code == P.OK and all(v == 0 for v in sts), (k, transpose, its, sts)
            Xh = _np(X)
            for c in range(k):
                assert np.linalg.norm(R[:, c] - Aop @ Xh[:, c]) < thr[c], (k, transpose, c)


def test_krylov_long_rows():
    # Rows far longer than a tile's LDS staging area (A~ and, with J_k = P(A~(:,k)),
    # M get rows of 2500 entries): the products fall back to reading those tiles from
    # global memory; every column still meets its true-residual threshold.
    n = 3000
    rng = np.random.default_rng(11)
    rows, cols = [], []
    for i in range(n):
        c = rng.choice(n, size=5, replace=False)
        rows += [i] * len(c)
        cols += c.tolist()
    for i in (100, 1700, 2900):
        c = rng.choice(n, size=2500, replace=False)
        rows += [i] * len(c)
        cols += c.tolist()
    vals = 0.05 * rng.standard_normal(len(rows))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.setdiag(0.0)
    A.eliminate_zeros()
    A = A + sp.diags(1.5 * np.asarray(abs(A).sum(axis=1)).ravel() + 1.0)
    A = sp.csr_matrix(A)
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    S = osplit.split(A)
    rp, ci, va = P.csr_to_device(A)
    g = P.Split(rp, ci, va)
    assert g.s == S.s
    pc = P.Precond(g, pattern=P.PAT_A, drop=P.DROP_NONE, precision=P.FP32)
    assert int(np.diff(_np(pc.arrays()["row_ptr"])).max()) >= 2500
    for k in (3, 11):
        R = rng.standard_normal((n, k))
        thr = [1e-10 * np.linalg.norm(R[:, c]) for c in range(k)]
        Rt = torch.from_numpy(R).cuda()
        for transpose in (False, True):
            Aop = S.At if not transpose else sp.csr_matrix(S.At.T)
            X, its, sts, code = P.krylov(g, pc, Rt, thr, transpose=transpose)
            assert code == P.OK and all(v == 0 for v in sts), (k, transpose, its, sts)
            Xh = _np(X)
            for c in range(k):
                assert np.linalg.norm(R[:, c] - Aop @ Xh[:, c]) < thr[c], (k, transpose, c)


def _csr32(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


@pytest.mark.parametrize("case", ["n1", "n2", "tridiag5", "stencil30_s0"])
def test_degenerate_sizes_and_no_dense_columns(case):
    """s = 0 (no irregular column: x = y, no SMW) and matrices of 1, 2 and 5 rows,
    through the split, both static patterns, the solve and (30 x 30) the adjoint."""
    if case == "n1":
        A = np.array([[3.0]])
    elif case == "n2":
        A = np.array([[4.0, -1.0], [-1.5, 3.0]])
    elif case == "tridiag5":
        A = sp.diags([np.full(4, -1.0), np.full(5, 2.5), np.full(4, -0.7)], [-1, 0, 1])
    else:
        r, c, v, nn = W.stencil((30, 30), 7)
        A = sp.coo_matrix((v, (r, c)), shape=(nn, nn))
    A = _csr32(A)
    n = A.shape[0]
    b = A @ np.linspace(1.0, 2.0, n)
    g = P.Split(*P.csr_to_device(A))
    assert g.s == 0
    xd = sp.linalg.spsolve(sp.csc_matrix(A), b) if n > 1 else b / A.toarray()[0, 0]
    for kind in (P.PAT_A, P.PAT_A2):
        pc = P.Precond(g, pattern=kind, drop=P.DROP_NONE, precision=P.FP64)
        x, st = P.solve(g, pc, torch.from_numpy(b).cuda(), eps=1e-8)
        xs = _np(x)
        rr = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
        assert rr < 1e-8, (case, kind, rr, st)  # s = 0: x = y, (stopb) gives rr < eps / 2
        assert np.linalg.norm(xs - xd) <= 1e-6 * np.linalg.norm(xd), (case, kind)
    if case == "stencil30_s0":
        gx = torch.from_numpy(np.cos(np.arange(n))).cuda()
        gb, ga, bst = P.backward(g, pc, x, gx)
        lam = sp.linalg.spsolve(sp.csc_matrix(A.T), _np(gx))
        assert np.linalg.norm(_np(gb) - lam) <= 1e-6 * np.linalg.norm(lam)


def test_repeat_runs_bit_identical():
    w, (rp, ci, va) = _load("c2_12")
    b = torch.from_numpy(w.b).cuda()
    outs = []
    for _ in range(2):
        g = P.Split(rp, ci, va)
        pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, precision=P.FP32)
        x, _ = P.solve(g, pc, b)
        outs.append(_np(x))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("kind", ["spai", "psai_tol"])
def test_adaptive_builds_bit_identical(kind):
    """The adaptive searches hand columns to workgroups dynamically (largest
    first); M and the solution must not depend on that order."""
    w, (rp, ci, va) = _load("c3_3000")
    b = torch.from_numpy(w.b).cuda()
    if kind == "spai":
        kw = dict(pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=0.05, spai_steps=3, spai_per_step=5)
    else:
        kw = dict(pattern=P.PAT_PSAI_TOL, delta=0.4, psai_lmax=0)
    outs = []
    for _ in range(2):
        g = P.Split(rp, ci, va)
        pc = P.Precond(g, precision=P.FP32, **kw)
        arr = pc.arrays()
        x, _ = P.solve(g, pc, b)
        outs.append([_np(arr[k]) for k in ("col_ptr", "row_idx", "cval")] + [_np(x)])
    for u, v in zip(*outs):
        assert np.array_equal(u, v)


def _oracle_rhs_and_M(w, S):
    """[b, U] and the oracle's FP64 M (P(|A~|^2), tau = 1e-3) for the workload."""
    n, s = w.A.shape[0], S.s
    R = np.zeros((n, s + 1))
    R[:, 0] = w.b
    R[:, 1:] = S.U.toarray()
    Mo, _ = opipe.build_M(S, "A2", "abs", 1e-3)
    return R, sp.csr_matrix(Mo)


@pytest.mark.parametrize("at", [1, 5])
def test_bicgstab_forced_restart(at):
    """The breakdown restart (r_hat = r, p = v = 0), forced at the end of
    iteration `at` for every active column, against the oracle restarted at the
    same iteration (same FP64 M up to 1e-12): iteration counts equal (one
    apart at most, for a column that meets its threshold within rounding), and
    every column within ||A~^{-1}|| (sum of the two true residuals) of the
    oracle's."""
    w, (rp, ci, va) = _load("c2_12")
    S = osplit.split(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP64)
    R, Mo = _oracle_rhs_and_M(w, S)
    thr = okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)
    try:
        P.tune_set("BRK_TEST", at)
        X, its, sts, code = P.krylov(g, pc, torch.from_numpy(R).cuda(), thr)
    finally:
        P.tune_set("BRK_TEST", 0)
    assert code == P.OK and all(v == 0 for v in sts), (its, sts)
    At = sp.csr_matrix(S.At)
    Xo, itso, stso = okry.solve_block(At, Mo, R, thr, force_restart_at=[at])
    assert all(v == "converged" for v in stso)
    Xh = _np(X)
    smin = float(np.linalg.svd(S.At.toarray(), compute_uv=False)[-1])
    for c in range(S.s + 1):
        assert abs(its[c] - itso[c]) <= 1, (c, its, itso)
        rg = np.linalg.norm(R[:, c] - At @ Xh[:, c])
        ro = np.linalg.norm(R[:, c] - At @ Xo[:, c])
        assert rg < thr[c]
        assert np.linalg.norm(Xh[:, c] - Xo[:, c]) <= (rg + ro) / smin, c
    print(f"restart at {at}: gpu iterations {its}, oracle {itso}")


def test_bicgstab_second_breakdown_vs_oracle():
    """Two forced breakdowns (iterations 3 and 6): every column still active at
    iteration 6 ends with status breakdown, sai_krylov returns SAI_EBREAKDOWN and
    the iterates it wrote equal the oracle's at that point (same FP64 M)."""
    w, (rp, ci, va) = _load("c2_12")
    S = osplit.split(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP64)
    R, Mo = _oracle_rhs_and_M(w, S)
    thr = okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)
    try:
        P.tune_set("BRK_TEST", 3)
        P.tune_set("BRK_TEST2", 6)
        X, its, sts, code = P.krylov(g, pc, torch.from_numpy(R).cuda(), thr)
        x, st = P.solve(g, pc, torch.from_numpy(w.b).cuda(), eps=1e-10, raise_on_error=False)
    finally:
        P.tune_set("BRK_TEST", 0)
        P.tune_set("BRK_TEST2", 0)
    Xo, itso, stso = okry.solve_block(sp.csr_matrix(S.At), Mo, R, thr, force_restart_at=[3, 6])
    assert code == P.EBREAKDOWN and st["code"] == P.EBREAKDOWN and st["status"] == P.EBREAKDOWN
    assert all(v == "breakdown" for v in stso) and all(v == 2 for v in sts), (sts, stso)
    assert list(its) == list(itso) == [6] * (S.s + 1), (its, itso)
    Xh = _np(X)
    for c in range(S.s + 1):
        assert np.linalg.norm(Xh[:, c] - Xo[:, c]) <= 1e-9 * np.linalg.norm(Xo[:, c]), c
    assert np.isfinite(_np(x)).all()


def _csr_from_dense(D):
    return _csr32(sp.csr_matrix(np.asarray(D, dtype=np.float64)))


def test_singular_K_from_singular_A():
    """A singular, A~ nonsingular: by Theorem 3.1, K = I + V^T W is singular.
    A~ = 2I plus a_01 = 1, one irregular column 0 (13 entries > 10p, p = 1,
    keep = 1) with a_10 = 4: then M = A~^{-1} exactly, the auxiliary solve is
    exact (one half step, alpha = 1), w_0 = -1 and K = 1 + w_0 = 0.  The GPU
    solve returns SAI_ESINGULAR; the oracle's recovery raises."""
    n = 40
    D = 2.0 * np.eye(n)
    D[0, 1] = 1.0
    D[1, 0] = 4.0
    for i in range(2, 13):
        D[i, 0] = 0.5 * i
    A = _csr_from_dense(D)
    assert abs(np.linalg.det(D)) < 1e-9
    b = A @ np.ones(n)
    g = P.Split(*P.csr_to_device(A))
    assert g.s == 1
    for prec in (P.FP64, P.FP32):
        pc = P.Precond(g, pattern=P.PAT_A, drop=P.DROP_NONE, precision=prec)
        with pytest.raises(P.SaiError) as e:
            P.solve(g, pc, torch.from_numpy(b).cuda(), eps=1e-8)
        assert e.value.code == P.ESINGULAR
    with pytest.raises(osmw.SingularK):
        opipe.run(A, b, kind="A", drop="none")


def test_rank_deficient_column_block():
    """A column block without full column rank: columns 3 and 4 of A~ each have
    one entry, in row 3 (values 2 and 4), and column 10 holds rows 3, 4, 10, so
    A~(I_10, J_10) with J_10 = P(A~(:, 10)) = {3, 4, 10} has rank 2.  The build
    returns SAI_ESINGULAR in both precisions; the oracle's triangular solve
    raises."""
    import scipy.linalg as sla
    n = 20
    D = 2.0 * np.eye(n)
    D[4, 4] = 0.0
    D[3, 4] = 4.0
    D[3, 10] = 1.0
    D[4, 10] = -1.0
    A = _csr_from_dense(D)
    g = P.Split(*P.csr_to_device(A))
    assert g.s == 0
    for prec in (P.FP64, P.FP32):
        with pytest.raises(P.SaiError) as e:
            P.Precond(g, pattern=P.PAT_A, drop=P.DROP_NONE, precision=prec)
        assert e.value.code == P.ESINGULAR
    C = opat.as_csc(osplit.split(A).At)
    assert list(opat.pattern_A(C, 10)) == [3, 4, 10]
    with pytest.raises(sla.LinAlgError):
        olsq.solve_column(C, opat.pattern_A(C, 10), 10)


def test_split_dense_cols_override():
    """host_dense_cols / s_given replace the count rule: the oracle's split with
    the same irregular columns (forced through a dense factor that selects
    exactly them) is reproduced bit for bit; s_given = 0 gives A~ = A; a bad
    list is rejected."""
    w, (rp, ci, va) = _load("c2_12")
    S = osplit.split(w.A)
    # the largest columns of the oracle's list, plus a regular one
    counts = np.diff(sp.csc_matrix(w.A).indptr)
    extra = int(np.argmax(np.where(np.isin(np.arange(len(counts)), S.D), -1, counts)))
    cols = sorted([int(S.D[0]), int(S.D[-1]), extra])
    g = P.Split(rp, ci, va, dense_cols=cols)
    arr = g.arrays()
    assert g.s == 3 and list(_np(arr["dense_cols"])) == cols
    # expected: the oracle split rule applied to exactly these columns
    So = osplit.split(w.A, dense_cols=cols)
    assert np.array_equal(_np(arr["t_col_idx"]), So.At.indices)
    assert np.array_equal(_np(arr["t_val"]), So.At.data)
    assert np.array_equal(_np(arr["t_row_ptr"]), So.At.indptr)
    g0 = P.Split(rp, ci, va, dense_cols=[])
    assert g0.s == 0 and g0.info.nnz_t == w.A.nnz
    for bad in ([5, 3], [1, 1], [-1], [w.A.shape[0]]):
        with pytest.raises(P.SaiError) as e:
            P.Split(rp, ci, va, dense_cols=bad)
        assert e.value.code == P.EINVAL


@pytest.mark.parametrize("init", [P.INIT_PATTERN_A, P.INIT_DIAG])
def test_spai_zero_steps(init):
    """spai_steps = 0: no augmentation, J_k = P(A~(:, k)) (then M is the static
    P(A~) build, bit for bit) or {k}; against the oracle."""
    from oracle import spai as ospai
    w, (rp, ci, va) = _load("c3_3000")
    S = osplit.split(w.A)
    n = w.A.shape[0]
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=0.4, spai_steps=0,
                   spai_per_step=5, spai_init=init, precision=P.FP64, keep_lists=True)
    arr = pc.arrays()
    jp, ji = _np(arr["j_ptr"]), _np(arr["j_idx"])
    mf = _np(arr["m_full"])
    out = ospai.spai(S.At, steps=0, per_step=5, delta=0.4,
                     init="A" if init == P.INIT_PATTERN_A else "diag")
    for k in range(n):
        J, I, m, res, taken = out[k]
        assert taken == 0
        assert np.array_equal(ji[jp[k]:jp[k + 1]], J), k
        assert np.linalg.norm(mf[jp[k]:jp[k + 1]] - m) <= 1e-12 * np.linalg.norm(m), k
    if init == P.INIT_PATTERN_A:
        ref = P.Precond(g, pattern=P.PAT_A, drop=P.DROP_NONE, precision=P.FP64).arrays()
        for key in ("col_ptr", "row_idx", "cval"):
            assert np.array_equal(_np(arr[key]), _np(ref[key])), key


@pytest.mark.parametrize("name,kind", [("c1", P.PAT_A), ("c2_12", P.PAT_A2), ("c2_13x9x7", P.PAT_A2),
                                       ("c3_3000", P.PAT_SPAI), ("banded", P.PAT_A2)])
@pytest.mark.parametrize("prec", [P.FP64, P.FP32])
def test_gather_vs_oracle(name, kind, prec):
    """sai_gather writes A~(I_k, J_k) for every column: bit-exact against the
    oracle's dense block (FP32: its float32 rounding).  Blocks of up to 256 rows,
    64 columns and 256 gathered entries are staged in LDS and written with
    16-byte stores (unaligned heads and tails element by element); the SPAI case
    also has blocks past those limits, which are filled element by element from
    global memory."""
    if name == "banded":
        A = W.banded(600, 8, 2, 0.5, 7)
        dev = P.csr_to_device(A)
    else:
        w, dev = _load(name)
        A = w.A
    S = osplit.split(A)
    C = opat.as_csc(S.At)
    g = P.Split(*dev)
    kw = dict(delta=0.05, spai_steps=3, spai_per_step=5) if kind == P.PAT_SPAI else {}
    pc = P.Precond(g, pattern=kind, drop=P.DROP_NONE, precision=P.FP32, keep_lists=True, **kw)
    arr = pc.arrays()
    jp, ji, ip, ii = (_np(arr[k]) for k in ("j_ptr", "j_idx", "i_ptr", "i_idx"))
    off, blocks = P.gather(g, pc, precision=prec)
    off, blocks = _np(off), _np(blocks)
    n = A.shape[0]
    assert off[0] == 0 and off[-1] == int(np.sum(np.diff(jp) * np.diff(ip)))
    colnnz = np.diff(C.indptr)
    big = 0
    for k in range(n):
        J, I = ji[jp[k]:jp[k + 1]], ii[ip[k]:ip[k + 1]]
        ref = olsq.dense_block(C, I, J)
        got = blocks[off[k]:off[k + 1]].reshape(len(J), len(I)).T
        if prec == P.FP32:
            ref = ref.astype(np.float32)
        assert np.array_equal(got, ref), k
        staged = len(I) <= 256 and len(J) <= 64 and int(colnnz[J].sum()) <= 256
        big += not staged
    if name == "c3_3000":
        assert big > 0
    print(f"{name}: {big} blocks past the staging limits")


def test_solve_equilibrated_vs_oracle():
    """Section 4's scaling of b (equilibrate): with b = 1e10 A 1 the unscaled
    solve misses eps by far (c = 1 makes the auxiliary thresholds far too
    loose), the scaled one meets rr < eps; x against the oracle's scaled solve
    through ||A^{-1}|| times both residuals, and x(1e-10 b) = 1e-10 x(b)."""
    w, (rp, ci, va) = _load("c2_12")
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP32)
    bb = 1e10 * w.b
    x0, st0 = P.solve(g, pc, torch.from_numpy(bb).cuda(), eps=1e-8, raise_on_error=False)
    rr0 = np.linalg.norm(bb - w.A @ _np(x0)) / np.linalg.norm(bb)
    x1, st1 = P.solve(g, pc, torch.from_numpy(bb).cuda(), eps=1e-8, equilibrate=True)
    xs = _np(x1)
    rr1 = np.linalg.norm(bb - w.A @ xs) / np.linalg.norm(bb)
    assert rr0 > 1e-3 and rr1 < 1e-8, (rr0, rr1)
    out = opipe.run(w.A, bb, kind="A2", drop="abs", tau=1e-3, equilibrate=True)
    assert np.linalg.norm(xs - out["x"]) <= _forward_bound("c2_12", w.A, bb, xs, out["x"])
    x2, st2 = P.solve(g, pc, torch.from_numpy(1e-10 * w.b).cuda(), eps=1e-8, equilibrate=True)
    assert np.linalg.norm(_np(x2) * 1e20 - xs) <= 1e-10 * np.linalg.norm(xs)
    print(f"unscaled rr {rr0:.2e}, scaled rr {rr1:.2e}, iterations {st1['iters']}")


@pytest.mark.parametrize("knobs", [dict(LP_MIN=2), dict(LP_MIN=4), dict(XMAP=0), dict(XMAP=3),
                                   dict(XMAP=16), dict(PERSIST=0), dict(SPMM_M_LP2=0)],
                         ids=["lp_min2", "lp_min4", "round_robin", "runs3", "runs16", "not_persistent",
                              "m_one_lane"])
def test_launch_knobs_vs_oracle(knobs):
    """Launch-shape knobs the tuning file may set (the smallest lane class, the
    tile-to-XCD maps: round-robin, runs of 3 or 16 tiles per XCD; grids larger
    than the resident count; the M product of one-column blocks on one lane per
    row instead of two) change only rounding: [b, U] of a 12^3 matrix and
    one seeded right-hand side solved with each, every true residual below its
    threshold, iterations within 2 of the oracle's, x within ||A~^{-1}| (sum of
    both true residuals) of the oracle's."""
    w, (rp, ci, va) = _load("c2_12")
    S = osplit.split(w.A)
    g = P.Split(rp, ci, va)
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP64)
    R, Mo = _oracle_rhs_and_M(w, S)
    r1 = np.random.default_rng(77).standard_normal((w.A.shape[0], 1))
    At = sp.csr_matrix(S.At)
    smin = float(np.linalg.svd(S.At.toarray(), compute_uv=False)[-1])
    for RR, thr in ((R, okry.thresholds(np.linalg.norm(w.b), S.s, 1e-10)),
                    (r1, [1e-10 * np.linalg.norm(r1)])):
        try:
            for kname, v in knobs.items():
                P.tune_set(kname, v)
            X, its, sts, code = P.krylov(g, pc, torch.from_numpy(np.ascontiguousarray(RR)).cuda(), thr)
        finally:
            P.tune_clear()
        assert code == P.OK and all(v == 0 for v in sts), (knobs, its, sts)
        Xh = _np(X)
        Xo, itso, _ = okry.solve_block(At, Mo, RR, thr)
        for c in range(RR.shape[1]):
            rg = np.linalg.norm(RR[:, c] - At @ Xh[:, c])
            ro = np.linalg.norm(RR[:, c] - At @ Xo[:, c])
            assert rg < thr[c] and abs(its[c] - itso[c]) <= 2, (knobs, c, rg, its, itso)
            assert np.linalg.norm(Xh[:, c] - Xo[:, c]) <= (rg + ro) / smin
