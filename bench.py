#!/usr/bin/env python3
"""Benchmark of the SMW-split SAI path on one MI355X.

Default workload (--workload 5, the largest single-GPU configuration): 3D
7-point convection-diffusion on a 160^3 grid (n = 4,096,000) with s = 50 seeded
dense columns at 1% density; static pattern P(|A~|^2) with absolute dropping
1e-3; M built in FP32 ("mixed"), Krylov/SMW/check in FP64; 51 right-hand sides
in one batched BiCGStab, eps = 1e-8; then the adjoint of the loss
0.5 ||x - x*||^2 from the forward solve's W = A~^{-1} U (one transposed system
per correction pass, its true residual below 1e-8) and the gradients.  Workloads 1-4 are the other
configurations (GMRES(30) on a 45x45 grid; the 100^3 grid with s = 10; SPAI on
a random n = 200,000 matrix; the 500x500 grid with the adjoint).

One step = the whole path on inputs already resident in HBM: split A into
A~ + U V^T, build M (patterns, column QR, dropping, CSC/CSR assembly), solve
the s+1 systems to the paper's stopping rules, SMW recovery and the FP64
residual check (plus, for the workloads with a loss, the adjoint solve and
the gradients).  value = n / (time per step): SAI columns carried to a 1e-8
solution per second.  The same step with M in FP64 ("plain") is timed after
it.  Before the GPU runs, the FP64 oracle is timed on the host (cpu_baseline).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))

# sources of the Krylov kernels: a stored counter measurement is used only while
# they hash to what was measured
KRYLOV_SOURCES = ("paper_1211_6866_amd/csrc/bicgstab_kernels.hpp", "paper_1211_6866_amd/csrc/krylov.hip")


def counted_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from a committed rocprofv3
    counter summary (profiles/counters_*.md, its json block), or None when there is
    none or the kernel sources changed since it was taken."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in KRYLOV_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    digest = h.hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "counters_*.md"))):
        with open(path) as f:
            m = re.search(r"```json\n(.*?)\n```", f.read(), re.S)
        if not m:
            continue
        info = json.loads(m.group(1))
        if (info.get("kernel") == kernel and info.get("workload") == workload
                and info.get("source_sha256") == digest):
            info["file"] = os.path.relpath(path, ROOT)
            return info
    return None
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector FMA rate without packed instructions (the build disables them)
FP32_VEC_TFLOPS = 78.6
FP64_VEC_TFLOPS = 78.6

# register LS kernel variants in the order the library assigns columns to them
LS_VARIANTS = {
    "f32": [(16, 8, "g16r1j8"), (32, 16, "g16r2j16"), (64, 25, "g16r4j25"), (64, 32, "g16r4j32"),
            (128, 32, "g64r2j32"), (256, 32, "g64r4j32"), (128, 64, "g64r2j64"), (8192, 512, "big")],
}


def workload_settings(P, idx):
    base = dict(pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3)
    solve = dict(method=P.BICGSTAB, eps=1e-8, maxit=500)
    if idx == 1:
        return ("2d5pt_45x45_s3_dense20pct_patternA_gmres30",
                dict(pattern=P.PAT_A, drop=P.DROP_NONE), dict(solve, method=P.GMRES, restart=30), False)
    if idx == 2:
        return "3d7pt_100^3_s10_dense5pct_psai_A2_drop1e-3", base, solve, False
    if idx == 3:
        return ("random_n200000_s20_dense2pct_spai_3x5_delta0.4",
                dict(pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=0.4, spai_steps=3, spai_per_step=5),
                solve, False)
    if idx == 4:
        return "2d5pt_500x500_s8_dense3pct_psai_A2_drop1e-3_adjoint", base, solve, True
    if idx == 5:
        return "3d7pt_160^3_s50_dense1pct_psai_A2_drop1e-3_adjoint", base, solve, True
    raise SystemExit(f"unknown workload {idx}")


def device_copy_gbs(torch, nbytes=1 << 31, reps=5):
    """Bytes read + written per second by a plain device-to-device copy of
    nbytes (torch's copy kernel), the median of reps after one warm-up."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e-3)
    del x, y
    ts.sort()
    return 2.0 * nbytes / ts[len(ts) // 2] / 1e9


def ls_flops(nI, nJ):
    """Householder QR of |I| x |J|, Q^T e and back-substitution."""
    return 2.0 * nJ * nJ * (nI - nJ / 3.0) + 4.0 * nI * nJ - nJ * nJ


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ CPU leg --
# The FP64 oracle, as it stands, on this host.  It runs before anything touches
# the GPU (its process pool forks), and its per-iteration Krylov costs are scaled
# by the GPU's iteration counts once those are known.

def _host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


_ORACLE_JOB = {}


def _oracle_columns(rng_):
    """Oracle column build (pattern, QR, drop) of columns [a, b): the kept rows and values."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import drop as odrop
    from oracle import lsq as olsq
    from oracle import pattern as opat
    from oracle import spai as ospai
    from oracle import psai as opsai
    a, b = rng_
    C, R, cn2, a1, bkw = (_ORACLE_JOB[key] for key in ("C", "R", "cn2", "a1", "bkw"))
    rows, vals, cnt = [], [], np.zeros(b - a, dtype=np.int64)
    with threadpool_limits(1):
        for k in range(a, b):
            if bkw.get("pattern") == 3:
                J, m, _, _ = opsai.psai_tol_column(C, k, bkw["delta"], bkw["psai_lmax"], a1)
            elif bkw.get("pattern") == 2:
                J, _, m, _, _ = ospai.spai_column(C, R, cn2, k, bkw["spai_steps"], bkw["spai_per_step"],
                                                  bkw["delta"])
            else:
                J = opat.pattern_A(C, k) if bkw.get("pattern") == 0 else opat.pattern_A2(C, k)
                _, m, _ = olsq.solve_column(C, J, k)
            if bkw.get("drop") == 1:
                keep = odrop.drop_column(m, bkw["tau"])
                J, m = J[keep], m[keep]
            rows.append(J.astype(np.int32))
            vals.append(m)
            cnt[k - a] = J.size
    return a, np.concatenate(rows), np.concatenate(vals), cnt


def cpu_baseline(w, bkw, adjoint, workers, dense_cols=None, gmres_m=None):
    """Time the oracle on this host: its split of the full matrix, its build of
    the whole M (columns in chunks over a fork pool of `workers` processes), and
    two BiCGStab iterations with its own M on two right-hand sides (and on the
    transposed system for the adjoint), whose per-iteration cost is scaled later
    by the iteration counts of the GPU solve.  For GMRES(m) (gmres_m) the
    per-iteration cost is the average over one full cycle of m steps."""
    import multiprocessing as mp

    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import drop as odrop
    from oracle import krylov as okry
    from oracle import pattern as opat
    from oracle import smw as osmw
    from oracle import spai as ospai
    from oracle import split as osplit

    n = w.A.shape[0]
    out = {}
    with threadpool_limits(1):
        t0 = time.perf_counter()
        S = osplit.split(w.A, dense_cols=dense_cols)
        out["split_s"] = time.perf_counter() - t0
    C = opat.as_csc(S.At)
    R = sp.csr_matrix(S.At)
    R.sort_indices()
    _ORACLE_JOB.update(C=C, R=R, cn2=ospai.column_norms2(C) if bkw.get("pattern") == 2 else None,
                       a1=odrop.norm1(C) if bkw.get("pattern") == 3 else None, bkw=bkw)
    chunk = max(1, min(65536, -(-n // (8 * workers))))
    ranges = [(a, min(n, a + chunk)) for a in range(0, n, chunk)]
    t0 = time.perf_counter()
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        parts = sorted(pool.imap_unordered(_oracle_columns, ranges), key=lambda t: t[0])
    out["build_s"] = time.perf_counter() - t0
    _ORACLE_JOB.clear()
    cnt = np.concatenate([p[3] for p in parts])
    cp = np.concatenate([[0], np.cumsum(cnt)])
    M = sp.csc_matrix((np.concatenate([p[2] for p in parts]), np.concatenate([p[1] for p in parts]), cp),
                      shape=(n, n))
    del parts
    out["nnz_M"] = int(M.nnz)
    Mr, At = sp.csr_matrix(M), sp.csr_matrix(S.At)
    rhs = [w.b] + ([S.U[:, 0].toarray().ravel()] if S.s else [])
    with threadpool_limits(1):
        its = gmres_m or 2

        def kry(Aop, Mop, c):
            if gmres_m:
                okry.gmres(Aop, Mop, c, 0.0, restart=gmres_m, maxit=gmres_m)
            else:
                okry.bicgstab(Aop, Mop, c, 0.0, maxit=2)
        out["krylov"] = f"GMRES({gmres_m})" if gmres_m else "BiCGStab"
        out["krylov_its"] = its
        t0 = time.perf_counter()
        for c in rhs:
            kry(At, Mr, c)
        out["iter_s"] = (time.perf_counter() - t0) / (its * len(rhs))
        if adjoint:
            AtT, MT = sp.csr_matrix(S.At.T), sp.csr_matrix(M.T)
            t0 = time.perf_counter()
            kry(AtT, MT, w.b)
            out["iter_adj_s"] = (time.perf_counter() - t0) / its
        Y = np.zeros((n, S.s + 1))
        Y[:, 0] = w.b
        t0 = time.perf_counter()
        x, _, _ = osmw.recover(Y[:, 0], Y[:, 1:], S.D)
        osmw.relres(w.A, x, w.b)
        out["smw_s"] = time.perf_counter() - t0
    return out


def cpu_m_error(w, bkw, arr, count=64, dense_cols=None):
    """Worst relative error, over a seeded sample of columns (the irregular
    columns, the first and the last included), of the FP32 M's columns m_k before
    dropping against the FP64 oracle's solve on the same pattern."""
    import numpy as np

    from oracle import lsq as olsq
    from oracle import pattern as opat
    from oracle import split as osplit
    S = osplit.split(w.A, dense_cols=dense_cols)
    C = opat.as_csc(S.At)
    n = w.A.shape[0]
    jp, ji = arr["j_ptr"].cpu().numpy(), arr["j_idx"].cpu().numpy()
    mf = arr["m_full"].cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(12116866)
    cols = sorted(set(rng.choice(n, size=min(count, n), replace=False).tolist())
                  | set(int(j) for j in S.D) | {0, n - 1})
    errs = []
    for k in cols:
        J = ji[jp[k]:jp[k + 1]]
        _, m, _ = olsq.solve_column(C, J, k)
        errs.append(float(np.linalg.norm(mf[jp[k]:jp[k + 1]] - m) / np.linalg.norm(m)))
    errs = np.asarray(errs)
    return dict(worst=float(errs.max()), median=float(np.median(errs)), columns=len(cols),
                reference="FP64 oracle column solve on the same J_k")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16)
    ap.add_argument("--approach", choices=("N", "S"), default="N",
                    help="N: split A = A~ + U V^T (the method); S: the standard approach, M built "
                         "on A itself and one system solved (no split), for comparison")
    ap.add_argument("--pattern", choices=("default", "spai", "psai_tol"), default="default",
                    help="override the workload's pattern: SPAI (delta 0.4, 3 x 5) or PSAI(tol) "
                         "(delta 0.4, l_max 10)")
    ap.add_argument("--n", type=int, default=None, help="size of the random workload (3)")
    ap.add_argument("--method", choices=("default", "bicgstab", "gmres"), default="default",
                    help="override the workload's Krylov method (GMRES: restart --restart)")
    ap.add_argument("--restart", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: --gpus must be 1 (the path shards by "
                                   "columns and right-hand sides, but no multi-GPU code is built)"}))
        sys.exit(2)

    import numpy as np

    import paper_1211_6866_amd as P
    import workloads as W

    name, bkw, skw, adjoint = workload_settings(P, args.workload)
    if args.pattern == "spai":
        bkw = dict(pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=0.4, spai_steps=3, spai_per_step=5)
        name += "_spai3x5"
    elif args.pattern == "psai_tol":
        bkw = dict(pattern=P.PAT_PSAI_TOL, delta=0.4, psai_lmax=10)
        name += "_psaitol0.4"
    if args.n is not None:
        name += f"_n{args.n}"
    if args.method == "gmres" and not (skw["method"] == P.GMRES and skw.get("restart") == args.restart):
        skw = dict(skw, method=P.GMRES, restart=args.restart)
        name += f"_gmres{args.restart}"
    elif args.method == "bicgstab" and skw["method"] != P.BICGSTAB:
        skw = dict(skw, method=P.BICGSTAB)
        name += "_bicgstab"
    gmres_m = skw.get("restart") if skw["method"] == P.GMRES else None
    split_kw = {}
    if args.approach == "S":
        # the standard approach: no irregular column is split off (A~ = A, s = 0)
        split_kw = dict(dense_cols=[])
        name += "_standard"
    log(f"bench: generating workload {args.workload} ({name})")
    w = W.make(args.workload, n=args.n) if args.n is not None else W.make(args.workload)
    n = w.A.shape[0]

    # the CPU oracle leg first: its process pool forks before anything touches the GPU
    cpu_raw = None
    model, ncpu, avail = _host_cpu()
    workers = max(1, min(args.cpu_workers, avail))
    if not args.no_cpu:
        log(f"bench: CPU oracle leg ({workers} processes for the build, {model}, {ncpu} CPUs)")
        cpu_raw = cpu_baseline(w, bkw, adjoint, workers, dense_cols=split_kw.get("dense_cols"),
                               gmres_m=gmres_m)
        log(f"bench: CPU oracle leg done: split {cpu_raw['split_s']:.1f} s, build {cpu_raw['build_s']:.1f} s, "
            f"{cpu_raw['iter_s'] * 1e3:.0f} ms per {cpu_raw['krylov']} iteration and right-hand side")

    import torch
    rp, ci, va = P.csr_to_device(w.A)
    # the autotuner's choices for this workload class (bucket edges, launch knobs)
    P.lib()
    tuned = P.load_tuning(workload=name) if os.environ.get("SAI_TUNING", "on") != "off" else None
    tuning = dict(knobs=tuned, record=P.tuning_record(name)) if tuned is not None else None
    b = torch.from_numpy(w.b).cuda()
    xstar = torch.from_numpy(W.x_star(n, w.seed)).cuda() if adjoint else None

    def step(prec):
        sp_ = P.Split(rp, ci, va, **split_kw)
        pc = P.Precond(sp_, precision=prec, **bkw)
        bst = None
        if adjoint:
            # the forward keeps [y, W]; the adjoint reuses W (sai_backward_y)
            x, Y, st = P.solve_y(sp_, pc, b, **skw)
            gb, ga, bst = P.backward_y(sp_, pc, x, Y, x - xstar, **skw)
            del Y
        else:
            x, st = P.solve(sp_, pc, b, **skw)
        return sp_, pc, x, st, bst

    try:
        for i in range(args.warmup):
            log(f"bench: warmup {i}")
            step(P.FP32)
        if args.warmup == 0:
            step(P.FP32)
    except P.SaiError as e:
        # a configuration the library refuses (e.g. the standard approach past its
        # size limits) is reported, not timed
        print(json.dumps({"metric": "SAI columns/s (whole SMW-split path to a 1e-8 residual, s+1 RHS)",
                          "value": None, "config": {"workload": name, "n": n},
                          "error": {"code": e.code, "message": str(e)}}), flush=True)
        return

    # one untimed mixed step with events around every kernel: the full table, and
    # the dominant kernel (the largest total among single kernels on the full-width
    # block; scopes that cover several launches, like "split" or "spai_search", are
    # listed but not chosen)
    log("bench: one step with events around every kernel")
    P.profile_enable(1)
    step(P.FP32)
    prof_all = P.profile_read()
    P.profile_enable(0)
    scopes = {"split", "smw_recover", "spai_search", "psai_search", "gmres_fused", "pattern_bounds",
              "pattern_fill", "pattern_pack", "bicg_init", "gmres_init", "gmres_orth", "gmres_step",
              "adjoint_correction", "adjoint_residual",
              "gmres_cycle_start", "gmres_cycle_end"}
    # launches on a narrowed BiCGStab block (names with "narrow") and those of the adjoint's transposed
    # solves (names with "_t_", one column) are left out: their bytes per launch do not follow from k
    dom = max((tot, nm) for nm, (l, tot) in prof_all.items()
              if nm not in scopes and "narrow" not in nm and "_t_" not in nm)[1]

    def timed(prec, K, only=None):
        torch.cuda.synchronize()
        if only:
            P.profile_enable(only=only)  # events only around the dominant kernel
        t0 = time.perf_counter()
        last = None
        builds, solves, backs = [], [], []
        for i in range(K):
            last = step(prec)
            builds.append(last[1].stats.t_total_ms)
            solves.append(last[3]["t_solve_ms"])
            if last[4] is not None:
                backs.append(last[4]["t_solve_ms"] + last[4]["t_smw_ms"] + last[4]["t_check_ms"])
            log(f"bench: step {i + 1}/{K} done")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = P.profile_read() if only else {}
        P.profile_enable(False)
        return (t1 - t0) / K * 1e3, last, prof, builds, solves, backs

    log(f"bench: timing {args.steps} mixed steps (events around {dom})")
    ms_mixed, (sp_m, pc_m, x_m, st_m, bst_m), prof, builds_m, solves_m, backs_m = timed(P.FP32, args.steps,
                                                                                      only=dom)
    kplain = args.plain_steps if args.plain_steps is not None else max(1, args.steps // 2)
    plain = None
    if kplain > 0:
        log(f"bench: timing {kplain} plain FP64 steps")
        # the same event overhead as the mixed steps: around the plain form of that kernel
        dom_p = dom.replace("_f32", "_f64")
        ms_plain, (sp_p, pc_p, x_p, st_p, bst_p), _, builds_p, solves_p, backs_p = timed(P.FP64, kplain,
                                                                                       only=dom_p)
        xhp = x_p.cpu().numpy()
        plain = dict(ms=ms_plain, build=float(np.mean(builds_p)), st=st_p,
                     rr_host=float(np.linalg.norm(w.b - w.A @ xhp) / np.linalg.norm(w.b)),
                     adjoint=float(np.mean(backs_p)) if backs_p else None)

    xh = x_m.cpu().numpy()
    rr_host = float(np.linalg.norm(w.b - w.A @ xh) / np.linalg.norm(w.b))
    adj_cmp = None
    if adjoint:
        # the other adjoint form once, for comparison (not in the step): s+1 systems
        # with A~^T (sai_backward), each residual recomputed on the host
        log("bench: the adjoint through s+1 transposed systems, once, for comparison")
        gv = (x_m - xstar).cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gb_t, _, bst_t = P.backward(sp_m, pc_m, x_m, x_m - xstar, want_a=False, **skw)
        torch.cuda.synchronize()
        ms_t = (time.perf_counter() - t0) * 1e3
        gb_y, _, bst_y = P.backward_y(sp_m, pc_m, x_m, P.solve_y(sp_m, pc_m, b, **skw)[1], x_m - xstar,
                                      want_a=False, **skw)
        gn = float(np.linalg.norm(gv))
        adj_cmp = dict(
            form="from the forward's W: one system with A~^T per correction pass (sai_backward_y)",
            rr_host=float(np.linalg.norm(gv - w.A.T @ gb_y.cpu().numpy()) / gn),
            column_iters=int(np.sum(bst_y["iters"])),
            transposed_split=dict(ms=round(ms_t, 3), column_iters=int(np.sum(bst_t["iters"])),
                                  rr_host=float(np.linalg.norm(gv - w.A.T @ gb_t.cpu().numpy()) / gn)))
        del gb_t, gb_y
    copy_gbs = device_copy_gbs(torch)

    # algorithmic work per kernel, for the roofline of the dominant one
    s = sp_m.s
    k = s + 1
    nnz_t = sp_m.info.nnz_t
    nnz_m = pc_m.stats.nnz_m
    pc_l = P.Precond(sp_m, precision=P.FP32, keep_lists=True, **bkw)
    arr = pc_l.arrays()
    nJ = np.diff(arr["j_ptr"].cpu().numpy())
    nI = np.diff(arr["i_ptr"].cpu().numpy())
    # the gather step on its own (sai_gather of the mixed build's blocks, float32):
    # algorithmic bytes = list offsets 24 n + J_k and I_k 4 (sum |J| + sum |I|) +
    # column pointers 8 sum |J| + gathered CSC entries 12 sum_k sum_{j in J_k} nnz(A~(:, j))
    # + blocks written 4 sum |I||J|
    gather = None
    try:
        log("bench: standalone gather of A~(I_k, J_k)")
        goff, gblk = P.gather(sp_m, pc_l, precision=P.FP32)
        P.profile_enable(only="gather")
        for _ in range(3):
            P.gather(sp_m, pc_l, precision=P.FP32, blk_off=goff, out=gblk)
        gl, gms = P.profile_read()["gather_f32"]
        P.profile_enable(False)
        del goff, gblk
        colnnz = np.diff(sp_m.arrays()["t_col_ptr"].cpu().numpy()).astype(np.int64)
        gathered = float(colnnz[arr["j_idx"].cpu().numpy()].sum())
        gbytes = (24.0 * n + 12.0 * nJ.sum() + 4.0 * nI.sum() + 12.0 * gathered
                  + 4.0 * float(np.sum(nJ.astype(np.float64) * nI)))
        gavg = gms / gl
        gather = dict(kernel="gather_f32", avg_launch_ms=round(gavg, 4), algorithmic_bytes=gbytes,
                      frac_of_copy=round(gbytes / (gavg * 1e-3) / 1e9 / copy_gbs, 4) if copy_gbs else None,
                      achieved_GBs=round(gbytes / (gavg * 1e-3) / 1e9, 1),
                      frac=round(gbytes / (gavg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      gathered_entries=int(gathered), block_elements=int(np.sum(nJ.astype(np.int64) * nI)))
    except Exception as e:  # noqa: BLE001 - reported, the step results stand
        gather = dict(error=str(e))
    m_err = None
    if not args.no_cpu:
        log("bench: FP32 M against the FP64 oracle on sampled columns")
        m_err = None if bkw.get("pattern") == P.PAT_PSAI_TOL else cpu_m_error(
            w, bkw, arr, dense_cols=split_kw.get("dense_cols"))
    del pc_l, arr
    flops = ls_flops(nI.astype(np.float64), nJ.astype(np.float64))
    ls_work = {}
    assigned = np.zeros(n, dtype=bool)
    for v, (maxI, maxJ, tag) in enumerate(LS_VARIANTS["f32"]):
        if v < len(LS_VARIANTS["f32"]) - 1:  # the bucket edges in effect (autotuned knobs)
            maxI = P.tune_get(f"LSB_F32_{v}_I", maxI)
            maxJ = P.tune_get(f"LSB_F32_{v}_J", maxJ)
        sel = (~assigned) & (nI <= maxI) & (nJ <= maxJ)
        assigned |= sel
        ls_work["ls_qr_f32_" + tag] = float(flops[sel].sum())
    bytes_kn = 8.0 * k * n
    hbm_bytes = {
        "bicg_spmm_M_f32": 8.0 * nnz_m + 4.0 * (n + 1) + 2 * bytes_kn,
        "bicg_spmm_A_dot1": 12.0 * nnz_t + 4.0 * (n + 1) + 3 * bytes_kn,
        "bicg_spmm_A_dot2": 12.0 * nnz_t + 4.0 * (n + 1) + 3 * bytes_kn,
        "bicg_p_update": 4 * bytes_kn,
        "bicg_s_update": 3 * bytes_kn,
        "bicg_xr_update": 8 * bytes_kn,
        "gmres_spmm_M_f32": 8.0 * nnz_m + 4.0 * (n + 1) + 2 * bytes_kn,
        "gmres_spmm_A": 12.0 * nnz_t + 4.0 * (n + 1) + 2 * bytes_kn,
    }
    dom_launches, dom_ms = prof[dom]
    avg_ms = dom_ms / dom_launches
    if dom.startswith("ls_qr_f32"):
        # FP32 vector FMA without packed instructions (the build disables them):
        # 256 CUs x 64 lanes x 2 flops x 2.4 GHz
        ach = ls_work.get(dom, 0.0) / (avg_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=round(ach, 3), peak=FP32_VEC_TFLOPS, unit="TFLOP/s",
                    frac=round(ach / FP32_VEC_TFLOPS, 4), traffic=None)
    elif dom in hbm_bytes:
        ach = hbm_bytes[dom] / (avg_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=None)
    else:
        roof = dict(bound="latency", achieved=None, peak=None, unit=None, frac=None, traffic=None)
    roof["kernel"] = dom
    roof["avg_launch_ms"] = round(avg_ms, 4)
    if copy_gbs and roof.get("bound") == "hbm":
        # against what a plain device copy reaches on this GPU
        roof["measured_copy_GBs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    roof["launches_per_step"] = dom_launches / args.steps
    if dom in hbm_bytes:
        roof["algorithmic_bytes_per_launch"] = hbm_bytes[dom]
    counted = counted_traffic(dom, name)
    if counted is not None:
        roof["traffic"] = counted["traffic_bytes_per_launch"]
        roof["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roof["traffic_source"] = counted["file"]

    kern_table = {nm: dict(launches=l, total_ms=round(t, 3), avg_ms=round(t / l, 4))
                  for t, nm, l in sorted(((tot, nm, l) for nm, (l, tot) in prof_all.items()),
                                         reverse=True)}
    for nm, wb in hbm_bytes.items():
        if nm in kern_table:
            kern_table[nm]["GB/s"] = round(wb / (kern_table[nm]["avg_ms"] * 1e-3) / 1e9, 1)
    for nm, wf in ls_work.items():
        if nm in kern_table and wf > 0:
            kern_table[nm]["TFLOP/s"] = round(wf / (kern_table[nm]["avg_ms"] * 1e-3) / 1e12, 2)

    cpu = None
    if cpu_raw is not None:
        it_fwd = int(np.sum(st_m["iters"]))
        it_adj = int(np.sum(bst_m["iters"])) if bst_m is not None else 0
        t_kry = cpu_raw["iter_s"] * it_fwd + cpu_raw.get("iter_adj_s", 0.0) * it_adj
        est = cpu_raw["split_s"] + cpu_raw["build_s"] + t_kry + cpu_raw["smw_s"]
        cpu = dict(
            value=round(n / est, 1), unit="columns/s", cores=workers, kind="oracle",
            cpu_model=model, nproc=ncpu,
            sample=(f"oracle split of the full matrix ({cpu_raw['split_s']:.1f} s, 1 thread); oracle build of "
                    f"all {n} columns of M ({cpu_raw['nnz_M']} entries) on {workers} processes "
                    f"({cpu_raw['build_s']:.1f} s); oracle {cpu_raw['krylov']} with that M: "
                    f"{cpu_raw['krylov_its']} iterations on 2 "
                    f"right-hand sides ({cpu_raw['iter_s'] * 1e3:.0f} ms per iteration and right-hand side, "
                    f"1 thread) scaled by the GPU solve's {it_fwd} column-iterations"
                    + (f", and on the transposed system ({cpu_raw['iter_adj_s'] * 1e3:.0f} ms) scaled by "
                       f"the adjoint's {it_adj}" if adjoint else "")
                    + f" ({t_kry:.0f} s extrapolated); SMW and residual check ({cpu_raw['smw_s']:.2f} s)"),
            est_seconds=round(est, 2))

    value = n / (ms_mixed * 1e-3)
    out = {
        "metric": "SAI columns/s (whole SMW-split path to a 1e-8 residual, s+1 RHS)",
        "value": round(value, 1),
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_mixed, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 M build + f64 Krylov/SMW/check",
        "data": "synthetic",
        "config": {"workload": name, "n": n, "s": s, "nnz_A": int(w.A.nnz), "rhs": k,
                   "solver": f"gmres{skw['restart']}" if skw["method"] == P.GMRES else "bicgstab",
                   "eps": skw["eps"],
                   "adjoint_in_step": adjoint, "parallelism": "single GPU"},
        "time_to_1e-8_ms": {"mixed": round(ms_mixed, 3),
                            "plain_fp64": round(plain["ms"], 3) if plain else None},
        # the forward path alone (split, build, solve, SMW, check): the step less its adjoint
        "forward_ms": {"mixed": round(ms_mixed - (float(np.mean(backs_m)) if backs_m else 0.0), 3),
                       "plain_fp64": (round(plain["ms"] - (plain["adjoint"] or 0.0), 3) if plain else None)},
        "build_ms": {"mixed": round(float(np.mean(builds_m)), 3),
                     "plain_fp64": round(plain["build"], 3) if plain else None},
        "build_columns_per_s": {"mixed": round(n / (np.mean(builds_m) * 1e-3), 1),
                                "plain_fp64": round(n / (plain["build"] * 1e-3), 1) if plain else None},
        "solve_ms": round(float(np.mean(solves_m)), 3),
        "adjoint_ms": {"mixed": round(float(np.mean(backs_m)), 3) if backs_m else None,
                       "plain_fp64": round(plain["adjoint"], 3) if plain and plain["adjoint"] else None},
        "adjoint": adj_cmp,
        "solve": {"mixed": {"iters": st_m["iters"], "rr": st_m["rr"], "rr_host": rr_host,
                            "c": st_m["c"],
                            "adjoint_iters": bst_m["iters"] if bst_m is not None else None},
                  "plain_fp64": ({"iters": plain["st"]["iters"], "rr": plain["st"]["rr"],
                                  "rr_host": plain["rr_host"]} if plain else None)},
        "M": {"nnz": int(nnz_m), "spar": round(pc_m.stats.spar, 4), "max_I": pc_m.stats.max_i,
              "max_J": pc_m.stats.max_j, "n_c": pc_m.stats.n_c, "l_m": pc_m.stats.l_m,
              "s": pc_m.stats.s, "p": pc_m.stats.p, "drop_undecidable_fp32": int(pc_m.stats.drop_flips),
              "fp32_vs_fp64_oracle": m_err},
        "roofline": roof,
        "tuning": tuning,
        "gather": gather,
        "kernels_one_step": kern_table,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
