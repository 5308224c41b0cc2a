"""Autotuner for the library's bucket edges and launch-shape knobs (sai_tune_set, SAI_TUNE_<name>).

    python -m paper_1211_6866_amd.autotune [--workload 2] [--reps 3] [--out PATH]

Run from the repository root (it builds the synthetic workloads of the
``workloads`` package).  Two searches, each keeping a change only when it beats
the current setting by more than ``--margin``:

* bucket edges of the column solver (knobs LSB_F32_<v>_I / _J): a column goes
  to the first register variant whose edges hold its |I| and |J|; each variant
  in turn is tried disabled (its columns then go to the next variant that
  holds them), timed on the column solves of whole builds (the median of
  ``reps`` after one warm-up);
* launch knobs of the Krylov solve, by coordinate descent: each knob in turn
  takes every candidate value while the others keep their current best, timed
  on whole steps (split, build, BiCGStab to 1e-8, SMW recovery, and for the
  workloads with a loss the adjoint from the forward's W).

The choices are stored per workload class (the benchmark's workload name) in
tuning/<device>.json (architecture and CU count), with the default and tuned
times; the benchmark loads its class's section before timing.  The knobs change
speed only; every setting gives deterministic results.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

# knob -> candidate values, the built-in default first
KNOBS_SOLVE = [
    ("SPMM_M", [1, 0, 2, 3, 4]),       # M product gather batches: 6/3, 8/4, 5/0, 16/8, 2/0
    ("SPMM_A", [0, 1, 2, 3, 4, 5]),    # A~ products: 4/2, 8/4, 7/0 (LDS-staged tiles); 8/4, 7/0 (no staging); 2/0
    ("SPMM_M_WIDE", [4, 0, 1]),        # the same for blocks over 32 columns: 2/0, 8/4, 6/3
    ("SPMM_A_WIDE", [5, 0, 1]),        # 2/0, 4/2, 8/4
    ("SGRID", [512, 1024, 256]),       # workgroups of the streaming updates
    ("LP_MIN", [1, 2]),                # smallest lane class (one-column blocks on tiles of 128 rows)
    ("SPMM_M_LP2", [1, 0]),            # one-column blocks: the M product alone on two lanes per row
    ("NT_STORE", [-1, 0, 1]),          # output blocks stored non-temporally: by size, never, always
    ("NT_LOAD", [0, 1]),               # streamed block reads non-temporal
    ("NARROW", [1, 0]),                # narrowing of the BiCGStab block
    ("NARROW_MIN", [1000000, 500000, 2000000, 8000000]),
]
KNOBS_SPAI = [
    ("SPAI_NT", [512, 256, 1024]),     # threads per column of the SPAI search
]
# register variants of the float column solver (|I|, |J| capacities, in the
# library's order; the global-memory variant after them is never disabled)
LS_F32 = [(16, 8), (32, 16), (64, 25), (64, 32), (128, 32), (256, 32), (128, 64)]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--margin", type=float, default=0.01, help="relative gain needed to change a knob")
    ap.add_argument("--out", default=None)
    ap.add_argument("--skip-solve", action="store_true", help="tune the bucket edges only")
    args = ap.parse_args(argv)

    import torch
    import paper_1211_6866_amd as P
    import workloads as W
    sys.path.insert(0, os.getcwd())
    from bench import workload_settings

    os.environ["SAI_TUNING"] = "off"  # start from the built-in defaults
    name, bkw, skw, adjoint = workload_settings(P, args.workload)
    if skw.get("method") != P.BICGSTAB:
        raise SystemExit("the autotuner covers the BiCGStab workloads (2-5)")
    w = W.make(args.workload)
    rp, ci, va = P.csr_to_device(w.A)
    b = torch.from_numpy(w.b).cuda()
    P.lib()
    P.tune_clear()

    def build_ls():
        sp_ = P.Split(rp, ci, va)
        pc = P.Precond(sp_, precision=P.FP32, **bkw)
        return pc.stats.t_ls_ms

    xstar = torch.from_numpy(W.x_star(w.A.shape[0], w.seed)).cuda() if adjoint else None

    def step():
        # the benchmark's step: with a loss, the adjoint from the forward's W too
        sp_ = P.Split(rp, ci, va)
        pc = P.Precond(sp_, precision=P.FP32, **bkw)
        if adjoint:
            x, Y, _ = P.solve_y(sp_, pc, b, **skw)
            P.backward_y(sp_, pc, x, Y, x - xstar, **skw)
        else:
            P.solve(sp_, pc, b, **skw)

    def timed(f):
        f()
        ts = []
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = f()
            torch.cuda.synchronize()
            ts.append(r if r is not None else (time.perf_counter() - t0) * 1e3)
        return statistics.median(ts)

    chosen = {}
    step_default = timed(step)  # every knob at its built-in default
    print(f"autotune: {name}: {step_default:.2f} ms per step with the built-in defaults", flush=True)
    # ---- bucket edges (float column solver)
    ls_default = timed(build_ls)
    ls_best = ls_default
    print(f"autotune: {name}: column solves {ls_default:.3f} ms with the default edges", flush=True)
    for v, (ci_, cj_) in enumerate(LS_F32):
        kn = f"LSB_F32_{v}_I"
        P.tune_set(kn, 0)
        ms = timed(build_ls)
        print(f"autotune: variant {v} ({ci_} x {cj_}) disabled: {ms:.3f} ms (current {ls_best:.3f})",
              flush=True)
        if ms < ls_best * (1.0 - args.margin):
            ls_best = ms
            chosen[kn] = 0
        else:
            P.tune_set(kn, ci_)
    # ---- Krylov launch knobs
    base = step_default
    if not args.skip_solve:
        knobs = KNOBS_SOLVE + (KNOBS_SPAI if bkw.get("pattern") == P.PAT_SPAI else [])
        s = P.Split(rp, ci, va).s
        if w.A.shape[0] * 8 * (s + 2) > (256 << 20):
            # the tile-to-XCD map of blocks larger than the MALL
            knobs = knobs + [("XCHUNK", [0, 3200, 12800])]
        best = {kname: vals[0] for kname, vals in knobs}
        for kname, v in best.items():
            P.tune_set(kname, v)
        base = timed(step)
        print(f"autotune: {name}: {base:.2f} ms per step (tuned edges, default launch knobs)", flush=True)
        for kname, vals in knobs:
            cur, cur_ms = best[kname], base
            for v in vals:
                if v == cur:
                    continue
                P.tune_set(kname, v)
                ms = timed(step)
                print(f"autotune: {kname}={v}: {ms:.2f} ms (current {kname}={cur}: {cur_ms:.2f})", flush=True)
                if ms < cur_ms * (1.0 - args.margin):
                    cur, cur_ms = v, ms
            best[kname] = cur
            base = cur_ms
            P.tune_set(kname, cur)
            if cur != vals[0]:
                chosen[kname] = cur
    out = args.out or os.path.join(P.TUNING_DIR, P.device_key() + ".json")
    rec = {}
    if os.path.exists(out):
        with open(out) as f:
            rec = json.load(f)
    rec.setdefault("device", P.device_key())
    rec.setdefault("knobs", {})
    rec.setdefault("classes", {})
    rec["classes"][name] = dict(knobs=chosen, column_solves_ms=dict(default=round(ls_default, 3),
                                                                    tuned=round(ls_best, 3)),
                                step_ms=dict(default=round(step_default, 3), tuned=round(base, 3)))
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"autotune: {name}: {json.dumps(rec['classes'][name])} -> {out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
