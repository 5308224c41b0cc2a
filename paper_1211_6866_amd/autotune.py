"""Autotuner for the library's launch-shape knobs (sai_tune_set, SAI_TUNE_<name>).

    python -m paper_1211_6866_amd.autotune [--workload 2] [--reps 3] [--out PATH]

Run from the repository root (it builds the synthetic workloads of the
``workloads`` package).  Coordinate descent over the knobs: each knob in turn
takes every candidate value while the others keep their current best, and is
timed on whole steps of the workload (split, build, BiCGStab to 1e-8, SMW
recovery), the median of ``reps`` after one warm-up; the fastest value is kept
when it beats the current one by more than ``--margin``.  The choices are
written to tuning/<device>.json (architecture and CU count), which the binding
passes to the library when it is first used on that device.

The knobs change speed only; every setting gives deterministic results.  Knobs
whose best value depends on the problem size (the XCD tile mapping, derived from
the block size, and the persistent grids) are left to their built-in rules.
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
    ("SPMM_M", [1, 0, 2, 3]),          # M product gather batches: 6/3, 8/4, 5/0, 16/8
    ("SPMM_A", [0, 1, 2]),             # A~ products: 4/2, 8/4, 7/0
    ("SGRID", [512, 1024, 256]),       # workgroups of the streaming updates
    ("NARROW", [1, 0]),                # narrowing of the BiCGStab block
    ("NARROW_MIN", [1000000, 500000, 2000000, 8000000]),
]
KNOBS_SPAI = [
    ("SPAI_NT", [512, 256, 1024]),     # threads per column of the SPAI search
]


def settings(P, idx):
    """Build and solve options of the BiCGStab workloads (as the benchmark uses them)."""
    solve = dict(method=P.BICGSTAB, eps=1e-8, maxit=500)
    psai = dict(pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3)
    if idx in (2, 4, 5):
        return psai, solve
    if idx == 3:
        return dict(pattern=P.PAT_SPAI, drop=P.DROP_NONE, delta=0.4, spai_steps=3, spai_per_step=5), solve
    raise SystemExit(f"workload {idx}: the autotuner covers the BiCGStab workloads 2-5")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--margin", type=float, default=0.01, help="relative gain needed to change a knob")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch
    import paper_1211_6866_amd as P
    import workloads as W

    os.environ["SAI_TUNING"] = "off"  # start from the built-in defaults
    bkw, skw = settings(P, args.workload)
    w = W.make(args.workload)
    rp, ci, va = P.csr_to_device(w.A)
    b = torch.from_numpy(w.b).cuda()
    P.lib()
    P.tune_clear()

    def step():
        sp_ = P.Split(rp, ci, va)
        pc = P.Precond(sp_, precision=P.FP32, **bkw)
        x, st = P.solve(sp_, pc, b, **skw)
        return st

    def timed():
        step()
        ts = []
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return statistics.median(ts)

    knobs = KNOBS_SOLVE + (KNOBS_SPAI if bkw.get("pattern") == P.PAT_SPAI else [])
    best = {name: vals[0] for name, vals in knobs}
    for name, v in best.items():
        P.tune_set(name, v)
    base = timed()
    print(f"autotune: workload {args.workload}, defaults {base:.2f} ms per step", flush=True)
    for name, vals in knobs:
        cur = best[name]
        cur_ms = base
        for v in vals:
            if v == cur:
                continue
            P.tune_set(name, v)
            ms = timed()
            print(f"autotune: {name}={v}: {ms:.2f} ms (current {name}={cur}: {cur_ms:.2f})", flush=True)
            if ms < cur_ms * (1.0 - args.margin):
                cur, cur_ms = v, ms
        best[name] = cur
        base = cur_ms
        P.tune_set(name, cur)
    out = args.out or os.path.join(P.TUNING_DIR, P.device_key() + ".json")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    rec = dict(device=P.device_key(), workload=args.workload, step_ms=round(base, 3),
               knobs={k: v for k, v in best.items() if v != dict(knobs)[k][0]})
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"autotune: {json.dumps(rec)} -> {out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
