"""Python binding of libsai, the gfx950 SMW-split sparse approximate inverse solver.

Argument marshalling only: every step runs in the HIP library declared in
include/sai.h.  PyTorch supplies device memory (through its caching allocator,
passed to the library as an allocator callback) and the current stream.
Importing this package does not load the library; the first call does, and
raises if libsai.so has not been built (python -m paper_1211_6866_amd.build).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsai.so")
TUNING_DIR = os.path.join(_HERE, "tuning")

# status codes (include/sai.h)
OK, EINVAL, EZERODIAG, ESINGULAR, ENOCONV, EBREAKDOWN, ENOMEM, EHIP, ETOOBIG = range(9)
KEEP_NEAREST, KEEP_LARGEST = 0, 1
PAT_A, PAT_A2, PAT_SPAI, PAT_PSAI_TOL = 0, 1, 2, 3
DROP_NONE, DROP_ABS, DROP_TOLK = 0, 1, 2
INIT_PATTERN_A, INIT_DIAG = 0, 1
FP32, FP64 = 0, 1
BICGSTAB, GMRES = 0, 1
C_ONE, C_ONE_THEN_REFINE = 0, 1


class SaiError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


_alloc_fn_t = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_free_fn_t = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _alloc_fn_t), ("free", _free_fn_t), ("ctx", C.c_void_p)]


class SplitOpts(C.Structure):
    _fields_ = [("dense_factor", C.c_double), ("keep", C.c_int32), ("rule", C.c_int32),
                ("host_dense_cols", C.POINTER(C.c_int32)), ("s_given", C.c_int32)]


class SplitInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("s", C.c_int32), ("p", C.c_int32), ("keep", C.c_int32),
                ("nnz_a", C.c_int64), ("nnz_t", C.c_int64), ("nnz_u", C.c_int64),
                ("t_row_ptr", C.c_void_p), ("t_col_idx", C.c_void_p), ("t_val", C.c_void_p),
                ("t_col_ptr", C.c_void_p), ("t_row_idx", C.c_void_p), ("t_cval", C.c_void_p),
                ("dense_cols", C.c_void_p), ("u_row_ptr", C.c_void_p), ("u_col", C.c_void_p),
                ("u_val", C.c_void_p)]


class BuildOpts(C.Structure):
    _fields_ = [("pattern", C.c_int32), ("drop", C.c_int32), ("tau", C.c_double),
                ("delta", C.c_double), ("spai_steps", C.c_int32), ("spai_per_step", C.c_int32),
                ("spai_init", C.c_int32), ("precision", C.c_int32), ("keep_lists", C.c_int32),
                ("psai_lmax", C.c_int32)]


class BuildStats(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz_m", C.c_int64), ("nnz_m_full", C.c_int64),
                ("sum_i", C.c_int64), ("max_i", C.c_int32), ("max_j", C.c_int32),
                ("n_c", C.c_int32), ("spar", C.c_double), ("bucket_cols", C.c_int64 * 16),
                ("t_pattern_ms", C.c_float), ("t_ls_ms", C.c_float), ("t_assemble_ms", C.c_float),
                ("t_total_ms", C.c_float), ("s", C.c_int32), ("p", C.c_int32), ("l_m", C.c_int32),
                ("drop_flips", C.c_int64)]


class PrecondInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("precision", C.c_int32), ("nnz", C.c_int64),
                ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p), ("cval", C.c_void_p),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("j_ptr", C.c_void_p), ("j_idx", C.c_void_p), ("i_ptr", C.c_void_p),
                ("i_idx", C.c_void_p), ("m_full", C.c_void_p), ("res", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("restart", C.c_int32), ("eps", C.c_double),
                ("maxit", C.c_int32), ("c_mode", C.c_int32), ("equilibrate", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("s", C.c_int32), ("status", C.c_int32), ("iters_max", C.c_int32),
                ("iters", C.POINTER(C.c_int32)), ("rr", C.c_double), ("a", C.c_double),
                ("c", C.c_double), ("t_solve_ms", C.c_float), ("t_smw_ms", C.c_float),
                ("t_check_ms", C.c_float)]


_lib = None
_alloc_struct = None
# number of device allocations the library has requested through the binding's
# allocator (for tests of the allocation-free entry point)
ALLOC_CALLS = [0]


def _torch():
    import torch
    return torch


def lib():
    """Load libsai.so (once).  Raises if it is missing: there is no fallback."""
    global _lib, _alloc_struct
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1211_6866_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.sai_split.argtypes = [i32, i64, vp, vp, vp, C.POINTER(SplitOpts), C.POINTER(_Allocator), vp,
                            C.POINTER(vp)]
    L.sai_split_get_info.argtypes = [vp, C.POINTER(SplitInfo)]
    L.sai_split_destroy.argtypes = [vp]
    L.sai_split_destroy.restype = None
    L.sai_build.argtypes = [vp, C.POINTER(BuildOpts), vp, C.POINTER(vp), C.POINTER(BuildStats)]
    L.sai_precond_get_info.argtypes = [vp, C.POINTER(PrecondInfo)]
    L.sai_precond_destroy.argtypes = [vp]
    L.sai_precond_destroy.restype = None
    L.sai_krylov.argtypes = [vp, vp, i32, i32, vp, vp, dp, C.POINTER(SolveOpts), vp,
                             C.POINTER(i32), C.POINTER(i32)]
    L.sai_smw.argtypes = [vp, vp, vp, dp, vp]
    L.sai_smw_noalloc.argtypes = [vp, vp, vp, dp, vp]
    L.sai_gather_offsets.argtypes = [vp, vp, C.POINTER(i64), vp]
    L.sai_gather.argtypes = [vp, vp, i32, vp, vp, vp]
    L.sai_residual.argtypes = [vp, vp, vp, dp, vp]
    L.sai_solve.argtypes = [vp, vp, vp, vp, C.POINTER(SolveOpts), vp, C.POINTER(SolveStats)]
    L.sai_backward.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(SolveOpts), vp,
                               C.POINTER(SolveStats)]
    L.sai_solve_y.argtypes = [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), vp, C.POINTER(SolveStats)]
    L.sai_backward_y.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(SolveOpts), vp,
                                 C.POINTER(SolveStats)]
    L.sai_strerror.restype = C.c_char_p
    L.sai_strerror.argtypes = [C.c_int]
    L.sai_last_error.restype = C.c_char_p
    L.sai_memcpy_d2d.argtypes = [vp, vp, C.c_size_t, vp]
    L.sai_profile_enable.argtypes = [i32]
    L.sai_profile_only.argtypes = [C.c_char_p]
    L.sai_profile_count.argtypes = []
    L.sai_profile_get.argtypes = [i32, C.c_char_p, i32, C.POINTER(i64), C.POINTER(C.c_double)]
    L.sai_tune_set.argtypes = [C.c_char_p, i32]
    L.sai_tune_get.argtypes = [C.c_char_p, i32, C.POINTER(i32)]
    L.sai_tune_clear.argtypes = []

    torch = _torch()

    def _alloc(ctx, nbytes, stream):
        ALLOC_CALLS[0] += 1
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:  # noqa: BLE001 - reported to the library as NULL
            return None

    def _free(ctx, ptr, stream):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)

    _alloc_struct = _Allocator(_alloc_fn_t(_alloc), _free_fn_t(_free), None)
    _lib = L
    if os.environ.get("SAI_TUNING", "on") != "off" and torch.cuda.is_available():
        load_tuning()
    return L


def device_key() -> str:
    """Name of the tuning file of the current device: arch and CU count."""
    p = _torch().cuda.get_device_properties(_torch().cuda.current_device())
    return f"{p.gcnArchName.split(':')[0]}_{p.multi_processor_count}cu"


def tune_set(name: str, value: int):
    """Set a launch-shape knob (sai_tune_set); SAI_TUNE_<name> still overrides."""
    _check(lib().sai_tune_set(name.encode(), int(value)), "sai_tune_set")


def tune_get(name: str, dflt: int = 0) -> int:
    v = C.c_int32()
    _check(lib().sai_tune_get(name.encode(), int(dflt), C.byref(v)), "sai_tune_get")
    return v.value


def tune_clear():
    _check(lib().sai_tune_clear(), "sai_tune_clear")


def load_tuning(path: Optional[str] = None, workload: Optional[str] = None) -> Optional[dict]:
    """Pass the knobs of a tuning file (by default tuning/<device_key()>.json,
    written by the autotuner) to the library: its device-wide knobs and, when
    `workload` names one of its classes, that class's knobs.  Returns the knobs
    set, or None when there is no file."""
    import json
    if path is None:
        path = os.path.join(TUNING_DIR, device_key() + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    knobs = dict(rec.get("knobs", {}))
    if workload is not None:
        knobs.update(rec.get("classes", {}).get(workload, {}).get("knobs", {}))
    for name, value in knobs.items():
        tune_set(name, value)
    return knobs


def tuning_record(workload: str, path: Optional[str] = None) -> Optional[dict]:
    """The autotuner's record for a workload class (knobs, default and tuned times)."""
    import json
    if path is None:
        path = os.path.join(TUNING_DIR, device_key() + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get("classes", {}).get(workload)


def _check(code: int, where: str):
    if code != OK:
        L = lib()
        raise SaiError(code, where, (L.sai_last_error() or L.sai_strerror(code)).decode())


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _export(ptr, count: int, dtype):
    """Copy `count` elements at device address `ptr` into a new torch tensor."""
    torch = _torch()
    out = torch.empty(int(count), dtype=dtype, device="cuda")
    if count:
        nbytes = out.element_size() * int(count)
        _check(lib().sai_memcpy_d2d(_ptr(out), C.c_void_p(ptr), nbytes, _stream()), "export")
    return out


class Split:
    """Handle of A = A~ + U V^T (owns device copies; freed with the object)."""

    def __init__(self, row_ptr, col_idx, val, dense_factor=10.0, keep=0, rule=KEEP_NEAREST,
                 dense_cols=None):
        """dense_cols: optional list of the irregular columns (overrides the count rule)."""
        torch = _torch()
        L = lib()
        assert row_ptr.dtype == torch.int32 and col_idx.dtype == torch.int32
        assert val.dtype == torch.float64 and row_ptr.is_cuda
        self.n = int(row_ptr.numel() - 1)
        self.nnz = int(col_idx.numel())
        h = C.c_void_p()
        o = SplitOpts(float(dense_factor), int(keep), int(rule))
        if dense_cols is not None:
            dl = [int(j) for j in dense_cols]
            self._dense_arr = (C.c_int32 * max(1, len(dl)))(*dl)
            o.host_dense_cols = C.cast(self._dense_arr, C.POINTER(C.c_int32))
            o.s_given = len(dl)
        _check(L.sai_split(self.n, self.nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(val), C.byref(o),
                           C.byref(_alloc_struct), _stream(), C.byref(h)), "sai_split")
        self.h = h
        self.info = SplitInfo()
        _check(L.sai_split_get_info(h, C.byref(self.info)), "sai_split_get_info")
        self.s, self.p = self.info.s, self.info.p

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sai_split_destroy(self.h)
            self.h = None

    def arrays(self):
        """Export A~ (CSR, CSC), U (row CSR) and the irregular columns as torch tensors."""
        torch = _torch()
        i = self.info
        n, nt, nu, s = i.n, i.nnz_t, i.nnz_u, i.s
        return dict(
            t_row_ptr=_export(i.t_row_ptr, n + 1, torch.int32),
            t_col_idx=_export(i.t_col_idx, nt, torch.int32),
            t_val=_export(i.t_val, nt, torch.float64),
            t_col_ptr=_export(i.t_col_ptr, n + 1, torch.int32),
            t_row_idx=_export(i.t_row_idx, nt, torch.int32),
            t_cval=_export(i.t_cval, nt, torch.float64),
            dense_cols=_export(i.dense_cols, s, torch.int32),
            u_row_ptr=_export(i.u_row_ptr, n + 1, torch.int32),
            u_col=_export(i.u_col, nu, torch.int32),
            u_val=_export(i.u_val, nu, torch.float64),
        )


class Precond:
    """Handle of M (CSC and CSR)."""

    def __init__(self, split: Split, pattern=PAT_A2, drop=DROP_ABS, tau=1e-3, delta=0.4,
                 spai_steps=3, spai_per_step=5, spai_init=INIT_PATTERN_A, precision=FP32,
                 keep_lists=False, psai_lmax=10):
        L = lib()
        self.split = split
        o = BuildOpts(int(pattern), int(drop), float(tau), float(delta), int(spai_steps),
                      int(spai_per_step), int(spai_init), int(precision), int(bool(keep_lists)),
                      int(psai_lmax))
        self.stats = BuildStats()
        h = C.c_void_p()
        _check(L.sai_build(split.h, C.byref(o), _stream(), C.byref(h), C.byref(self.stats)),
               "sai_build")
        self.h = h
        self.info = PrecondInfo()
        _check(L.sai_precond_get_info(h, C.byref(self.info)), "sai_precond_get_info")
        self.precision = precision

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sai_precond_destroy(self.h)
            self.h = None

    def arrays(self):
        torch = _torch()
        i = self.info
        n, nnz = i.n, i.nnz
        vt = torch.float32 if i.precision == FP32 else torch.float64
        out = dict(
            col_ptr=_export(i.col_ptr, n + 1, torch.int32),
            row_idx=_export(i.row_idx, nnz, torch.int32),
            cval=_export(i.cval, nnz, vt),
            row_ptr=_export(i.row_ptr, n + 1, torch.int32),
            col_idx=_export(i.col_idx, nnz, torch.int32),
            val=_export(i.val, nnz, vt),
        )
        if i.j_ptr:
            jp = _export(i.j_ptr, n + 1, torch.int64)
            ip = _export(i.i_ptr, n + 1, torch.int64)
            nj, ni = int(jp[-1].item()), int(ip[-1].item())
            out.update(j_ptr=jp, j_idx=_export(i.j_idx, nj, torch.int32), i_ptr=ip,
                       i_idx=_export(i.i_idx, ni, torch.int32),
                       m_full=_export(i.m_full, nj, vt), res=_export(i.res, n, torch.float64))
        return out

    def stats_dict(self):
        s = self.stats
        return dict(n=s.n, nnz_m=s.nnz_m, nnz_m_full=s.nnz_m_full, sum_i=s.sum_i, max_i=s.max_i,
                    max_j=s.max_j, n_c=s.n_c, spar=s.spar, bucket_cols=list(s.bucket_cols),
                    t_pattern_ms=s.t_pattern_ms, t_ls_ms=s.t_ls_ms,
                    t_assemble_ms=s.t_assemble_ms, t_total_ms=s.t_total_ms, s=s.s, p=s.p,
                    l_m=s.l_m, drop_flips=s.drop_flips)


def _sopts(method=BICGSTAB, restart=30, eps=1e-8, maxit=500, c_mode=C_ONE, equilibrate=False):
    return SolveOpts(int(method), int(restart), float(eps), int(maxit), int(c_mode), int(bool(equilibrate)))


def krylov(split: Split, pc: Precond, R, thr, transpose=False, raise_on_error=True, **kw):
    """Solve A~ X = R (or A~^T X = R) for the columns of the row-major n x k block R."""
    torch = _torch()
    k = int(R.shape[1])
    X = torch.empty_like(R)
    thr_arr = (C.c_double * k)(*[float(t) for t in thr])
    its = (C.c_int32 * k)()
    sts = (C.c_int32 * k)()
    o = _sopts(**kw)
    code = lib().sai_krylov(split.h, pc.h, int(bool(transpose)), k, _ptr(R), _ptr(X), thr_arr,
                            C.byref(o), _stream(), its, sts)
    if raise_on_error and code not in (OK, ENOCONV, EBREAKDOWN):
        _check(code, "sai_krylov")
    return X, list(its), list(sts), code


def smw(split: Split, Y):
    torch = _torch()
    x = torch.empty(split.n, dtype=torch.float64, device="cuda")
    c = C.c_double()
    _check(lib().sai_smw(split.h, _ptr(Y), _ptr(x), C.byref(c), _stream()), "sai_smw")
    return x, c.value


def gather(split: Split, pc: Precond, precision=FP32, blk_off=None, out=None):
    """The dense blocks A~(I_k, J_k) (sai_gather) of a preconditioner built with
    keep_lists: returns (blk_off int64 tensor of n + 1 offsets, flat tensor of the
    column-major blocks)."""
    torch = _torch()
    L = lib()
    if blk_off is None:
        blk_off = torch.empty(split.n + 1, dtype=torch.int64, device="cuda")
        total = C.c_int64()
        _check(L.sai_gather_offsets(pc.h, _ptr(blk_off), C.byref(total), _stream()), "sai_gather_offsets")
        total = total.value
    else:
        total = int(blk_off[-1].item())
    if out is None:
        out = torch.empty(max(1, total), dtype=torch.float32 if precision == FP32 else torch.float64,
                          device="cuda")
    _check(L.sai_gather(split.h, pc.h, int(precision), _ptr(blk_off), _ptr(out), _stream()), "sai_gather")
    return blk_off, out


def smw_noalloc(split: Split, Y, x):
    """sai_smw_noalloc into the caller's x (the library allocates nothing); returns c."""
    c = C.c_double()
    _check(lib().sai_smw_noalloc(split.h, _ptr(Y), _ptr(x), C.byref(c), _stream()), "sai_smw_noalloc")
    return c.value


def residual(split: Split, b, x) -> float:
    rr = C.c_double()
    _check(lib().sai_residual(split.h, _ptr(b), _ptr(x), C.byref(rr), _stream()), "sai_residual")
    return rr.value


def _stats_dict(st, iters):
    return dict(s=st.s, status=st.status, iters_max=st.iters_max, iters=list(iters), rr=st.rr,
                a=st.a, c=st.c, t_solve_ms=st.t_solve_ms, t_smw_ms=st.t_smw_ms,
                t_check_ms=st.t_check_ms)


def solve(split: Split, pc: Precond, b, raise_on_error=True, **kw):
    """Procedure * for one right-hand side; returns (x, stats dict)."""
    torch = _torch()
    x = torch.empty(split.n, dtype=torch.float64, device="cuda")
    iters = (C.c_int32 * (split.s + 1))()
    st = SolveStats()
    st.iters = C.cast(iters, C.POINTER(C.c_int32))
    o = _sopts(**kw)
    code = lib().sai_solve(split.h, pc.h, _ptr(b), _ptr(x), C.byref(o), _stream(), C.byref(st))
    if raise_on_error:
        _check(code, "sai_solve")
    d = _stats_dict(st, iters)
    d["code"] = code
    return x, d


def solve_y(split: Split, pc: Precond, b, raise_on_error=True, **kw):
    """sai_solve_y: Procedure * keeping the Krylov solutions; returns (x, Y, stats dict)
    with Y = [y, W] (n x (s+1) float64) for backward_y."""
    torch = _torch()
    x = torch.empty(split.n, dtype=torch.float64, device="cuda")
    Y = torch.empty((split.n, split.s + 1), dtype=torch.float64, device="cuda")
    iters = (C.c_int32 * (split.s + 1))()
    st = SolveStats()
    st.iters = C.cast(iters, C.POINTER(C.c_int32))
    o = _sopts(**kw)
    code = lib().sai_solve_y(split.h, pc.h, _ptr(b), _ptr(x), _ptr(Y), C.byref(o), _stream(), C.byref(st))
    if raise_on_error:
        _check(code, "sai_solve_y")
    d = _stats_dict(st, iters)
    d["code"] = code
    return x, Y, d


def backward_y(split: Split, pc: Precond, x, Y, grad_x, want_b=True, want_a=True, raise_on_error=True,
               **kw):
    """sai_backward_y: the gradients of backward from the forward's Y (solve_y), one
    system with A~^T per correction pass; returns (grad_b, grad_a, stats dict)."""
    torch = _torch()
    gb = torch.empty(split.n, dtype=torch.float64, device="cuda") if want_b else None
    ga = torch.empty(split.nnz, dtype=torch.float64, device="cuda") if want_a else None
    iters = (C.c_int32 * (split.s + 1))()
    st = SolveStats()
    st.iters = C.cast(iters, C.POINTER(C.c_int32))
    o = _sopts(**kw)
    code = lib().sai_backward_y(split.h, pc.h, _ptr(x), _ptr(Y) if Y is not None else None, _ptr(grad_x),
                                _ptr(gb) if gb is not None else None,
                                _ptr(ga) if ga is not None else None, C.byref(o), _stream(),
                                C.byref(st))
    if raise_on_error:
        _check(code, "sai_backward_y")
    d = _stats_dict(st, iters)
    d["code"] = code
    return gb, ga, d


def backward(split: Split, pc: Precond, x, grad_x, want_b=True, want_a=True, raise_on_error=True,
             **kw):
    """Gradients (dL/db, dL/dA values in A's CSR order) for dL/dx = grad_x.

    The adjoint's auxiliary solves are refined to the theorem's threshold with the
    computed c' unless c_mode is given (see sai_backward in include/sai.h).
    """
    torch = _torch()
    kw.setdefault("c_mode", C_ONE_THEN_REFINE)
    gb = torch.empty(split.n, dtype=torch.float64, device="cuda") if want_b else None
    ga = torch.empty(split.nnz, dtype=torch.float64, device="cuda") if want_a else None
    iters = (C.c_int32 * (split.s + 1))()
    st = SolveStats()
    st.iters = C.cast(iters, C.POINTER(C.c_int32))
    o = _sopts(**kw)
    code = lib().sai_backward(split.h, pc.h, _ptr(x), _ptr(grad_x),
                              _ptr(gb) if gb is not None else None,
                              _ptr(ga) if ga is not None else None, C.byref(o), _stream(),
                              C.byref(st))
    if raise_on_error:
        _check(code, "sai_backward")
    return gb, ga, _stats_dict(st, iters)


def profile_enable(mode=1, only=None):
    """Start (and reset) the library's per-kernel HIP-event timing: 1 = every kernel,
    2 = only the kernels that can dominate (products, column solvers), 0/False = stop;
    with `only` (a name prefix) just the kernels whose name starts with it."""
    L = lib()
    if only is not None:
        _check(L.sai_profile_only(str(only).encode()), "sai_profile_only")
        mode = 3
    _check(L.sai_profile_enable(int(mode)), "sai_profile_enable")


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} accumulated since profile_enable(True)."""
    L = lib()
    out = {}
    cnt = L.sai_profile_count()
    if cnt < 0:
        raise SaiError(EHIP, "sai_profile_count", "event query failed")
    buf = C.create_string_buffer(128)
    for i in range(cnt):
        nl, ms = C.c_int64(), C.c_double()
        _check(L.sai_profile_get(i, buf, 128, C.byref(nl), C.byref(ms)), "sai_profile_get")
        out[buf.value.decode()] = (nl.value, ms.value)
    return out


def csr_to_device(A):
    """scipy CSR (int32 indices, float64 values) -> three CUDA tensors."""
    torch = _torch()
    return (torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(A.data, dtype=np.float64)).cuda())


from .autograd import SAISolve  # noqa: E402,F401
