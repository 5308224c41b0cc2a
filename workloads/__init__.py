"""Seeded synthetic inputs for the SMW-split SAI path.

This module builds test matrices and right-hand sides only.  It holds none of
the method's arithmetic (no split, no pattern, no least squares, no Krylov
step); both the FP64 oracle's tests and the GPU path's tests and benchmark
draw their inputs from here.

The paper measures on matrices of the University of Florida collection
(Section 5, Tables 2-3: circuit, semiconductor, 2D/3D and CFD problems with a
few nearly dense columns).  Those matrices are not available here; the five
workloads below stand in for them, each a regular sparse base (2D/3D
convection-diffusion stencil or a random sparse matrix) plus ``s`` seeded
dense columns.  The right-hand side is b = A*1, as in Section 5.

Recipe (seed = 12116866 + workload index; numpy ``default_rng([seed, stream])``
with one stream per random quantity so that changing one does not move the
others):

* stencil workloads: lexicographic grid (x fastest), Dirichlet boundary;
  diagonal ``2*d + 0.1*U[0,1]`` (d = 2 or 3), off-diagonals
  ``-1 + 0.2*U[-1,1]`` drawn independently per entry (nonsymmetric values).
* random workload: column k gets G_k ~ Geometric(1/7) (mean 7, capped at 70)
  off-diagonal entries at uniform rows != k, values N(0,1); after the dense
  columns are added, diag_i = 1.5 * sum_{j != i} |A_ij| (1.0 if that is 0),
  so A is strictly row diagonally dominant.
* dense columns: ``s`` distinct column indices; each receives round(rho*n)
  extra entries at rows not already present in it, values U[-1,1]
  (N(0,1) for the random workload).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

BASE_SEED = 12116866

# stream ids for default_rng([seed, stream])
S_DIAG, S_OFF, S_DCOL_IDX, S_DCOL_ROWS, S_DCOL_VALS, S_XSTAR, S_FD, S_PATTERN = range(8)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([seed, stream])


@dataclasses.dataclass
class Workload:
    name: str
    A: sp.csr_matrix            # int32 indices, float64 values, sorted, no duplicates
    b: np.ndarray               # float64, = A @ ones
    dense_cols: np.ndarray      # the seeded dense-column indices (ascending)
    seed: int
    meta: dict


def _csr(rows, cols, vals, n) -> sp.csr_matrix:
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def stencil(dims, seed: int, diag_base: Optional[float] = None):
    """2D 5-point or 3D 7-point convection-diffusion-like stencil as COO triplets."""
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    n = int(np.prod(dims))
    if diag_base is None:
        diag_base = 2.0 * nd
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    rows = [idx]
    cols = [idx]
    vals = [diag_base + 0.1 * _rng(seed, S_DIAG).random(n)]
    # 2*nd neighbour slots, values drawn for every slot (masked afterwards)
    off = -1.0 + 0.2 * _rng(seed, S_OFF).uniform(-1.0, 1.0, size=(2 * nd, n))
    slot = 0
    for a in range(nd):
        for sgn in (-1, 1):
            c = coords[a] + sgn
            ok = (c >= 0) & (c < dims[a])
            rows.append(idx[ok])
            cols.append(idx[ok] + sgn * strides[a])
            vals.append(off[slot][ok])
            slot += 1
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n


def random_irregular_base(n: int, seed: int, mean_extra: float = 7.0, cap: int = 70):
    """Column k: G_k ~ Geometric(1/mean) off-diagonal rows (uniform, != k), N(0,1) values."""
    rg = _rng(seed, S_PATTERN)
    G = np.minimum(rg.geometric(1.0 / mean_extra, size=n), cap)
    rows = np.empty(int(G.sum()), dtype=np.int64)
    cols = np.repeat(np.arange(n, dtype=np.int64), G)
    pos = 0
    for k in range(n):
        g = int(G[k])
        r = rg.choice(n - 1, size=g, replace=False)
        r = r + (r >= k)                      # skip the diagonal
        rows[pos:pos + g] = r
        pos += g
    vals = _rng(seed, S_OFF).standard_normal(rows.size)
    return rows, cols, vals


def _skip_existing(cand: np.ndarray, existing_sorted: np.ndarray) -> np.ndarray:
    """Map c in [0, n - len(existing)) to the c-th integer not in ``existing_sorted``."""
    e = existing_sorted
    adj = e - np.arange(e.size)
    return cand + np.searchsorted(adj, cand, side="right")


def add_dense_columns(rows, cols, vals, n, s, density, seed, normal_values=False,
                      dense_cols: Optional[np.ndarray] = None):
    """Append round(density*n) entries to each of ``s`` seeded columns, at rows not present."""
    if dense_cols is None:
        dense_cols = np.sort(_rng(seed, S_DCOL_IDX).choice(n, size=s, replace=False))
    dense_cols = np.asarray(dense_cols, dtype=np.int64)
    rr = _rng(seed, S_DCOL_ROWS)
    rv = _rng(seed, S_DCOL_VALS)
    m = int(round(density * n))
    order = np.argsort(cols, kind="stable")
    cs = cols[order]
    add_r, add_c, add_v = [], [], []
    for j in dense_cols:
        lo, hi = np.searchsorted(cs, [j, j + 1])
        existing = np.sort(rows[order[lo:hi]])
        mm = min(m, n - existing.size)
        cand = rr.choice(n - existing.size, size=mm, replace=False)
        newr = _skip_existing(np.sort(cand), existing)
        add_r.append(newr)
        add_c.append(np.full(mm, j, dtype=np.int64))
        add_v.append(rv.standard_normal(mm) if normal_values else rv.uniform(-1.0, 1.0, mm))
    if add_r:
        rows = np.concatenate([rows] + add_r)
        cols = np.concatenate([cols] + add_c)
        vals = np.concatenate([vals] + add_v)
    return rows, cols, vals, dense_cols


# --- the five workloads --------------------------------------------------------

WORKLOADS = {
    1: dict(name="stencil2d_45x45_s3", kind="2d", dims=(45, 45), s=3, density=0.20,
            pattern="A", solver="gmres", restart=30, precision="fp64"),
    2: dict(name="stencil3d_100^3_s10", kind="3d", dims=(100, 100, 100), s=10, density=0.05,
            pattern="A2", solver="bicgstab", tau=1e-3, precision="fp32"),
    3: dict(name="random_n200000_s20", kind="random", n=200000, s=20, density=0.02,
            pattern="spai", solver="bicgstab", spai_steps=3, spai_per_step=5, delta=0.4,
            precision="fp32"),
    4: dict(name="stencil2d_500x500_s8", kind="2d", dims=(500, 500), s=8, density=0.03,
            pattern="A2", solver="bicgstab", tau=1e-3, precision="fp32"),
    5: dict(name="stencil3d_160^3_s50", kind="3d", dims=(160, 160, 160), s=50, density=0.01,
            pattern="A2", solver="bicgstab", tau=1e-3, precision="fp32"),
}


def make(index: int, dims=None, n: Optional[int] = None, s: Optional[int] = None,
         density: Optional[float] = None, diag_base: Optional[float] = None) -> Workload:
    """Build workload ``index`` (1..5), optionally at a smaller grid / n / s for tests."""
    cfg = dict(WORKLOADS[index])
    seed = BASE_SEED + index
    s = cfg["s"] if s is None else s
    density = cfg["density"] if density is None else density
    if cfg["kind"] in ("2d", "3d"):
        dims = cfg["dims"] if dims is None else tuple(dims)
        r, c, v, nn = stencil(dims, seed, diag_base)
        r, c, v, D = add_dense_columns(r, c, v, nn, s, density, seed)
        A = _csr(r, c, v, nn)
        meta = dict(cfg, dims=dims, s=s, density=density)
    else:
        nn = cfg["n"] if n is None else int(n)
        r, c, v = random_irregular_base(nn, seed)
        r, c, v, D = add_dense_columns(r, c, v, nn, s, density, seed, normal_values=True)
        off = _csr(r, c, v, nn)
        rowabs = np.asarray(abs(off).sum(axis=1)).ravel()
        dv = np.where(rowabs > 0, 1.5 * rowabs, 1.0)
        A = _csr(np.concatenate([r, np.arange(nn)]), np.concatenate([c, np.arange(nn)]),
                 np.concatenate([v, dv]), nn)
        meta = dict(cfg, n=nn, s=s, density=density)
    b = A @ np.ones(A.shape[0])
    meta["n"] = A.shape[0]
    meta["nnz"] = int(A.nnz)
    return Workload(cfg["name"], A, b, np.asarray(D, dtype=np.int64), seed, meta)


def x_star(n: int, seed: int) -> np.ndarray:
    """Target vector x* ~ N(0,1) for the loss 0.5*||x - x*||^2."""
    return _rng(seed, S_XSTAR).standard_normal(n)


def fd_entries(A: sp.csr_matrix, dense_cols: np.ndarray, seed: int, count: int = 16):
    """Seeded nonzero positions of A (CSR value indices) for finite-difference checks.

    Half of them are drawn among entries outside the dense columns (at least two
    of them diagonal), half among entries inside the dense columns.
    """
    rg = _rng(seed, S_FD)
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices.astype(np.int64)
    in_dense = np.isin(cols, dense_cols)
    diag_pos = np.flatnonzero((rows == cols) & ~in_dense)
    off_pos = np.flatnonzero((rows != cols) & ~in_dense)
    dense_pos = np.flatnonzero(in_dense & (rows != cols))
    half = count // 2
    pick = [rg.choice(diag_pos, size=2, replace=False),
            rg.choice(off_pos, size=half - 2, replace=False),
            rg.choice(dense_pos, size=count - half, replace=False)]
    return np.concatenate(pick).astype(np.int64)


def random_sparse(n: int, density: float, seed: int, diag: float = 0.0) -> sp.csr_matrix:
    """Small random sparse matrix with a full diagonal, for oracle self-tests."""
    rg = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rg, format="coo")
    r = np.concatenate([M.row, np.arange(n)])
    c = np.concatenate([M.col, np.arange(n)])
    v = np.concatenate([rg.uniform(-1, 1, M.nnz), diag + rg.uniform(0.5, 1.5, n)])
    A = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def banded(n: int, half_bw: int, s: int, density: float, seed: int) -> sp.csr_matrix:
    """Seeded banded matrix (|i - j| <= half_bw, diagonally dominant) plus ``s`` dense
    columns: wide enough bands make the candidate lists of the static pattern
    P(|A~|^2 e_k) long (about (4 hb + 1)(2 hb + 1) entries), for tests."""
    rg = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int64)
    rows, cols, vals = [], [], []
    for d in range(-half_bw, half_bw + 1):
        ok = (i + d >= 0) & (i + d < n)
        rows.append(i[ok])
        cols.append(i[ok] + d)
        vals.append(np.full(ok.sum(), 2.0 * half_bw + 1.0 + rg.random()) if d == 0
                    else rg.uniform(-1.0, 1.0, ok.sum()))
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    r, c, v, _ = add_dense_columns(r, c, v, n, s, density, seed)
    return _csr(r, c, v, n)
