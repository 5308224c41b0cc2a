"""Oracle split (Procedure * step 1, Section 4): pins against Table 3 and brute force."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import split as osplit
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3.txt")


def _table3():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, n, s, p, pd, nnz, nnzt, keep = line.split()
        rows.append(dict(name=name, n=int(n), s=int(s), p=int(p), pd=int(pd), nnz=int(nnz),
                         nnzt=int(nnzt), keep=None if keep == "-" else int(keep)))
    return rows


def _matrix_like(row, seed=0):
    """A matrix with Table 3's n, nnz, s and densest column p_d.

    Irregular columns: one with p_d entries, the other s-1 with 10p+1 entries
    (tols4000: all 18 with p_d = 22).  Regular columns share the remaining entries,
    each at most 10p, and one regular column holds exactly 10p entries so that
    the strict reading of "exceeds 10p" is exercised.
    """
    rng = np.random.default_rng(seed)
    n, s, p, pd, nnz = row["n"], row["s"], row["p"], row["pd"], row["nnz"]
    counts = np.zeros(n, dtype=np.int64)
    dense = rng.choice(n, size=s, replace=False)
    counts[dense] = 10 * p + 1
    counts[dense[0]] = pd
    if row["name"] == "tols4000":
        counts[dense] = pd
    regular = np.setdiff1d(np.arange(n), dense)
    counts[regular[0]] = 10 * p
    rest = regular[1:]
    remaining = nnz - counts.sum()
    base, extra = divmod(remaining, rest.size)
    counts[rest] = base
    counts[rest[:extra]] += 1
    assert counts.max() <= max(pd, 10 * p) and counts[rest].max() <= 10 * p and counts.min() >= 1
    rows_l, cols_l = [], []
    for j in range(n):
        c = int(counts[j])
        others = rng.choice(n - 1, size=c - 1, replace=False)
        others = others + (others >= j)
        rows_l.append(np.concatenate([[j], others]))
        cols_l.append(np.full(c, j))
    r = np.concatenate(rows_l)
    c = np.concatenate(cols_l)
    A = sp.csr_matrix((rng.uniform(0.5, 1.0, r.size), (r, c)), shape=(n, n))
    A.sort_indices()
    assert A.nnz == nnz
    return A


@pytest.mark.parametrize("row", _table3(), ids=lambda r: r["name"])
def test_table3_p_s_and_nnz(row):
    A = _matrix_like(row)
    S = osplit.split(A, keep=row["keep"])
    assert S.p == row["p"]
    assert S.s == row["s"]
    if row["keep"] is not None:
        assert S.At.nnz == row["nnzt"]


@pytest.mark.parametrize("seed", range(6))
def test_split_bruteforce_random(seed):
    rng = np.random.default_rng(seed)
    n = 40
    A = W.random_sparse(n, 0.04, seed)
    A = A.tolil()
    for j in rng.choice(n, size=2, replace=False):
        rows = rng.choice(n, size=30, replace=False)
        for i in rows:
            A[i, j] = rng.uniform(-1, 1) or 0.5
    A = sp.csr_matrix(A)
    A.sort_indices()
    pins.check_split_bruteforce(osplit.split, A)
    pins.check_split_bruteforce(osplit.split, A, keep=1)
    pins.check_split_bruteforce(osplit.split, A, keep=4)


def test_split_tie_break_smaller_row():
    # column 10 holds rows 8 and 12 (distance 2 both) plus far rows; keep = 2
    n = 30
    A = sp.lil_matrix((n, n))
    for i in range(n):
        A[i, i] = 4.0
    for i in [8, 12] + list(range(20, 30)):
        A[i, 10] = 1.0
    A = sp.csr_matrix(A)
    S = osplit.split(A, dense_factor=2.0, keep=2)   # p = 1 -> threshold 2
    assert list(S.D) == [10]
    kept = sp.csc_matrix(S.At)[:, 10].nonzero()[0].tolist()
    assert kept == [8, 10]


def test_split_zero_diagonal_raises():
    n = 20
    A = sp.lil_matrix((n, n))
    for i in range(n):
        if i != 3:
            A[i, i] = 1.0
    for i in range(n):
        if i != 3:
            A[i, 3] = 0.5
    with pytest.raises(osplit.ZeroDiagonal):
        osplit.split(sp.csr_matrix(A))


@pytest.mark.parametrize("idx,kw", [(1, {}), (2, dict(dims=(12, 12, 12), s=3)),
                                    (3, dict(n=4000, s=4, density=0.05)),
                                    (4, dict(dims=(40, 40), s=2, density=0.1))])
def test_split_workloads_invariants(idx, kw):
    w = W.make(idx, **kw)
    S = osplit.split(w.A)
    assert list(S.D) == list(w.dense_cols)
    recon = S.At + sp.csr_matrix(S.U @ sp.csr_matrix(
        (np.ones(S.s), (np.arange(S.s), S.D)), shape=(S.s, w.A.shape[0])))
    diff = (recon - w.A)
    assert abs(diff).max() == 0.0
    assert S.At.nnz + S.U.nnz == w.A.nnz
    C = sp.csc_matrix(S.At)
    for j in S.D:
        assert C[j, j] != 0 and C[:, j].nnz == S.p


def test_split_largest_rule():
    n = 40
    rng = np.random.default_rng(3)
    A = sp.lil_matrix((n, n))
    for i in range(n):
        A[i, i] = 2.0
    vals = rng.permutation(np.linspace(0.1, 3.0, 30))
    for t, i in enumerate(rng.choice([i for i in range(n) if i != 7], 30, replace=False)):
        A[i, 7] = vals[t]
    A = sp.csr_matrix(A)
    S = osplit.split(A, keep=3, rule="largest")
    col = sp.csc_matrix(S.At)[:, 7].toarray().ravel()
    off = sorted([abs(v) for v in sp.csc_matrix(A)[:, 7].toarray().ravel()], reverse=True)
    kept_off = sorted([abs(col[i]) for i in np.flatnonzero(col) if i != 7], reverse=True)
    assert kept_off == [v for v in off if v != 2.0][:2]


def test_split_with_given_columns_matches_detection():
    """Naming the irregular columns reproduces the count rule's split exactly, and
    naming none leaves A~ = A."""
    import workloads as W
    from oracle import split as osplit
    w = W.make(2, dims=(9, 8, 7), s=3, density=0.3)
    S = osplit.split(w.A)
    S2 = osplit.split(w.A, dense_cols=list(S.D))
    assert (S2.At != S.At).nnz == 0 and (S2.U != S.U).nnz == 0 and list(S2.D) == list(S.D)
    S0 = osplit.split(w.A, dense_cols=[])
    assert S0.s == 0 and (S0.At != w.A).nnz == 0
