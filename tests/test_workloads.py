"""Synthetic workloads: sizes, p, and the seeded dense columns are detected."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("idx,n,p,s", [(1, 2025, 5, 3), (2, 1000000, 7, 10), (3, 200000, 8, 20),
                                       (4, 250000, 5, 8)])
def test_workload_shapes(idx, n, p, s):
    w = W.make(idx)
    A = w.A
    assert A.shape == (n, n)
    assert A.indptr.dtype == np.int32 and A.indices.dtype == np.int32
    assert A.nnz // n == p
    counts = np.bincount(A.indices, minlength=n)
    assert sorted(np.flatnonzero(counts > 10 * p).tolist()) == list(w.dense_cols)
    assert np.all(np.diff(A.indices[A.indptr[0]:A.indptr[1]]) > 0)
    assert np.allclose(w.b, A @ np.ones(n))


def test_workload_deterministic():
    a = W.make(1)
    b = W.make(1)
    assert (a.A != b.A).nnz == 0 and np.array_equal(a.b, b.b)


def test_banded_generator():
    A = W.banded(600, 8, 2, 0.5, 7)
    assert A.shape == (600, 600) and A.indptr.dtype == np.int32
    B = W.banded(600, 8, 2, 0.5, 7)
    assert (A != B).nnz == 0
    r, c = A.nonzero()
    counts = np.bincount(c, minlength=600)
    dense = np.flatnonzero(counts > 10 * (A.nnz // 600))
    assert dense.size == 2
    band = ~np.isin(c, dense)
    assert np.all(np.abs(r[band] - c[band]) <= 8)
    # interior columns hold the full band
    assert np.all(counts[np.setdiff1d(np.arange(8, 592), dense)] == 17)
