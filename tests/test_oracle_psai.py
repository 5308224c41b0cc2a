"""Oracle PSAI(tol) (Section 2.2: the power patterns P(|A~|^l e_k), (lsprob), (tolk))."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import drop as odrop, lsq, pattern as opat, psai, split as osplit


def _tridiag(n, d=2.5):
    A = sp.diags([np.full(n - 1, -1.0), np.full(n, d), np.full(n - 1, -1.0)], [-1, 0, 1]).tocsr()
    A.sort_indices()
    return A


def test_full_pattern_limit_gives_inverse():
    # the power pattern of a tridiagonal matrix grows by one index on each side
    # per loop; with a tiny delta nothing of the (slowly decaying) inverse is
    # dropped, the loop reaches the full pattern and the column is A^{-1} e_k
    n = 8
    A = _tridiag(n)
    Ainv = np.linalg.inv(A.toarray())
    Ss, ms, rs, ls = psai.psai_tol(A, delta=1e-10, lmax=20)
    for k in range(n):
        assert np.array_equal(Ss[k], np.arange(n)), k
        np.testing.assert_allclose(ms[k], Ainv[:, k], rtol=1e-12, atol=1e-14)
        assert rs[k] <= 1e-12
        # the pattern is full once both ends are reached: max(k, n-1-k) loops
        assert ls[k] == max(k, n - 1 - k), (k, ls[k])


@pytest.mark.parametrize("idx,kw", [(3, dict(n=400, s=3, density=0.1)),
                                    (4, dict(dims=(20, 18), s=2, density=0.1)),
                                    (2, dict(dims=(7, 6, 5), s=2, density=0.2))])
def test_two_delta_bound_after_dropping(idx, kw):
    # Section 2.2: with (tolk), a column whose residual fell below delta keeps
    # ||A~ m_k - e_k|| <= 2 delta after its small entries are dropped
    w = W.make(idx, **kw)
    At = osplit.split(w.A).At
    C = opat.as_csc(At)
    delta, lmax = 0.4, 6
    cols = list(range(0, At.shape[0], 7))
    Ss, ms, rs, ls = psai.psai_tol(At, delta=delta, lmax=lmax, cols=cols)
    stopped = 0
    for t, k in enumerate(cols):
        assert 1 <= ls[t] <= lmax + 1
        assert Ss[t].size == ms[t].size and np.all(np.diff(Ss[t]) > 0)
        if rs[t] <= delta:
            stopped += 1
            x = np.zeros(At.shape[0])
            x[Ss[t]] = ms[t]
            e = np.zeros(At.shape[0])
            e[k] = 1.0
            assert np.linalg.norm(C @ x - e) <= 2 * delta + 1e-12, k
    assert stopped == len(cols)


def test_first_loop_pattern_and_values():
    # delta >= 1 stops after the first loop (any LS solution has residual <=
    # ||e_k|| = 1): the pattern is P(A~ e_k) union {k}, the values its LS
    # solution with the (tolk) drop
    w = W.make(3, n=300, s=2, density=0.1)
    At = osplit.split(w.A).At
    C = opat.as_csc(At)
    a1 = odrop.norm1(At)
    for k in [0, 17, 150, 299]:
        S, m, r, nl = psai.psai_tol_column(C, k, delta=1.0, lmax=5, a1=a1)
        assert nl == 1
        S0 = np.union1d(opat.pattern_A(C, k), [k])
        _, m0, r0 = lsq.solve_column(C, S0, k)
        keep = odrop.drop_column(m0, 1.0 / (S0.size * a1))
        assert np.array_equal(S, S0[keep])
        np.testing.assert_array_equal(m, m0[keep])
        assert r == r0
