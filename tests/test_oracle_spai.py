"""Oracle SPAI augmentation (Section 2.1 (candi), (ls1d), (muj), (rhoj))."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lsq, pattern as opat, spai, split as osplit
from tests import pins


def _setup(n=300, seed=3):
    w = W.make(3, n=n, s=2, density=0.2)
    S = osplit.split(w.A)
    C = opat.as_csc(S.At)
    R = sp.csr_matrix(S.At)
    R.sort_indices()
    return S, C, R, spai.column_norms2(C)


def test_gains_bruteforce():
    S, C, R, cn2 = _setup()
    for k in [0, 5, 77, int(S.D[0])]:
        J = opat.pattern_A(C, k)
        I, m, res = lsq.solve_column(C, J, k)
        r = lsq.dense_block(C, I, J) @ m - (I == k)
        pins.check_spai_gains(spai.candidate_gains, S.At, J, I, r)


def test_steps_monotone_and_bounded_by_rho():
    S, C, R, cn2 = _setup()
    for k in range(0, 300, 23):
        J = opat.pattern_A(C, k)
        prev = None
        for _ in range(3):
            I, m, res = lsq.solve_column(C, J, k)
            if prev is not None:
                assert res <= prev[0] + 1e-12          # residual never grows
                assert res <= prev[1] + 1e-12          # at most the best single-index rho_j
            r = lsq.dense_block(C, I, J) @ m - (I == k)
            cand, tau, g, rho2 = spai.candidate_gains(C, R, cn2, J, I, r)
            add = spai.select(cand, g, min(5, cand.size))
            chosen = np.isin(cand, add)
            # the chosen indices carry the largest gains (smallest rho_j)
            if (~chosen).any():
                assert g[chosen].min() >= g[~chosen].max()
            prev = (res, float(np.sqrt(max(rho2[chosen].min(), 0.0))))
            J = np.array(sorted(set(J.tolist()) | set(add.tolist())))


def test_delta_zero_many_steps_reaches_inverse():
    At = W.random_sparse(14, 0.12, 5, diag=2.0)
    C = opat.as_csc(At)
    R = sp.csr_matrix(At)
    R.sort_indices()
    cn2 = spai.column_norms2(C)
    inv = np.linalg.inv(At.toarray())
    for k in range(14):
        J, I, m, res, taken = spai.spai_column(C, R, cn2, k, steps=14, per_step=1, delta=0.0,
                                              init="diag")
        full = np.zeros(14)
        full[J] = m
        assert res < 1e-10 and np.allclose(full, inv[:, k], atol=1e-10)


def test_stops_at_delta():
    S, C, R, cn2 = _setup()
    out = spai.spai(S.At, steps=3, per_step=5, delta=0.4, cols=range(40))
    for J, I, m, res, taken in out:
        assert taken <= 3
        if taken < 3:
            assert res <= 0.4
