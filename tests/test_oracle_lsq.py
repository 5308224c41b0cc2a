"""Oracle column LS problems (Section 2 (subprob), (lsprob)): optimality and special cases."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lsq, pattern as opat, split as osplit
from tests import pins


@pytest.mark.parametrize("seed", range(3))
def test_full_pattern_gives_inverse(seed):
    At = W.random_sparse(30, 0.1, seed, diag=2.0)
    pins.check_full_pattern_inverse(lsq.solve_column, At)


def test_block_diagonal_exact_inverse():
    rng = np.random.default_rng(0)
    blocks = [rng.uniform(-1, 1, (4, 4)) + 4 * np.eye(4) for _ in range(5)]
    At = sp.csr_matrix(sp.block_diag(blocks))
    C = opat.as_csc(At)
    inv = np.linalg.inv(At.toarray())
    for k in range(20):
        J = np.arange(4 * (k // 4), 4 * (k // 4) + 4)
        I, m, res = lsq.solve_column(C, J, k)
        assert np.allclose(m, inv[J, k], atol=1e-12) and res < 1e-12


@pytest.mark.parametrize("kind", ["A", "A2"])
def test_normal_equations_and_pythagoras(kind):
    w = W.make(2, dims=(7, 7, 7), s=2, density=0.2)
    S = osplit.split(w.A)
    C = opat.as_csc(S.At)
    f = opat.pattern_A if kind == "A" else opat.pattern_A2
    for k in list(range(0, 343, 17)) + list(S.D):
        pins.check_ls_optimality(lsq.solve_column, S.At, f(C, int(k)), int(k))
