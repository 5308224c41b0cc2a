"""Oracle patterns: brute force, lattice counts, envelope inclusion (Sections 2.2, 4)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import pattern as opat
from oracle import split as osplit
from tests import pins


@pytest.mark.parametrize("seed", range(4))
def test_A2_bruteforce(seed):
    At = W.random_sparse(50, 0.05, seed)
    pins.check_pattern_A2_bruteforce(opat.pattern_A2, At)
    C = opat.as_csc(At)
    Js = [opat.pattern_A2(C, k) for k in range(50)]
    pins.check_rows_of_bruteforce(opat.rows_of, At, Js)


def test_stencil_lattice_counts():
    # interior point of a 2D 5-point / 3D 7-point stencil: |P(A)|, |P(A^2)|, |P(A^3)|
    for dims, expect in [((9, 9), (5, 13, 25)), ((7, 7, 7), (7, 25, 63))]:
        r, c, v, n = W.stencil(dims, seed=1)
        A = sp.csr_matrix((v, (r, c)), shape=(n, n))
        C = opat.as_csc(A)
        mid = int(np.ravel_multi_index(tuple(d // 2 for d in dims[::-1]), dims[::-1]))
        J1 = opat.pattern_A(C, mid)
        J2 = opat.pattern_A2(C, mid)
        I2 = opat.rows_of(C, J2)
        assert (len(J1), len(J2), len(I2)) == expect
        assert mid in J1 and mid in J2 and mid in I2


def test_envelope_inclusion():
    # P((I+|A~|)^2) is contained in P((I+|A|)^2)  (Section 4, fifth issue)
    w = W.make(2, dims=(8, 8, 8), s=2, density=0.2)
    S = osplit.split(w.A)
    Ct = opat.as_csc(S.At)
    Ca = opat.as_csc(w.A)
    for k in range(w.A.shape[0]):
        assert set(opat.pattern_A2(Ct, k)) <= set(opat.pattern_A2(Ca, k))
