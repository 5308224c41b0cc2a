"""Oracle dropping (Section 2.2 (tolk)) and assembly of M."""
import numpy as np

import workloads as W
from oracle import drop, lsq, pattern as opat, split as osplit
from tests import pins


def test_tolk_2delta_bound():
    w = W.make(2, dims=(6, 6, 6), s=2, density=0.2)
    S = osplit.split(w.A)
    C = opat.as_csc(S.At)
    n = S.At.shape[0]
    Js = [opat.pattern_A2(C, k) for k in range(n)]
    _, ms, res = lsq.build_columns(S.At, Js)
    for delta in (0.4, 0.1, 2.0):
        pins.check_drop_bound(drop.assemble, S.At, Js, ms, res, delta)


def test_abs_threshold_semantics():
    m = np.array([1e-3, -2e-3, 5e-4, -1e-3, 0.3])
    keep = drop.drop_column(m, 1e-3)
    assert keep.tolist() == [False, True, False, False, True]
    # the largest entry survives any threshold
    assert drop.drop_column(m, 10.0).tolist() == [False, False, False, False, True]
