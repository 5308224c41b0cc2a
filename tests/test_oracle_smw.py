"""Oracle SMW recovery (Theorem 3.1, Procedure * (update1), (composi), (rry))."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import pipeline, smw, split as osplit
from tests import pins


@pytest.mark.parametrize("idx,kw", [(1, {}), (2, dict(dims=(7, 7, 7), s=3, density=0.15))])
def test_recover_exact_and_identity(idx, kw):
    w = W.make(idx, **kw)
    S = osplit.split(w.A)
    U = S.U.toarray()
    pins.check_smw_exact(smw.recover, w.A, S.At, U, S.D, w.b)
    pins.check_residual_identity(smw.recover, w.A, S.At, U, S.D, w.b, np.random.default_rng(idx))


def test_sherman_morrison_s1():
    w = W.make(1, s=1)
    S = osplit.split(w.A)
    assert S.s == 1
    Atd = S.At.toarray()
    u = S.U.toarray()[:, 0]
    j = int(S.D[0])
    y = np.linalg.solve(Atd, w.b)
    wv = np.linalg.solve(Atd, u)
    x_sm = y - wv * (y[j] / (1.0 + wv[j]))
    x, z, c = smw.recover(y, wv[:, None], S.D)
    assert np.allclose(x, x_sm, rtol=0, atol=1e-13 * np.abs(x_sm).max())


def test_determinant_lemma():
    w = W.make(2, dims=(5, 5, 5), s=3, density=0.4)
    S = osplit.split(w.A)
    Atd = S.At.toarray()
    Wx = np.linalg.solve(Atd, S.U.toarray())
    K = np.eye(S.s) + Wx[S.D, :]
    sA, ldA = np.linalg.slogdet(w.A.toarray())
    sT, ldT = np.linalg.slogdet(Atd)
    sK, ldK = np.linalg.slogdet(K)
    assert sK == sA * sT and abs(ldK - (ldA - ldT)) < 1e-9


def test_singular_K_raises():
    y = np.ones(6)
    Wm = np.zeros((6, 2))
    Wm[1, 1] = 1.0
    Wm[4, 0] = 1.0
    with pytest.raises(smw.SingularK):
        smw.recover(y, Wm, np.array([1, 4]))


def test_s0_path():
    w = W.make(1, s=0)
    out = pipeline.run(w.A, w.b, kind="A", method="gmres")
    assert out["split"].s == 0 and out["rr"] < 1e-8


@pytest.mark.parametrize("idx,kw,method", [(1, {}, "gmres"), (1, {}, "bicgstab"),
                                           (2, dict(dims=(7, 7, 7), s=3, density=0.15), "bicgstab")])
def test_pipeline_matches_dense_lu(idx, kw, method):
    w = W.make(idx, **kw)
    out = pipeline.run(w.A, w.b, kind="A" if idx == 1 else "A2", drop="abs" if idx != 1 else "none",
                       method=method)
    xd = np.linalg.solve(w.A.toarray(), w.b)
    kappa = np.linalg.cond(w.A.toarray(), 1)
    assert out["rr"] < 2e-8
    assert np.linalg.norm(out["x"] - xd) <= 2 * kappa * 1e-8 * np.linalg.norm(xd)
