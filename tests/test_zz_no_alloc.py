"""sai_smw_noalloc (the allocation-free SMW recovery) against sai_smw, through the C ABI.

Two calls in a row on different splits, the second smaller, each compared with
sai_smw on the same Y (same kernels: bit-identical x and c); no allocation
request reaches the allocator during the call; s > 64 is rejected; a singular K
is reported and a following call is unaffected.
"""
import numpy as np
import pytest

import workloads as W
from oracle import krylov as okry
from oracle import split as osplit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1211_6866_amd as P  # noqa: E402


def _case(idx, **kw):
    w = W.make(idx, **kw)
    S = osplit.split(w.A)
    g = P.Split(*P.csr_to_device(w.A))
    pc = P.Precond(g, pattern=P.PAT_A2, drop=P.DROP_ABS, tau=1e-3, precision=P.FP32)
    n, s = w.A.shape[0], S.s
    R = np.zeros((n, s + 1))
    R[:, 0] = w.b
    R[:, 1:] = S.U.toarray()
    thr = okry.thresholds(np.linalg.norm(w.b), s, 1e-10)
    Y, its, sts, code = P.krylov(g, pc, torch.from_numpy(R).cuda(), thr)
    assert code == P.OK
    return w, g, Y


def _compare(g, Y):
    x_ref, c_ref = P.smw(g, Y)
    x = torch.full_like(x_ref, float("nan"))
    torch.cuda.synchronize()
    before = P.ALLOC_CALLS[0]
    c = P.smw_noalloc(g, Y, x)
    assert P.ALLOC_CALLS[0] == before, "the allocation-free entry point requested memory"
    assert torch.equal(x, x_ref) and c == c_ref, (c, c_ref)
    return c


def test_noalloc_matches_smw_two_calls():
    w1, g1, Y1 = _case(2, dims=(12, 12, 12), s=6, density=0.2)
    w2, g2, Y2 = _case(2, dims=(9, 8, 7), s=3, density=0.3)
    assert w2.A.shape[0] < w1.A.shape[0] and g2.s < g1.s
    c1 = _compare(g1, Y1)
    c2 = _compare(g2, Y2)
    assert c1 > 0 and c2 > 0


def test_noalloc_rejects_s_above_64_and_reports_singular():
    rp, ci, va = P.csr_to_device(W.make(2, dims=(12, 12, 12), s=2, density=0.2).A)
    g = P.Split(rp, ci, va, dense_cols=list(range(0, 1300, 20)))
    assert g.s == 65
    Y = torch.zeros((g.n, g.s + 1), dtype=torch.float64, device="cuda")
    x = torch.empty(g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SaiError) as e:
        P.smw_noalloc(g, Y, x)
    assert e.value.code == P.ETOOBIG
    # K = I + W(j, :) singular: W(j_1, 0) = -1 with s = 1
    g1 = P.Split(rp, ci, va, dense_cols=[100])
    Y1 = torch.zeros((g1.n, 2), dtype=torch.float64, device="cuda")
    Y1[100, 1] = -1.0
    with pytest.raises(P.SaiError) as e:
        P.smw_noalloc(g1, Y1, x)
    assert e.value.code == P.ESINGULAR
    # the flag is cleared by the next call
    Y1[100, 1] = 1.0
    Y1[:, 0] = 1.0
    c = P.smw_noalloc(g1, Y1, x)
    assert abs(c - 0.5) < 1e-15 and torch.allclose(x, torch.full_like(x, 1.0) - Y1[:, 1] * 0.5)
