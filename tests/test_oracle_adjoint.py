"""Oracle adjoint through the transposed split: dense solves, trace identity, FD."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import adjoint, pipeline


def _problem():
    w = W.make(1, dims=(15, 15), s=2, density=0.3)
    out = pipeline.run(w.A, w.b, kind="A2", drop="none", eps=1e-12, method="bicgstab")
    return w, out


def test_adjoint_matches_dense_solve_and_trace_identity():
    w, out = _problem()
    x = out["x"]
    xs = W.x_star(w.A.shape[0], w.seed)
    g = x - xs
    adj = adjoint.adjoint(out["split"], out["M"], x, g, eps=1e-12)
    lam_d = np.linalg.solve(w.A.toarray().T, g)
    assert np.linalg.norm(adj["lam"] - lam_d) <= 1e-9 * np.linalg.norm(lam_d)
    G = adjoint.grad_A_values(w.A, adj["lam"], x)
    # sum_ij A_ij G_ij = -lambda^T A x = -lambda^T b
    lhs = float(np.dot(w.A.data, G))
    assert abs(lhs + adj["lam"] @ w.b) <= 1e-9 * abs(adj["lam"] @ w.b)


def test_gradients_central_differences():
    w, out = _problem()
    A = w.A.toarray()
    xs = W.x_star(A.shape[0], w.seed)
    x = np.linalg.solve(A, w.b)
    g = x - xs
    adj = adjoint.adjoint(out["split"], out["M"], out["x"], out["x"] - xs, eps=1e-12)
    G = adjoint.grad_A_values(w.A, adj["lam"], out["x"])
    pos = W.fd_entries(w.A, w.dense_cols, w.seed, 16)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(w.A.indptr))
    h = 1e-6

    def loss(Am, b):
        xx = np.linalg.solve(Am, b)
        return 0.5 * np.sum((xx - xs) ** 2)

    for q in pos:
        i, j = rows[q], w.A.indices[q]
        E = np.zeros_like(A)
        E[i, j] = h
        fd = (loss(A + E, w.b) - loss(A - E, w.b)) / (2 * h)
        assert abs(fd - G[q]) <= 1e-5 * max(abs(G[q]), 1e-3 * np.abs(G).max()), (q, fd, G[q])
    # dL/db by central differences on a few entries
    for i in [0, 7, 100]:
        e = np.zeros(A.shape[0])
        e[i] = h
        fd = (loss(A, w.b + e) - loss(A, w.b - e)) / (2 * h)
        assert abs(fd - adj["grad_b"][i]) <= 1e-5 * max(abs(fd), 1e-3)


# ---- the adjoint from the forward solve's W (one system with A~^T) ----------------

def test_forward_correction_exact():
    """A~^{-T} of the corrected right-hand side is A^{-T} g, with exact W; s = 2 and
    s = 4 (K = I + V^T W not symmetric)."""
    from tests import pins
    for dims, s in (((15, 15), 2), ((14, 16), 4)):
        w = W.make(1, dims=dims, s=s, density=0.3)
        S = pipeline.split_mod.split(w.A)
        g = np.random.default_rng(7).standard_normal(w.A.shape[0])
        pins.check_forward_correction_exact(adjoint.forward_correction, w.A, S.At, S.U, S.D, g)


def test_adjoint_from_forward_matches_dense_and_transposed_split():
    """With the forward's W (eps 1e-12) lambda equals the dense A^{-T} g and the
    transposed-split oracle's lambda; the trace identity holds."""
    w, out = _problem()
    x = out["x"]
    g = x - W.x_star(w.A.shape[0], w.seed)
    r = adjoint.adjoint_from_forward(out["split"], out["M"], out["Y"][:, 1:], g, eps=1e-12)
    lam_d = np.linalg.solve(w.A.toarray().T, g)
    assert r["status"] == "converged"
    assert np.linalg.norm(r["lam"] - lam_d) <= 1e-9 * np.linalg.norm(lam_d)
    a = adjoint.adjoint(out["split"], out["M"], x, g, eps=1e-12)
    assert np.linalg.norm(r["lam"] - a["lam"]) <= 1e-9 * np.linalg.norm(lam_d)
    G = adjoint.grad_A_values(w.A, r["lam"], x)
    lhs = float(np.dot(w.A.data, G))
    assert abs(lhs + r["lam"] @ w.b) <= 1e-9 * abs(r["lam"] @ w.b)


def test_adjoint_from_forward_residual_at_eps():
    """At eps = 1e-8 (W from an eps = 1e-8 forward solve) the reported rr is the
    true adjoint residual and below eps, for BiCGStab and GMRES(20)."""
    from tests import pins
    for name, kw in (("c1", {}), ("c2", dict(dims=(10, 10, 10), s=4, density=0.2))):
        w = W.make(1 if name == "c1" else 2, **kw)
        for method in ("bicgstab", "gmres"):
            out = pipeline.run(w.A, w.b, kind="A2", drop="none", eps=1e-8, method=method, restart=20)
            g = out["x"] - W.x_star(w.A.shape[0], w.seed)

            def fn(S, M, Wm, gg, eps):
                return adjoint.adjoint_from_forward(S, M, Wm, gg, eps=eps, method=method, restart=20)
            pins.check_adjoint_reported_residual(fn, w.A, out["split"], out["M"], out["Y"][:, 1:], g, 1e-8)


def test_adjoint_from_forward_zero_gradient():
    w, out = _problem()
    r = adjoint.adjoint_from_forward(out["split"], out["M"], out["Y"][:, 1:], np.zeros(w.A.shape[0]))
    assert r["iters"] == 0 and not r["lam"].any() and r["status"] == "converged"
