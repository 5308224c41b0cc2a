"""Plant plausible mistakes in copies of oracle functions; the pins must catch each one.

Nothing here touches the GPU: every mistake is planted in the CPU oracle.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import lsq, pattern as opat, smw, spai, split as osplit
from tests import pins
from tests.test_oracle_split import _matrix_like, _table3


def _tie_matrix():
    n = 30
    A = sp.lil_matrix((n, n))
    for i in range(n):
        A[i, i] = 4.0
    for i in [8, 12] + list(range(20, 30)):
        A[i, 10] = 1.0
    return sp.csr_matrix(A)


def _split_variant(mode):
    def f(A, dense_factor=10.0, keep=None, rule="nearest"):
        A = sp.csr_matrix(A)
        n = A.shape[0]
        if mode == "round_p":
            p_override = int(round(A.nnz / n))
        elif mode == "ge_threshold":
            p_override = None
        else:
            p_override = None
        S = osplit.split(A, dense_factor if mode != "ge_threshold" else dense_factor - 1e-9,
                         keep=keep, rule=rule)
        if p_override is not None:
            S.p = p_override
        if mode == "tie_larger":
            # redo the selection with ties going to the larger row index
            C = A.tocsc()
            C.sort_indices()
            kk = S.keep
            At = A.toarray()
            Ud = np.zeros((n, S.s))
            for d, j in enumerate(S.D):
                rows = [i for i in C.indices[C.indptr[j]:C.indptr[j + 1]] if i != j]
                rows.sort(key=lambda i: (abs(i - j), -i))
                for i in rows[kk - 1:]:
                    Ud[i, d] = At[i, j]
                    At[i, j] = 0.0
            S.At = sp.csr_matrix(At)
            S.U = sp.csc_matrix(Ud)
        if mode == "keep_minus_one":
            return osplit.split(A, dense_factor, keep=max(1, (keep or A.nnz // n) - 1), rule=rule)
        return S
    return f


@pytest.mark.parametrize("mode", ["round_p", "ge_threshold"])
def test_table3_catches(mode):
    f = _split_variant(mode)
    caught = False
    for row in _table3():
        A = _matrix_like(row)
        S = f(A, keep=row["keep"])
        if S.p != row["p"] or S.s != row["s"]:
            caught = True
            break
    assert caught


@pytest.mark.parametrize("mode", ["tie_larger", "keep_minus_one"])
def test_split_bruteforce_catches(mode):
    f = _split_variant(mode)
    A = _tie_matrix()
    with pytest.raises(AssertionError):
        # the brute-force pin on the tie matrix (p = 1, so the threshold factor is 2)
        pins.check_split_bruteforce(lambda M, keep=None: f(M, 2.0, keep=keep), A, keep=2,
                                    dense_factor=2.0)


def test_pattern_transposed_operand_caught():
    At = W.random_sparse(50, 0.05, 0)

    def wrong(C, k):
        R = sp.csr_matrix(C)
        out = set()
        for j in R.indices[R.indptr[k]:R.indptr[k + 1]]:
            out.update(R.indices[R.indptr[j]:R.indptr[j + 1]].tolist())
        return np.array(sorted(out))
    with pytest.raises(AssertionError):
        pins.check_pattern_A2_bruteforce(wrong, At)


def test_lsq_missing_rows_caught():
    w = W.make(2, dims=(7, 7, 7), s=2, density=0.2)
    S = osplit.split(w.A)
    C = opat.as_csc(S.At)

    def wrong(C, J, k):
        I = opat.col_rows(C, k)          # rows of column k only, not of A~(:, J)
        pos = {int(i): t for t, i in enumerate(I)}
        Ah = np.zeros((len(I), len(J)))
        for c, j in enumerate(J):
            for i, v in zip(C.indices[C.indptr[j]:C.indptr[j + 1]], C.data[C.indptr[j]:C.indptr[j + 1]]):
                if int(i) in pos:
                    Ah[pos[int(i)], c] = v
        e = (I == k).astype(float)
        m = np.linalg.lstsq(Ah, e, rcond=None)[0]
        return I, m, float(np.linalg.norm(Ah @ m - e))
    k = 171
    with pytest.raises(AssertionError):
        pins.check_ls_optimality(wrong, S.At, opat.pattern_A2(C, k), k)


def test_lsq_transposed_block_caught():
    At = W.random_sparse(20, 0.15, 1, diag=2.0)

    def wrong(C, J, k):
        I, m, res = lsq.solve_column(sp.csc_matrix(sp.csr_matrix(C).T), J, k)
        return I, m, res
    with pytest.raises(AssertionError):
        pins.check_full_pattern_inverse(wrong, At)


def test_spai_gain_without_norm_caught():
    w = W.make(3, n=300, s=2, density=0.2)
    S = osplit.split(w.A)
    C = opat.as_csc(S.At)
    k = 5
    J = opat.pattern_A(C, k)
    I, m, res = lsq.solve_column(C, J, k)
    r = lsq.dense_block(C, I, J) @ m - (I == k)

    def wrong(C, R, cn2, J, I, r):
        return spai.candidate_gains(C, R, np.ones_like(cn2), J, I, r)
    with pytest.raises(AssertionError):
        pins.check_spai_gains(wrong, S.At, J, I, r)


@pytest.mark.parametrize("mistake", ["sign", "transposed_rows"])
def test_smw_mistakes_caught(mistake):
    w = W.make(1)
    S = osplit.split(w.A)
    U = S.U.toarray()

    def wrong(y, Wm, D):
        s = len(D)
        K = np.eye(s) + (Wm[D, :] if mistake == "sign" else Wm[D, :].T)
        z = np.linalg.solve(K, y[D])
        x = y + Wm @ z if mistake == "sign" else y - Wm @ z
        return x, z, float(np.linalg.norm(z))
    with pytest.raises(AssertionError):
        pins.check_smw_exact(wrong, w.A, S.At, U, S.D, w.b)


def _bicgstab_mutant(old, new):
    """A copy of oracle.krylov.bicgstab with one textual change (the planted mistake)."""
    import inspect
    import textwrap

    from oracle import krylov
    src = textwrap.dedent(inspect.getsource(krylov.bicgstab))
    assert src.count(old) == 1, old
    ns = dict(vars(krylov))
    exec(compile(src.replace(old, new), "<bicgstab mutant>", "exec"), ns)
    return ns["bicgstab"]


_RESTART_MISTAKES = {
    "old_rhat": ("        rhat = r.copy()\n        rho_old = alpha = omega = 1.0\n",
                 "        rho_old = alpha = omega = 1.0\n"),
    "keep_p_v": ("        v = np.zeros(n)\n        p = np.zeros(n)\n        note(", "        note("),
    "keep_v": ("        v = np.zeros(n)\n        p = np.zeros(n)\n", "        p = np.zeros(n)\n"),
}


@pytest.mark.parametrize("mistake", sorted(_RESTART_MISTAKES))
def test_bicgstab_restart_mistakes_caught(mistake):
    f = _bicgstab_mutant(*_RESTART_MISTAKES[mistake])
    A = W.random_sparse(150, 0.04, 1, diag=2.0)
    b = A @ np.ones(150)
    with pytest.raises(AssertionError):
        pins.check_bicgstab_restart_is_fresh_start(f, A, sp.identity(150, format="csr"), b,
                                                   1e-11 * np.linalg.norm(b), 4)


def test_bicgstab_endless_restarts_caught():
    f = _bicgstab_mutant("        return restarts <= 1\n", "        return True\n")
    A = W.random_sparse(150, 0.04, 5, diag=2.0)
    b = A @ np.ones(150)
    with pytest.raises(AssertionError):
        pins.check_bicgstab_second_breakdown(f, A, sp.identity(150, format="csr"), b,
                                             1e-11 * np.linalg.norm(b), 3, 4)


_REPLACE_MISTAKES = {
    # the recursive residual is kept after a failed true-residual check
    "no_replacement": ("            r_rec, r = r, rt\n", "            r_rec = r\n"),
    # sign of the true residual
    "sign": ("            r_rec, r = r, rt\n", "            r_rec, r = r, -rt\n"),
    # convergence declared on the recursive residual at the full step
    "recursive_accept": ("            if np.linalg.norm(rt) < thr:\n                return x, it, \"converged\"\n",
                         "            return x, it, \"converged\"\n"),
}


@pytest.mark.parametrize("mistake", sorted(_REPLACE_MISTAKES))
def test_bicgstab_replacement_mistakes_caught(mistake):
    f = _bicgstab_mutant(*_REPLACE_MISTAKES[mistake])
    A = W.random_sparse(60, 0.08, 13, diag=0.5)
    b = A @ np.ones(60)
    with pytest.raises(AssertionError):
        pins.check_bicgstab_replacement(f, A, sp.identity(60, format="csr"), b, 1e-14 * np.linalg.norm(b))


@pytest.mark.parametrize("mistake", ["inverted_alpha", "not_scaled_back"])
def test_equilibration_mistakes_caught(mistake):
    from oracle import pipeline as opipe
    from tests.test_oracle_krylov import check_equilibration
    w = W.make(2, dims=(9, 8, 7), s=3, density=0.3)

    def wrong(A, b, equilibrate=False):
        alpha = opipe.equilibration_factor(A, b)
        if mistake == "inverted_alpha":
            out = opipe.run(A, b / alpha / alpha if alpha else b, kind="A2", drop="abs", tau=1e-3)
            out["x"] = out["x"] * alpha * alpha
            out["rr"] = float(np.linalg.norm(b - A @ out["x"]) / np.linalg.norm(b))
            return out
        out = opipe.run(A, b, kind="A2", drop="abs", tau=1e-3, equilibrate=True)
        out["x"] = out["x"] * out["alpha"]
        out["rr"] = float(np.linalg.norm(b - A @ out["x"]) / np.linalg.norm(b))
        return out
    with pytest.raises(AssertionError):
        check_equilibration(wrong, w.A, w.b)


def _gmres_mutant(old, new):
    """A copy of oracle.krylov.gmres with one textual change (the planted mistake)."""
    import inspect
    import textwrap

    from oracle import krylov
    src = textwrap.dedent(inspect.getsource(krylov.gmres))
    assert src.count(old) == 1, old
    ns = dict(vars(krylov))
    exec(compile(src.replace(old, new), "<gmres mutant>", "exec"), ns)
    return ns["gmres"]


_GMRES_MISTAKES = {
    "givens_sign": ("g[j + 1] = -sn[j] * g[j]", "g[j + 1] = sn[j] * g[j]"),
    "no_back_substitution": ("y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]", "y[i] = g[i] / H[i, i]"),
    "restart_from_rhs": ("r = rhs - A @ x", "r = rhs.copy()"),
    "stale_rotations": ("H[i + 1, j] = -sn[i] * a + cs[i] * b", "H[i + 1, j] = b"),
    "wrong_basis_vector": ("w = w - H[i, j] * V[i]", "w = w - H[i, j] * V[0]"),
}


@pytest.mark.parametrize("mistake", sorted(_GMRES_MISTAKES))
def test_gmres_mistakes_caught(mistake):
    f = _gmres_mutant(*_GMRES_MISTAKES[mistake])
    A = W.random_sparse(80, 0.04, 4, diag=3.0)
    Ad = A.toarray()
    Minv = np.linalg.inv(Ad)
    Minv[np.abs(Minv) < 0.05 * np.abs(Minv).max()] = 0.0
    b = np.random.default_rng(4).standard_normal(80)
    with pytest.raises(AssertionError):
        pins.check_gmres_cycles_minimise(f, A, sp.csr_matrix(Minv), b, 5, 2)


_CORRECTION_MISTAKES = {
    "K_not_transposed": ("z = np.linalg.solve(K.T, W.T @ v)", "z = np.linalg.solve(K, W.T @ v)"),
    "plus_sign": ("rhs[D] -= z", "rhs[D] += z"),
    "no_K": ("z = np.linalg.solve(K.T, W.T @ v)", "z = W.T @ v"),
}


def _adjoint_mutant(fn, old, new):
    """A copy of an oracle.adjoint function with one textual change."""
    import inspect
    import textwrap

    from oracle import adjoint
    src = textwrap.dedent(inspect.getsource(getattr(adjoint, fn)))
    assert src.count(old) == 1, old
    ns = dict(vars(adjoint))
    exec(compile(src.replace(old, new), "<adjoint mutant>", "exec"), ns)
    return ns[fn]


@pytest.mark.parametrize("mistake", sorted(_CORRECTION_MISTAKES))
def test_forward_correction_mistakes_caught(mistake):
    f = _adjoint_mutant("forward_correction", *_CORRECTION_MISTAKES[mistake])
    w = W.make(1, dims=(14, 16), s=4, density=0.3)
    S = osplit.split(w.A)
    g = np.random.default_rng(7).standard_normal(w.A.shape[0])
    with pytest.raises(AssertionError):
        pins.check_forward_correction_exact(f, w.A, S.At, S.U, S.D, g)


@pytest.mark.parametrize("mistake", ["residual_without_U", "no_accumulation"])
def test_adjoint_from_forward_mistakes_caught(mistake):
    from oracle import pipeline
    old, new = {"residual_without_U": ("rho[D] -= U.T @ lam", "pass"),
                "no_accumulation": ("lam = lam + X[:, 0]", "lam = X[:, 0]")}[mistake]
    f = _adjoint_mutant("adjoint_from_forward", old, new)
    w = W.make(1)
    out = pipeline.run(w.A, w.b, kind="A2", drop="none", eps=1e-8)
    g = out["x"] - W.x_star(w.A.shape[0], w.seed)
    with pytest.raises(AssertionError):
        pins.check_adjoint_reported_residual(f, w.A, out["split"], out["M"], out["Y"][:, 1:], g, 1e-8)
