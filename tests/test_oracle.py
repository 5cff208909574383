"""Pins of the float64 CPU oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own code.

* exact rational pseudoinverse by another formula (tiny integer matrices)
* SVD pseudoinverse on inputs with a clear rank gap
* closed forms: full column rank (Section 1), G = U V, G = P diag(s) Q'
* the four Penrose conditions with the paper's 2e-10 bound on its own
  matrix family (Section 3, Table 1)
* exact ranks of constructions, strict pivot test, invariances, edge cases
* planted mistakes in the oracle are caught by these pins
"""
import json
import os

import numpy as np
import pytest

from oracle import exact
from oracle import geninv_ref as o
from paper_0804_4809_amd import workloads as w


def _int_cases():
    rng = np.random.default_rng(11)
    cases = []
    # tall, rank 3 of 5, one zero column
    G = rng.integers(-3, 4, size=(7, 3)) @ rng.integers(-3, 4, size=(3, 5))
    G[:, 2] = 0
    cases.append(G)
    # duplicate columns and a column that is a sum of two earlier ones
    B = rng.integers(-4, 5, size=(8, 4))
    cases.append(np.column_stack([B[:, 0], B[:, 1], B[:, 0], B[:, 2], B[:, 1] + B[:, 2], B[:, 3]]))
    # wide (transpose branch), rank 2
    cases.append(rng.integers(-2, 3, size=(3, 2)) @ rng.integers(-2, 3, size=(2, 6)))
    # rank one
    cases.append(np.outer([1, 2, -1, 3], [2, 0, -1]))
    # full column rank
    cases.append(np.array([[2, 1, 0], [1, 3, 1], [0, 1, 4], [1, 0, 1]]))
    # square singular
    cases.append(np.array([[1, 2, 3], [4, 5, 6], [7, 8, 9]]))
    # single column and single row
    cases.append(np.array([[3], [4]]))
    cases.append(np.array([[1, -2, 2]]))
    return cases


# ---------------------------------------------------------------------------
# the exact oracle is itself pinned by exact Penrose identities
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ci", range(len(_int_cases())))
def test_exact_oracle_satisfies_penrose_exactly(ci):
    G = _int_cases()[ci]
    Y, r, piv, d = exact.exact_pinv(G)
    assert exact.is_exact_pinv(G, Y)
    assert r == np.linalg.matrix_rank(G.astype(float))


@pytest.mark.parametrize("ci", range(len(_int_cases())))
def test_oracle_matches_exact_rational(ci):
    G = _int_cases()[ci]
    Yx, rx, pivx, dx = exact.exact_pinv(G if G.shape[0] >= G.shape[1] else G.T)
    res = o.geninv(G.astype(np.float64))
    assert res.rank == rx
    assert list(res.piv) == list(pivx)
    Yref = exact.to_float(Yx)
    if G.shape[0] < G.shape[1]:
        Yref = Yref.T
    assert o.rel_fro(res.Y, Yref) <= 1e-12
    # accepted pivots equal the exact squared distance to the span of the
    # earlier accepted columns; rejected ones are zero up to rounding
    dx = np.array([float(v) for v in dx])
    acc = np.zeros(len(dx), bool)
    acc[pivx] = True
    assert np.allclose(res.d[acc], dx[acc], rtol=1e-10, atol=0)
    assert np.all(np.abs(res.d[~acc]) <= res.tol)


# ---------------------------------------------------------------------------
# textbook routine and closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,r,seed", [(30, 12, 7, 0), (60, 40, 40, 1), (25, 25, 10, 2), (9, 20, 4, 3)])
def test_oracle_vs_svd_pinv(m, n, r, seed):
    G, _ = w.lowrank_uv(m, n, r, seed)
    res = o.geninv(G)
    assert res.rank == r
    s = np.linalg.svd(G, compute_uv=False)
    rcond = np.sqrt(s[r - 1] * (s[r] if r < len(s) else 0.0)) / s[0] if r < len(s) else 1e-14
    assert o.rel_fro(res.Y, np.linalg.pinv(G, rcond=rcond)) <= 1e-10


def test_c1_vs_svd_pinv():
    G, F = w.c1_problem(0)
    res = o.geninv(G)
    assert res.rank == 40
    assert o.rel_fro(res.Y, np.linalg.pinv(G, rcond=1e-10)) <= 1e-10


def test_full_column_rank_closed_form():
    # Section 1: with rank n, G^+ = (G'G)^-1 G'
    rng = np.random.default_rng(3)
    G = rng.standard_normal((40, 15))
    res = o.geninv(G)
    assert res.rank == 15
    ref = np.linalg.solve(G.T @ G, G.T)
    assert o.rel_fro(res.Y, ref) <= 1e-12


def test_full_rank_factorization_closed_form():
    # G = U V with U, V of full rank r: G^+ = V'(V V')^-1 (U'U)^-1 U'
    rng = np.random.default_rng(4)
    U = rng.standard_normal((50, 9))
    V = rng.standard_normal((9, 21))
    G = U @ V
    ref = V.T @ np.linalg.solve(V @ V.T, np.linalg.solve(U.T @ U, U.T))
    res = o.geninv(G)
    assert res.rank == 9
    assert o.rel_fro(res.Y, ref) <= 1e-10


def test_svd_family_closed_form():
    # G = P diag(s) Q' with orthonormal P, Q: G^+ = Q diag(1/s) P'
    G, _, P, s, Q = w.svd_family(300, 80, 60, 1e-2, seed=5)
    res = o.geninv(G)
    assert res.rank == 60
    ref = (Q / s[None, :]) @ P.T
    # the Gram route squares the condition number (1e4 here): rounding floor ~ kappa^2 u
    assert o.rel_fro(res.Y, ref) <= 1e-9


def test_rank_one_closed_form():
    u = np.array([1.0, -2.0, 0.5, 3.0])
    v = np.array([2.0, 1.0, -1.0])
    G = np.outer(u, v)
    ref = np.outer(v, u) / (u @ u) / (v @ v)
    res = o.geninv(G)
    assert res.rank == 1
    assert o.rel_fro(res.Y, ref) <= 1e-14


# ---------------------------------------------------------------------------
# the paper's own accuracy claim on its own matrix family (Section 3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [32, 64, 128, 256, 512])
def test_table1_family_penrose_bound(n, golden_dir):
    with open(os.path.join(golden_dir, "paper_table1.json")) as f:
        bound = json.load(f)["penrose_max_abs_bound"]
    G = w.table1(n, seed=n)
    res = o.geninv(G)
    assert res.rank == 7 * n // 8
    errs = o.penrose_errors(G, res.Y)
    assert max(errs.values()) <= bound, errs


# ---------------------------------------------------------------------------
# rank and pivot decisions
# ---------------------------------------------------------------------------
def test_strict_pivot_comparison():
    # Appendix: a column is kept only if its updated pivot is strictly above tol
    G = np.diag([3.0, 2.0])                        # A = diag(9, 4)
    assert o.geninv(G, tol=4.0).rank == 1          # second pivot 4 == tol: dropped
    assert o.geninv(G, tol=3.999).rank == 2
    G = np.diag([2.0, 3.0])                        # A = diag(4, 9)
    res = o.geninv(G, tol=4.0)                     # first pivot 4 == tol: dropped
    assert res.rank == 1 and list(res.piv) == [1]


def test_default_tol_is_1e9_min_positive_diag():
    G = np.diag([3.0, 0.0, 0.5, 10.0])
    res = o.geninv(G)
    assert res.tol == pytest.approx(0.25e-9, rel=1e-15)
    assert res.rank == 3 and list(res.piv) == [0, 2, 3]


def test_zero_matrix_gives_rank_zero():
    for shape in [(5, 3), (3, 5), (4, 4)]:
        res = o.geninv(np.zeros(shape))
        assert res.rank == 0 and res.tol is None
        assert res.Y.shape == shape[::-1] and not res.Y.any()


def test_empty_shapes():
    for shape in [(0, 3), (4, 0), (0, 0)]:
        res = o.geninv(np.zeros(shape))
        assert res.rank == 0 and res.Y.shape == shape[::-1]


def test_rbf_duplicates_rejected():
    G, F, idx = w.rbf_design(600, 3, 40, 12, 0.4, seed=7, k=2)
    res = o.geninv(G)
    seen = set()
    dup_cols = []
    for j, c in enumerate(idx):
        if c in seen:
            dup_cols.append(j)
        seen.add(c)
    assert len(dup_cols) == 12
    assert not set(dup_cols) & set(res.piv.tolist())
    assert res.rank <= 40


def test_exact_rank_constructions():
    G, _ = w.c1_problem(0)
    assert o.geninv(G).rank == 40
    B = w.batch_lowrank(12, seed=1, m_hi=200, n_hi=40)
    for b in range(12):
        res = o.geninv(B.G[b].astype(np.float64))
        assert res.rank == B.rank[b]


def test_cholesky_factor_structure():
    G, _ = w.lowrank_uv(40, 18, 11, seed=9)
    A = o.gram(G)
    L, r, piv, d = o.full_rank_cholesky(A, o.paper_tol(A))
    assert r == 11
    assert np.linalg.norm(L @ L.T - A) <= 1e-13 * np.linalg.norm(A)
    for c in range(r):
        assert L[piv[c], c] > 0
        assert not L[: piv[c], c].any()
    assert np.all(np.diff(piv) > 0)


def test_spd_inverse_closed_form():
    B = np.array([[4.0, 2.0], [2.0, 3.0]])
    ref = np.array([[3.0, -2.0], [-2.0, 4.0]]) / 8.0
    assert np.allclose(o.spd_inverse(B), ref, rtol=1e-15, atol=1e-16)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((30, 30))
    S = X @ X.T + 30 * np.eye(30)
    assert np.linalg.norm(o.spd_inverse(S) @ S - np.eye(30)) <= 1e-13


# ---------------------------------------------------------------------------
# invariances and least squares
# ---------------------------------------------------------------------------
def test_transpose_invariance():
    G, _ = w.lowrank_uv(35, 14, 9, seed=12)
    a = o.geninv(G)
    b = o.geninv(np.ascontiguousarray(G.T))
    assert b.transposed and list(a.piv) == list(b.piv)
    assert o.rel_fro(b.Y, a.Y.T) <= 1e-12


def test_scaling_invariance():
    G, _ = w.lowrank_uv(35, 14, 9, seed=13)
    a = o.geninv(G)
    b = o.geninv(8.0 * G)          # power of two: exact scaling of every step
    assert list(a.piv) == list(b.piv)
    assert o.rel_fro(b.Y * 8.0, a.Y) <= 1e-15


def test_lstsq_min_norm_solution():
    G, F = w.lowrank_uv(80, 30, 17, seed=14, k=3)
    W, res = o.lstsq(G, F)
    # normal equations: the residual is orthogonal to range(G)
    R = G @ W - F
    assert np.linalg.norm(G.T @ R) <= 1e-10 * np.linalg.norm(G) * np.linalg.norm(F)
    # minimum norm: W lies in range(G'), so projecting onto it changes nothing
    assert np.linalg.norm(res.Y @ (G @ W) - W) <= 1e-10 * np.linalg.norm(W)
    # another least-squares solution (W + null vector) has a larger norm
    null = np.linalg.svd(G)[2][17:].T
    W2 = W + null[:, :1] @ np.ones((1, 3))
    assert np.linalg.norm(G @ W2 - F) == pytest.approx(np.linalg.norm(R), rel=1e-9)
    assert np.linalg.norm(W2) > np.linalg.norm(W)


def test_matlab_stale_entries_no_effect_on_exact_rank():
    G, _ = w.c1_problem(0)
    a = o.geninv(G)
    b = o.geninv(G, matlab_stale=True)
    assert a.rank == b.rank
    assert o.rel_fro(b.Y, a.Y) <= 1e-9


# ---------------------------------------------------------------------------
# planted mistakes in the oracle are caught by the pins above
# ---------------------------------------------------------------------------
def _pins_pass():
    """Run a compact subset of the pins above; True if all hold."""
    try:
        for ci in (0, 1, 2, 5):
            G = _int_cases()[ci]
            Yx, rx, pivx, _ = exact.exact_pinv(G if G.shape[0] >= G.shape[1] else G.T)
            Yref = exact.to_float(Yx)
            if G.shape[0] < G.shape[1]:
                Yref = Yref.T
            res = o.geninv(G.astype(np.float64))
            if res.rank != rx or o.rel_fro(res.Y, Yref) > 1e-12:
                return False
        if o.geninv(np.diag([3.0, 2.0]), tol=4.0).rank != 1:
            return False
        G = w.table1(64, seed=64)
        res = o.geninv(G)
        if max(o.penrose_errors(G, res.Y).values()) > 2e-10:
            return False
        return True
    except Exception:
        return False


def test_pins_accept_true_oracle():
    assert _pins_pass()


def _mutant_cholesky(kind):
    def f(A, tol, matlab_stale=False):
        n = A.shape[0]
        L = np.zeros((n, n))
        piv, d, r = [], np.zeros(n), 0
        for k in range(n):
            if kind == "dropped_update":
                v = A[k:, k].copy()
            elif kind == "sign":
                v = A[k:, k] + L[k:, :r] @ L[k, :r]
            elif kind == "wrong_index":
                v = A[k:, k] - L[k:, :r] @ L[min(k + 1, n - 1), :r]
            else:
                v = A[k:, k] - L[k:, :r] @ L[k, :r]
            d[k] = v[0]
            keep = (v[0] >= tol) if kind == "non_strict" else (v[0] > tol)
            if tol is not None and keep:
                s = np.sqrt(v[0])
                L[k, r] = s
                L[k + 1:, r] = v[1:] / (s * s if kind == "no_sqrt_scale" else s)
                piv.append(k)
                r += 1
        return L[:, :r].copy(), r, np.array(piv, dtype=np.int64), d
    return f


@pytest.mark.parametrize("kind", ["dropped_update", "sign", "wrong_index", "no_sqrt_scale", "non_strict"])
def test_pins_catch_cholesky_mutants(kind, monkeypatch):
    monkeypatch.setattr(o, "full_rank_cholesky", _mutant_cholesky(kind))
    assert not _pins_pass()


def test_pins_catch_uninverted_gram_of_factor(monkeypatch):
    # M = L'L instead of (L'L)^-1
    monkeypatch.setattr(o, "spd_inverse", lambda B: np.array(B, dtype=np.float64))
    assert not _pins_pass()


def test_pins_catch_transposed_gram(monkeypatch):
    # A = G G' where the method needs G'G (differs for square non-normal G)
    monkeypatch.setattr(o, "gram", lambda G: np.asarray(G, np.float64) @ np.asarray(G, np.float64).T
                        if G.shape[0] == G.shape[1] else np.asarray(G, np.float64).T @ np.asarray(G, np.float64))
    assert not _pins_pass()
