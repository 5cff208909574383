"""Pins of the oracle's checkers and of its Newton-Schulz step.

The checkers decide the verdict of every float64 parity test, so each is
pinned to facts fixed by mathematics, not to its own code:

* ``penrose_errors`` (Section 1, the four Penrose conditions; Section 3 uses
  their max-abs entries as the accuracy criterion): closed-form 2 x 2 and
  1 x 2 cases in which exactly one condition fails by a known amount;
* ``self_spread`` (rounding sensitivity of the method on an input): exactly
  zero on integer inputs whose Gram matrix every summation order forms
  exactly, and within a factor of ten of the oracle's true forward error,
  measured against the closed-form pseudoinverse of G = P diag(s) Q';
* ``ambiguity_band`` (decisions within rounding of tol): between the
  classical Cholesky backward-error term and an analytic upper bound on a
  2 x 2 matrix whose second pivot is placed at tol (1 + 1e-3), tiny for a
  pivot far from tol, invariant under power-of-two scaling, and wide
  enough to cover the pivot's change under random rounding-size
  perturbations of A;
* ``gram_extended``: equal to the exact integer Gram matrix rounded once;
* ``newton_schulz_step``: G^+ is a fixed point, the residual on the range of
  G is squared by each step, and the factored form on P gives the same
  iterates (X = P G').

The last tests plant a mistake in each checker and require these pins to
fail.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact
from oracle import geninv_ref as o

U = np.finfo(np.float64).eps / 2


# ---------------------------------------------------------------------------
# penrose_errors
# ---------------------------------------------------------------------------
def _penrose_cases():
    t = 0.375
    return [
        # G = I, Y = diag(1, 2): G Y G - G = diag(0, 1), Y G Y - Y = diag(0, 2),
        # both products symmetric
        (np.eye(2), np.diag([1.0, 2.0]), {"GYG-G": 1.0, "YGY-Y": 2.0, "(GY)'-GY": 0.0, "(YG)'-YG": 0.0}),
        # G = [1 0], Y = [1; t]: G Y = 1, Y G = [[1, 0], [t, 0]] is not symmetric
        (np.array([[1.0, 0.0]]), np.array([[1.0], [t]]),
         {"GYG-G": 0.0, "YGY-Y": 0.0, "(GY)'-GY": 0.0, "(YG)'-YG": t}),
        # G = [1; 0], Y = [1 t]: G Y = [[1, t], [0, 0]] is not symmetric
        (np.array([[1.0], [0.0]]), np.array([[1.0, t]]),
         {"GYG-G": 0.0, "YGY-Y": 0.0, "(GY)'-GY": t, "(YG)'-YG": 0.0}),
        # the exact pseudoinverse: every condition holds exactly
        (np.array([[2.0, 0.0], [0.0, 0.0]]), np.array([[0.5, 0.0], [0.0, 0.0]]),
         {"GYG-G": 0.0, "YGY-Y": 0.0, "(GY)'-GY": 0.0, "(YG)'-YG": 0.0}),
    ]


@pytest.mark.parametrize("ci", range(4))
def test_penrose_errors_closed_forms(ci):
    G, Y, want = _penrose_cases()[ci]
    got = o.penrose_errors(G, Y)
    assert set(got) == set(want)
    for key, val in want.items():
        assert got[key] == val, (key, got[key], val)


def test_penrose_errors_one_wrong_entry():
    # exact G^+ of an integer matrix with one entry of Y moved by delta:
    # G (Y + delta e_i e_j') G - G = delta G[:, i] G[j, :]
    G = np.array([[1, 2, 0], [0, 1, 1], [1, 3, 1], [2, 0, 1]])
    Yx, _, _, _ = exact.exact_pinv(G)
    Y = exact.to_float(Yx)
    delta = 2.0 ** -10
    i, j = 1, 2
    Yb = Y.copy()
    Yb[i, j] += delta
    got = o.penrose_errors(G.astype(float), Yb)
    want = delta * np.max(np.abs(np.outer(G[:, i], G[j, :])))
    assert abs(got["GYG-G"] - want) <= 1e-12 * want
    base = o.penrose_errors(G.astype(float), Y)
    assert max(base.values()) <= 1e-14


# ---------------------------------------------------------------------------
# self_spread
# ---------------------------------------------------------------------------
def test_self_spread_zero_on_exact_gram():
    # small integers: every Gram entry is an exact float64 sum in any order,
    # so all the Gram matrices compared are identical
    rng = np.random.default_rng(3)
    G = (rng.integers(-3, 4, size=(60, 6)) @ rng.integers(-3, 4, size=(6, 9))).astype(float)
    assert o.self_spread(G) == 0.0


@pytest.mark.parametrize("kappa", [1e2, 1e3, 1e4])
def test_self_spread_tracks_true_forward_error(kappa):
    rng = np.random.default_rng(int(np.log10(kappa)))
    m, n = 3000, 40
    P, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -np.log10(kappa), n)
    G = (P * s) @ Q.T
    res = o.geninv(G)
    assert res.rank == n
    true_err = o.rel_fro(res.Y, (Q / s) @ P.T)     # closed form G^+ = Q diag(1/s) P'
    spread = o.self_spread(G, base=res)
    assert true_err / 10 <= spread <= 10 * true_err, (spread, true_err)


def test_self_spread_small_on_orthonormal_columns():
    rng = np.random.default_rng(9)
    P, _ = np.linalg.qr(rng.standard_normal((500, 30)))
    assert o.self_spread(P) <= 1e-14


# ---------------------------------------------------------------------------
# ambiguity_band
# ---------------------------------------------------------------------------
def _near_tol_2x2(scale=1.0):
    a, b, tol = 1.0, 0.75, 1e-9
    c = b * b / a + tol * (1 + 1e-3)        # second pivot c - b^2/a at tol (1 + 1e-3)
    A = np.array([[a, b], [b, c]]) * scale
    return A, tol * scale, a, b, c


def test_ambiguity_band_width_near_tol():
    A, tol, a, b, c = _near_tol_2x2()
    band = o.ambiguity_band(A, tol)
    n = 2
    eps = 2 * np.sqrt(n) * U + 2 * U       # relative perturbation, plus its own rounding
    # d2 = c - b^2/a: |d d2| <= eps (c + 2 b^2/a + b^2/a) for relative
    # perturbations eps of a, b, c; band = (4 max|d d2| + 2 (n+1) u c) / tol
    upper = (4 * eps * (c + 3 * b * b / a) + 2 * (n + 1) * U * c) / tol
    lower = 2 * (n + 1) * U * c / tol
    assert lower <= band[1] <= upper, (lower, band[1], upper)
    # the pivot at tol (1 + 1e-3) lies outside the band: a decision there is not ambiguous
    d = o.full_rank_cholesky(A, tol)[3]
    assert abs(d[1] / tol - 1) > band[1]


def test_ambiguity_band_tiny_far_from_tol():
    A = np.diag([1.0, 0.5])
    tol = 1e-9
    band = o.ambiguity_band(A, tol)
    # a pivot equal to its diagonal entry moves by its own relative
    # perturbation only: band = (4 eps + 2 (n+1) u) A_kk / tol at most
    eps = 2 * np.sqrt(2) * U + 2 * U
    dA = np.diag(A)
    assert np.all(band <= (4 * eps + 6 * U) * dA / tol)
    assert np.all(band >= 6 * U * dA / tol)
    # in tol units: about 1e-6 against a distance |d / tol - 1| of ~1e9
    assert np.all(band < 1e-14 * np.abs(dA / tol - 1))


def test_ambiguity_band_scale_invariant():
    A, tol, *_ = _near_tol_2x2()
    b1 = o.ambiguity_band(A, tol)
    b2 = o.ambiguity_band(A * 2.0 ** 40, tol * 2.0 ** 40)
    assert np.array_equal(b1, b2)


def test_ambiguity_band_covers_rounding_perturbations():
    # the band must cover the pivot changes that rounding-size (u relative)
    # perturbations of A actually cause, here on a 12 x 12 Gram matrix whose
    # last pivots fall near tol
    rng = np.random.default_rng(4)
    B = rng.standard_normal((40, 10))
    G = np.column_stack([B, B[:, 0] + 1e-4 * rng.standard_normal(40), B[:, 1] - 2e-4 * rng.standard_normal(40)])
    A = G.T @ G
    tol = o.paper_tol(A)
    L, r, piv, d0 = o.full_rank_cholesky(A, tol)
    keep = np.zeros(12, bool)
    keep[piv] = True
    band = o.ambiguity_band(A, tol, keep)
    worst = np.zeros(12)
    for _ in range(30):
        E = rng.uniform(-1, 1, size=A.shape)
        E = np.tril(E) + np.tril(E, -1).T
        d1 = o.full_rank_cholesky(A * (1 + U * E), tol, forced=keep)[3]
        worst = np.maximum(worst, np.abs(d1 - d0) / tol)
    assert np.all(worst <= band), (worst, band)


# ---------------------------------------------------------------------------
# gram_extended
# ---------------------------------------------------------------------------
def test_gram_extended_is_exact_gram_rounded_once():
    # entries 2^27 + odd: each product needs 55 bits and the sums of eight
    # 58 bits, more than float64 holds; the 64-bit extended significand holds
    # them, so one rounding at the end gives the correctly rounded value
    rng = np.random.default_rng(0)
    Gi = (2 ** 27 + 2 * rng.integers(-2 ** 20, 2 ** 20, size=(8, 4)) + 1).astype(np.int64)
    ex = np.array([[float(Fraction(int(sum(int(Gi[k, i]) * int(Gi[k, j]) for k in range(8))))) for j in range(4)]
                   for i in range(4)])
    G = Gi.astype(np.float64)
    assert np.array_equal(o.gram_extended(G), ex)
    assert not np.array_equal(G.T @ G, ex)     # float64 products do lose bits here


# ---------------------------------------------------------------------------
# Newton-Schulz step
# ---------------------------------------------------------------------------
def test_newton_schulz_fixed_point():
    G = np.array([[1, 2, 0], [0, 1, 1], [1, 3, 1], [2, 0, 1]])
    Yx, _, _, _ = exact.exact_pinv(G)
    Y = exact.to_float(Yx)
    assert o.rel_fro(o.newton_schulz_step(Y, G.astype(float)), Y) <= 1e-14
    # rank-deficient: G^+ (not any inverse) is the fixed point
    Gr = np.array([[1, 2, 3], [2, 4, 6], [1, 0, 1]])
    Yx, _, _, _ = exact.exact_pinv(Gr)
    Yr = exact.to_float(Yx)
    assert o.rel_fro(o.newton_schulz_step(Yr, Gr.astype(float)), Yr) <= 1e-14


def test_newton_schulz_squares_the_residual():
    # X_0 = G' / ||G||_2^2: the residual E = GG^+ - G X on the range of G
    # satisfies E_{k+1} = E_k^2, so its spectral norm is squared each step
    rng = np.random.default_rng(6)
    G = rng.standard_normal((30, 8)) @ rng.standard_normal((8, 12))      # rank 8
    Gp = np.linalg.pinv(G)
    X = G.T / np.linalg.norm(G, 2) ** 2
    R = G @ Gp
    e_prev = np.linalg.norm(R - G @ X, 2)
    for _ in range(6):
        X = o.newton_schulz_step(X, G)
        e = np.linalg.norm(R - G @ X, 2)
        assert abs(e - e_prev ** 2) <= 1e-12 + 1e-9 * e_prev ** 2, (e, e_prev)
        e_prev = e
    for _ in range(12):
        X = o.newton_schulz_step(X, G)
    assert o.rel_fro(X, Gp) <= 1e-11


def test_newton_schulz_factored_form_same_iterates():
    rng = np.random.default_rng(7)
    G = rng.standard_normal((25, 6))
    A = G.T @ G
    P = np.eye(6) / np.linalg.norm(A, 2)
    X = P @ G.T
    for _ in range(4):
        P = o.newton_schulz_factored_step(P, A)
        X = o.newton_schulz_step(X, G)
        assert o.rel_fro(P @ G.T, X) <= 1e-13


# ---------------------------------------------------------------------------
# planted mistakes in the checkers are caught by the pins above
# ---------------------------------------------------------------------------
_PINS = [
    lambda: [test_penrose_errors_closed_forms(i) for i in range(4)],
    test_penrose_errors_one_wrong_entry,
    test_self_spread_zero_on_exact_gram,
    lambda: test_self_spread_tracks_true_forward_error(1e3),
    test_self_spread_small_on_orthonormal_columns,
    test_ambiguity_band_width_near_tol,
    test_ambiguity_band_tiny_far_from_tol,
    test_ambiguity_band_scale_invariant,
    test_ambiguity_band_covers_rounding_perturbations,
    test_gram_extended_is_exact_gram_rounded_once,
    test_newton_schulz_fixed_point,
    test_newton_schulz_squares_the_residual,
    test_newton_schulz_factored_form_same_iterates,
]


def _checker_pins_pass():
    for pin in _PINS:
        try:
            pin()
        except (AssertionError, ValueError, FloatingPointError, np.linalg.LinAlgError):
            return False
    return True


def test_checker_pins_accept_true_oracle():
    assert _checker_pins_pass()


_ZERO_PENROSE = {"GYG-G": 0.0, "YGY-Y": 0.0, "(GY)'-GY": 0.0, "(YG)'-YG": 0.0}


@pytest.mark.parametrize("name,mutant", [
    ("penrose_errors", lambda G, Y: dict(_ZERO_PENROSE)),
    # a transposed product in one condition
    ("penrose_errors", lambda G, Y: {**o.__dict__["_orig_penrose"](G, Y),
                                     "(YG)'-YG": float(np.max(np.abs((np.asarray(G) @ np.asarray(Y)).T
                                                                     - np.asarray(G) @ np.asarray(Y)),
                                                              initial=0.0))}),
    ("self_spread", lambda *a, **k: 1.0),
    ("self_spread", lambda *a, **k: 0.0),
    ("ambiguity_band", lambda A, tol, keep=None, **k: np.full(np.asarray(A).shape[0], 1e6)),
    ("ambiguity_band", lambda A, tol, keep=None, **k: np.zeros(np.asarray(A).shape[0])),
    ("gram_extended", lambda G: np.asarray(G, np.float64).T @ np.asarray(G, np.float64)),
    ("newton_schulz_step", lambda X, G: X - (np.asarray(X) @ np.asarray(G)) @ np.asarray(X)),
    ("newton_schulz_step", lambda X, G: np.asarray(X) - 2.0 * (np.asarray(X) @ np.asarray(G)) @ np.asarray(X)),
    ("newton_schulz_factored_step", lambda P, A: 2.0 * np.asarray(P) - np.asarray(P) @ np.asarray(A)),
])
def test_checker_pins_catch_mutants(name, mutant, monkeypatch):
    monkeypatch.setitem(o.__dict__, "_orig_penrose", o.penrose_errors)
    monkeypatch.setattr(o, name, mutant)
    assert not _checker_pins_pass()
