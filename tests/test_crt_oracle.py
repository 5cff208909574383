"""Pins of the int8 engine's reference (oracle/crt_ref.py) against facts
fixed by number theory and exact arithmetic, not by its own code.

* the moduli are pairwise coprime, at most 255, and their product M bounds
  the integer sums beta allows (and beta + 1 would not fit);
* the textbook Chinese remainder reconstruction, in Python integers, of the
  residues of the exact integer product gives that product back (the route
  the GPU takes, checked against the definition the reference uses);
* the representation error is at most half a unit of the last bit, and
  values with short mantissas are represented exactly;
* the exact integer product equals a brute-force Fraction triple loop;
* products of small integers come out exact, the Gram matrix is exactly
  symmetric, and the error against the float64 product stays within the
  representation bound.
"""
from fractions import Fraction
from math import gcd

import numpy as np
import pytest

from oracle import crt_ref as c


@pytest.mark.parametrize("N", [1, 8, 12, 14, 16, 18])
def test_moduli_pairwise_coprime_and_bounded(N):
    ps = c.moduli(N)
    assert len(ps) == N and len(set(ps)) == N
    assert all(2 <= p <= 255 for p in ps)
    assert all(gcd(a, b) == 1 for i, a in enumerate(ps) for b in ps[i + 1:])
    assert ps == sorted(ps, reverse=True)
    # greedy: every skipped integer above the smallest chosen shares a factor
    for q in range(min(ps), 256):
        if q not in ps:
            assert any(gcd(q, p) > 1 for p in ps if p > q)


@pytest.mark.parametrize("N,K", [(16, 1 << 17), (16, 8192), (14, 32768), (12, 4096), (8, 100), (16, 1)])
def test_beta_is_the_largest_that_fits(N, K):
    M = 1
    for p in c.moduli(N):
        M *= p
    b = c.beta_bits(N, K)
    assert 0 <= b <= 52
    assert 2 * K * 2 ** (2 * b) * (1 + 2 ** -20) <= M
    if b < 52:
        assert 2 * K * 2 ** (2 * b + 2) * (1 + 2 ** -20) > M


def test_sixteen_moduli_give_float64_bits_at_2_to_17():
    # the configuration the mixed form uses for double-precision results
    assert c.beta_bits(16, 1 << 17) == 52


def _crt_textbook(residues, ps):
    M = 1
    for p in ps:
        M *= p
    x = 0
    for r, p in zip(residues, ps):
        Mi = M // p
        x += r * Mi * pow(Mi, -1, p)
    x %= M
    return x - M if x > M // 2 else x


def test_textbook_crt_recovers_the_exact_product():
    rng = np.random.default_rng(1)
    N, K = 12, 300
    b = c.beta_bits(N, K)
    lim = 2 ** b
    A = rng.integers(-lim, lim + 1, size=(5, K), dtype=np.int64)
    B = rng.integers(-lim, lim + 1, size=(K, 4), dtype=np.int64)
    A[0, :] = lim                       # extreme sums of both signs
    B[:, 0] = lim
    B[:, 1] = -lim
    X = c.exact_int_product(A, B)
    ps = c.moduli(N)
    for i in range(5):
        for j in range(4):
            res = [int(X[i, j]) % p for p in ps]
            assert _crt_textbook(res, ps) == int(X[i, j])


def test_exact_int_product_brute_force():
    rng = np.random.default_rng(2)
    A = rng.integers(-(2 ** 52), 2 ** 52, size=(3, 7), dtype=np.int64)
    B = rng.integers(-(2 ** 52), 2 ** 52, size=(7, 2), dtype=np.int64)
    X = c.exact_int_product(A, B)
    for i in range(3):
        for j in range(2):
            assert X[i, j] == sum(Fraction(int(A[i, k])) * int(B[k, j]) for k in range(7))


def test_representation_error_half_unit():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 30)) * np.exp(rng.uniform(-20, 20, size=(40, 1)))
    for axis in (0, 1):
        e = c.exponents(X, axis)
        for beta in (10, 31, 52):
            R = c.int_representation(X, e, beta, axis)
            assert np.all(np.abs(R) <= 2 ** beta)
            back = np.ldexp(R.astype(np.float64), (e - beta)[:, None] if axis == 1 else (e - beta)[None, :])
            bound = np.ldexp(np.ones_like(X), (e - beta - 1)[:, None] if axis == 1 else (e - beta - 1)[None, :])
            assert np.all(np.abs(back - X) <= bound)
    # short mantissas are exact
    Y = rng.integers(-1000, 1000, size=(6, 5)).astype(np.float64) * 0.125
    e = c.exponents(Y, 1)
    R = c.int_representation(Y, e, 20, 1)
    assert np.array_equal(np.ldexp(R.astype(np.float64), (e - 20)[:, None]), Y)


def test_exponents_definition():
    X = np.array([[0.0, 0.0], [0.5, -1.0], [3.0, 0.25]])
    assert list(c.exponents(X, 1)) == [0, 1, 2]      # 0 row; max 1 < 2^1; 3 < 2^2
    assert list(c.exponents(X, 0)) == [2, 1]


def test_small_integer_products_are_exact():
    rng = np.random.default_rng(4)
    A = rng.integers(-50, 51, size=(20, 33)).astype(np.float64)
    B = rng.integers(-50, 51, size=(33, 17)).astype(np.float64)
    C, beta, _, _ = c.crt_product(A, B, 8)
    assert beta >= 7
    assert np.array_equal(C, A @ B)


def test_gram_symmetric_and_within_representation_bound():
    rng = np.random.default_rng(5)
    G = rng.standard_normal((500, 40)) * np.exp(rng.uniform(-3, 3, size=(1, 40)))
    for N in (8, 12, 16):
        A, beta, e = c.crt_gram(G, N)
        assert np.array_equal(A, A.T)
        ref = G.T @ G
        bound = c.representation_error_bound(G.T, G, beta, e, e) + 4 * np.finfo(float).eps * np.abs(G.T) @ np.abs(G)
        assert np.all(np.abs(A - ref) <= bound)


def test_sixteen_moduli_match_float64_accuracy():
    # with beta = 52 the representation error is at most 2^-53 of each
    # row/column maximum: the product is as accurate as a float64 GEMM
    rng = np.random.default_rng(6)
    A = rng.standard_normal((30, 200))
    B = rng.standard_normal((200, 20))
    C, beta, _, _ = c.crt_product(A, B, 16)
    assert beta == 52
    ref = (A.astype(np.longdouble) @ B.astype(np.longdouble)).astype(np.float64)
    assert np.max(np.abs(C - ref) / (np.abs(A) @ np.abs(B))) <= 4 * np.finfo(float).eps
