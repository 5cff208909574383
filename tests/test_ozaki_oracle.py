"""Pins of the slicing reference (oracle/ozaki_ref.py) against exact facts."""
import numpy as np
import pytest

from oracle import ozaki_ref as z
from paper_0804_4809_amd import workloads as w


def test_exponents_bound_column_max():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((50, 7)) * np.array([1e-3, 1, 1e3, 0.5, 1.0, 2.0, 3.999])
    X[:, 4] = 0.0
    e = z.column_exponents(X)
    mx = np.abs(X).max(axis=0)
    for j in range(7):
        if mx[j] == 0:
            assert e[j] == 0
        else:
            assert mx[j] < 2.0 ** e[j] <= 2 * mx[j]
    # exact powers of two: max = 2^k  ->  e = k + 1
    assert z.column_exponents(np.array([[4.0], [-1.0]]))[0] == 3


def test_slices_are_bounded_integers():
    G, _ = w.lowrank_uv(64, 9, 5, seed=1)
    S, e = z.slice_columns(G, 4)
    assert S.dtype == np.int64 and np.abs(S).max() <= 255
    # truncation toward zero: every slice has the sign of its element (or is 0)
    assert np.all((S * np.sign(G)[None]) >= 0)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 6])
def test_reconstruction_error_bound(s):
    rng = np.random.default_rng(s)
    G = rng.standard_normal((200, 11)) * 10.0 ** rng.uniform(-3, 3, size=11)
    S, e = z.slice_columns(G, s)
    Gs = z.reconstruct(S, e)
    # |G - G_s| < 2^(e_j - 8 s) elementwise, and G_s is G truncated toward zero
    assert np.all(np.abs(G - Gs) < np.ldexp(1.0, e[None, :] - 8 * s))
    assert np.all(np.abs(Gs) <= np.abs(G))


def test_short_mantissas_are_represented_exactly():
    # entries with at most 16 significant bits below the column bound are exact with 2 slices
    rng = np.random.default_rng(3)
    ints = rng.integers(-2 ** 15, 2 ** 15, size=(40, 5)).astype(np.float64)
    G = ints * 2.0 ** -10
    S, e = z.slice_columns(G, 2)
    assert np.array_equal(z.reconstruct(S, e), G)


def test_sliced_gram_equals_gram_of_representation():
    # the sliced product of the representation is the exact Gram of G_s,
    # checked against float64 G_s'G_s computed in exact rational arithmetic
    from fractions import Fraction
    rng = np.random.default_rng(4)
    G = rng.standard_normal((12, 4))
    S, e = z.slice_columns(G, 3)
    Gs = z.reconstruct(S, e)
    A = z.sliced_gram(G, 3)
    for i in range(4):
        for j in range(4):
            exact = sum(Fraction(Gs[k, i]) * Fraction(Gs[k, j]) for k in range(12))
            assert A[i, j] == float(exact)


def test_sliced_gram_approaches_gram():
    G, _ = w.lowrank_uv(300, 20, 12, seed=5)
    A = G.T @ G
    for s, tol in [(2, 1e-4), (3, 1e-6), (4, 1e-8)]:
        As = z.sliced_gram(G, s)
        assert np.linalg.norm(As - A) / np.linalg.norm(A) < tol


def test_chunk_of_256_pair_products_is_exact_in_float32():
    # the accumulation argument of the GPU kernel: 256 products of slices
    # bounded by 255 sum to less than 2^24, so float32 partial sums are exact
    assert 256 * 255 * 255 < 2 ** 24
    rng = np.random.default_rng(6)
    a = rng.integers(-255, 256, size=256)
    b = rng.integers(-255, 256, size=256)
    acc = np.float32(0.0)
    for x, y in zip(a, b):
        acc = np.float32(acc + np.float32(x) * np.float32(y))
    assert int(acc) == int(np.dot(a, b))


@pytest.mark.parametrize("pairs,stages,exact", [(1, 6, True), (2, 3, True), (3, 2, True), (4, 2, True),
                                                 (4, 3, False), (2, 5, False), (1, 9, False)])
def test_class_period_bound_of_the_gpu_kernel(pairs, stages, exact):
    # the GPU kernel sums the slice products of one weight class (1 to 4
    # pairs) over `stages` 32-deep K stages in float32 before moving the sum
    # to float64: 6 stages for one pair, 3 for two, 2 for three or four.  The
    # sum stays an exact integer iff pairs * 32 * stages * 255^2 <= 2^24.
    n = pairs * 32 * stages
    assert (n * 255 * 255 <= 2 ** 24) == exact
    if exact:   # worst case: every product +255^2, summed in float32 order
        acc = np.float32(0.0)
        for _ in range(n):
            acc = np.float32(acc + np.float32(255.0 * 255.0))
        assert int(acc) == n * 255 * 255


@pytest.mark.parametrize("s,c", [(4, 0), (4, 3), (4, 4), (3, 2), (2, 1)])
def test_truncated_pair_set_is_the_sum_of_its_pairs(s, c):
    # brute force: each slice pair's product formed separately from the
    # exact per-slice reconstructions (small k: every float64 sum is exact)
    rng = np.random.default_rng(10 * s + c)
    A = rng.standard_normal((5, 3))
    B = rng.standard_normal((5, 4))
    SA, ea = z.slice_columns(A, s)
    SB, eb = z.slice_columns(B, s)
    got = z.sliced_product_exact(SA, ea, SB, eb, max_class=c)
    want = np.zeros((3, 4))
    for t in range(s):
        for u in range(s):
            if t + u <= c:
                At = np.ldexp(SA[t].astype(np.float64), -8 * (t + 1)) * np.ldexp(1.0, ea)[None, :]
                Bu = np.ldexp(SB[u].astype(np.float64), -8 * (u + 1)) * np.ldexp(1.0, eb)[None, :]
                want += At.T @ Bu
    assert np.array_equal(got, want)


def test_full_class_range_is_every_pair():
    rng = np.random.default_rng(3)
    SA, ea = z.slice_columns(rng.standard_normal((6, 2)), 3)
    SB, eb = z.slice_columns(rng.standard_normal((6, 5)), 3)
    assert np.array_equal(z.sliced_product_exact(SA, ea, SB, eb, max_class=4),
                          z.sliced_product_exact(SA, ea, SB, eb))
