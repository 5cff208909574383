"""The bench's flop model against multiply-adds counted one by one.

The headline `value` is algorithmic flops per second, so its flop model is
pinned here: every term except the inverse's conventional r^3 is recounted
with explicit loops over the products the method forms (2 flops per
multiply-add), on small sizes with an uneven rank history."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _gram(m, n):        # lower triangle of G'G, diagonal included
    return sum(2 for i in range(n) for j in range(i + 1) for _ in range(m))


def _cholesky(n, r_before):   # column k: rows k..n-1 against the r_k columns accepted before it
    return sum(2 for k in range(n) for _ in range(k, n) for _ in range(r_before[k]))


def _ltl(n, r):         # lower triangle of L'L
    return sum(2 for i in range(r) for j in range(i + 1) for _ in range(n))


def _chain(m, n, r):    # K = L M, P = K K' (lower), Y = P G'
    k_lm = sum(2 for i in range(n) for j in range(r) for _ in range(r))
    p_kk = sum(2 for i in range(n) for j in range(i + 1) for _ in range(r))
    y_pg = sum(2 for i in range(n) for j in range(m) for _ in range(n))
    return k_lm + p_kk + y_pg


@pytest.mark.parametrize("m,n,acc,k", [
    (9, 6, [1, 1, 0, 1, 0, 1], 0),
    (11, 7, [1, 0, 1, 1, 1, 0, 1], 3),
    (5, 4, [0, 0, 0, 0], 2),
    (8, 8, [1] * 8, 1),
])
def test_geninv_flop_model_counts_every_product(bench, m, n, acc, k):
    r_before = [sum(acc[:j]) for j in range(n)]
    r = sum(acc)
    counted = _gram(m, n) + _cholesky(n, r_before) + _ltl(n, r) + _chain(m, n, r)
    counted += sum(2 for i in range(n) for j in range(k) for _ in range(m))   # W = Y F
    assert bench.algorithmic_flops(m, n, r_before, r, k) == counted + r ** 3


@pytest.mark.parametrize("m,n,r,k", [(9, 6, 4, 2), (12, 5, 5, 4), (7, 7, 0, 1)])
def test_lstsq_flop_model_counts_every_product(bench, m, n, r, k):
    r_before = [min(j, r) for j in range(n)]   # generic exact-rank input
    counted = _gram(m, n) + _cholesky(n, r_before) + _ltl(n, r)
    # W = L (M (M (L' (G'F))))
    counted += sum(2 for i in range(n) for j in range(k) for _ in range(m))   # G'F
    counted += sum(2 for i in range(r) for j in range(k) for _ in range(n))   # L'(.)
    counted += 2 * sum(2 for i in range(r) for j in range(k) for _ in range(r))   # M(.), twice
    counted += sum(2 for i in range(n) for j in range(k) for _ in range(r))   # L(.)
    assert bench.lstsq_flops(m, n, r, k) == counted + r ** 3
