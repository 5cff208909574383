"""Reference of the fixed-point operand slicing used by the mixed-precision
form, and of its exact sliced products.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Nothing here is part
of the paper; this is the error-free splitting of matrix products of Ozaki,
Ogita, Oishi and Rump (Numerical Algorithms 59, 2012), written from its
definition:

* every column j of X gets an exponent e_j, the smallest integer with
  max_i |X_ij| < 2^e_j;
* X_ij / 2^e_j lies in (-1, 1) and is cut, most significant first, into s
  signed integer slices of ``bits`` bits each, by truncation toward zero:
      r_0 = X_ij 2^-e_j,   S_t = trunc(2^bits r_t),   r_{t+1} = 2^bits r_t - S_t
  so that X_ij = 2^e_j (sum_t S_t 2^(-bits (t+1)) + r_s 2^(-bits s)), |r_s| < 1;
* a product of two sliced operands is the sum over slice pairs (t, u) of
  integer matrix products, each exact, scaled by powers of two.

With bits = 8 every slice is an integer of magnitude at most 255, exactly
representable in bfloat16, and a sum of 256 products of two slices stays
below 2^24, so float32 accumulation of such a chunk is exact.
"""
from __future__ import annotations

import numpy as np

SLICE_BITS = 8


def column_exponents(X: np.ndarray) -> np.ndarray:
    """e_j = smallest integer with max_i |X_ij| < 2^e_j (0 for a zero column)."""
    X = np.asarray(X, np.float64)
    mx = np.max(np.abs(X), axis=0) if X.shape[0] else np.zeros(X.shape[1])
    e = np.zeros(X.shape[1], dtype=np.int64)
    nz = mx > 0
    # frexp: mx = f 2^p with f in [0.5, 1)  =>  mx < 2^p and mx >= 2^(p-1)
    _, p = np.frexp(mx[nz])
    e[nz] = p
    return e


def slice_columns(X: np.ndarray, s: int, bits: int = SLICE_BITS):
    """Integer slices S (s x rows x cols, int64) and exponents e (cols) of X."""
    X = np.asarray(X, np.float64)
    e = column_exponents(X)
    r = np.ldexp(X, -e[None, :])
    S = np.zeros((s,) + X.shape, dtype=np.int64)
    for t in range(s):
        r = r * float(2 ** bits)
        St = np.trunc(r)
        r = r - St
        S[t] = St.astype(np.int64)
    return S, e


def reconstruct(S: np.ndarray, e: np.ndarray, bits: int = SLICE_BITS) -> np.ndarray:
    """X_s = 2^e_j sum_t S_t 2^(-bits (t+1)), evaluated exactly then rounded
    once (the slices of one element share a binade, so the float64 sum is
    exact whenever s * bits <= 53)."""
    s = S.shape[0]
    out = np.zeros(S.shape[1:], np.float64)
    for t in range(s):
        out += np.ldexp(S[t].astype(np.float64), -bits * (t + 1))
    return np.ldexp(out, e[None, :])


def sliced_product_exact(SA: np.ndarray, ea: np.ndarray, SB: np.ndarray, eb: np.ndarray,
                         bits: int = SLICE_BITS, max_class: int | None = None) -> np.ndarray:
    """C = A_s' B_s for column-sliced A (k x M) and B (k x N):
    C_ij = 2^(ea_i + eb_j) sum_{t,u} 2^(-bits (t+u+2)) (S^A_t' S^B_u)_ij over
    every slice pair, or, with ``max_class``, over the pairs with
    t + u <= max_class only (the truncated pair set of the Ozaki scheme).

    The integer products are exact in int64 (|entries| <= 255^2 k); the pair
    sums are formed exactly with Python integers and rounded to float64 once.
    Intended for small sizes."""
    s_a, s_b = SA.shape[0], SB.shape[0]
    M, N = SA.shape[2], SB.shape[2]
    # integer total in units of 2^(-bits (s_a + s_b))
    tot = np.zeros((M, N), dtype=object)
    for t in range(s_a):
        for u in range(s_b):
            if max_class is not None and t + u > max_class:
                continue
            prod = SA[t].T.astype(np.int64) @ SB[u].astype(np.int64)
            shift = bits * ((s_a - 1 - t) + (s_b - 1 - u))
            tot = tot + prod.astype(object) * (1 << shift)
    base = -bits * (s_a + s_b)
    out = np.empty((M, N), np.float64)
    for i in range(M):
        for j in range(N):
            out[i, j] = _ldexp_int(int(tot[i, j]), base + int(ea[i]) + int(eb[j]))
    return out


def _ldexp_int(v: int, e: int) -> float:
    """float64 nearest to v * 2^e for a Python integer v (one rounding)."""
    if v == 0:
        return 0.0
    neg = v < 0
    v = -v if neg else v
    nb = v.bit_length()
    if nb > 53:
        shift = nb - 53
        q, rem = divmod(v, 1 << shift)
        half = 1 << (shift - 1)
        if rem > half or (rem == half and (q & 1)):
            q += 1
        v, e = q, e + shift
    f = float(np.ldexp(float(v), e))
    return -f if neg else f


def sliced_gram(G: np.ndarray, s: int, bits: int = SLICE_BITS) -> np.ndarray:
    """Gram matrix of the sliced representation, G_s' G_s, every slice pair
    included, computed exactly and rounded to float64 once per entry."""
    S, e = slice_columns(G, s, bits)
    return sliced_product_exact(S, e, S, e, bits)
