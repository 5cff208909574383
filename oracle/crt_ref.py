"""Reference of the integer-representation products of the mixed form's
int8 engine.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Nothing here is part
of the paper.  The int8 engine evaluates a product C = A B as the exact
product of fixed-point integer representations of A and B, obtained on the
GPU from int8 matrix products modulo small coprime integers and the Chinese
remainder theorem (the modular product scheme of Ozaki, Uchino and Imamura,
"Ozaki scheme II", 2025).  What it computes has a plain definition, written
out here without any modular arithmetic:

* every row i of A gets the exponent ea_i, the smallest integer with
  max_k |A_ik| < 2^ea_i (0 for a zero row), and every column j of B the
  exponent eb_j likewise;
* with a bit count beta, a_ik = rint(A_ik 2^(beta - ea_i)) and
  b_kj = rint(B_kj 2^(beta - eb_j)) are integers of magnitude <= 2^beta
  (rint: round to nearest, ties to even);
* C_ij = 2^(ea_i + eb_j - 2 beta) sum_k a_ik b_kj, the integer sum exact and
  the result rounded once to float64.

The moduli are the N largest pairwise coprime integers not above 255, taken
greedily from 255 down (residues of magnitude <= 127 fit int8, and 127^2
times 2^17 terms stays below 2^31).  beta is the largest bit count, at most
52, for which K 2^(2 beta) stays below M / 2 with a margin of 2^-20 relative
(M = product of the moduli, K = inner dimension), so that the modular
residues determine the signed integer sum uniquely.
"""
from __future__ import annotations

from math import gcd

import numpy as np

MODULUS_MAX = 255
BETA_MAX = 52


def moduli(N: int) -> list[int]:
    """The N largest pairwise coprime integers <= 255, descending."""
    out: list[int] = []
    p = MODULUS_MAX
    while len(out) < N and p > 1:
        if all(gcd(p, q) == 1 for q in out):
            out.append(p)
        p -= 1
    if len(out) < N:
        raise ValueError(f"fewer than {N} pairwise coprime integers below {MODULUS_MAX + 1}")
    return out


def modulus_product(N: int) -> int:
    M = 1
    for p in moduli(N):
        M *= p
    return M


def beta_bits(N: int, K: int) -> int:
    """Largest beta <= 52 with 2 K 2^(2 beta) (1 + 2^-20) <= M: every integer
    sum of K products of two integers of magnitude <= 2^beta then lies
    strictly inside (-M/2, M/2), with room for the float64 rounding of the
    reconstruction's quotient.  -1 if even beta = 0 does not fit."""
    M = modulus_product(N)
    K = max(int(K), 1)
    beta = -1
    for b in range(BETA_MAX + 1):
        need = 2 * K * (1 << (2 * b))
        if need + (need >> 20) <= M:
            beta = b
    return beta


def exponents(X: np.ndarray, axis: int) -> np.ndarray:
    """e = smallest integer with max |x| < 2^e along `axis` (0 for zeros):
    axis=1 gives one exponent per row, axis=0 one per column."""
    X = np.asarray(X, np.float64)
    mx = np.max(np.abs(X), axis=axis) if X.shape[axis] else np.zeros(X.shape[1 - axis])
    e = np.zeros(mx.shape, dtype=np.int64)
    nz = mx > 0
    _, p = np.frexp(mx[nz])     # mx = f 2^p, f in [0.5, 1): mx < 2^p
    e[nz] = p
    return e


def int_representation(X: np.ndarray, e: np.ndarray, beta: int, axis: int) -> np.ndarray:
    """rint(X 2^(beta - e)) as int64, e per row (axis=1) or per column (axis=0)."""
    X = np.asarray(X, np.float64)
    sh = (beta - np.asarray(e, np.int64))
    sh = sh[:, None] if axis == 1 else sh[None, :]
    return np.rint(np.ldexp(X, sh)).astype(np.int64)


def exact_int_product(Ai: np.ndarray, Bi: np.ndarray) -> np.ndarray:
    """Exact integer product of int64 matrices with entries below 2^53, as
    an object array of Python ints: each operand is split into three limbs
    of 18 bits (|limb| < 2^18), every limb product is an int64 matrix
    product with no overflow (K < 2^27), and the nine are combined in
    Python integers."""
    Ai = np.asarray(Ai, np.int64)
    Bi = np.asarray(Bi, np.int64)
    K = Ai.shape[1]
    if K >= (1 << 27):
        raise ValueError("inner dimension too large for the limb products")

    def limbs(X):
        s = np.sign(X)
        a = np.abs(X)
        return [s * ((a >> (18 * t)) & ((1 << 18) - 1)) for t in range(3)]

    La, Lb = limbs(Ai), limbs(Bi)
    out = np.zeros((Ai.shape[0], Bi.shape[1]), dtype=object)
    for t in range(3):
        for u in range(3):
            part = (La[t] @ Lb[u]).astype(object)
            out += part * (1 << (18 * (t + u)))
    return out


def crt_product(A: np.ndarray, B: np.ndarray, N: int):
    """C = A B as the int8 engine defines it with N moduli.  Returns
    (C float64, beta, ea, eb)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    K = A.shape[1]
    beta = beta_bits(N, K)
    if beta < 0:
        raise ValueError("too few moduli for this inner dimension")
    ea = exponents(A, axis=1)
    eb = exponents(B, axis=0)
    X = exact_int_product(int_representation(A, ea, beta, 1), int_representation(B, eb, beta, 0))
    C = np.empty(X.shape, np.float64)
    for i in range(X.shape[0]):
        for j in range(X.shape[1]):
            # int -> float rounds to nearest once; the power-of-two scaling is exact
            C[i, j] = np.ldexp(float(X[i, j]), int(ea[i] + eb[j] - 2 * beta))
    return C, beta, ea, eb


def crt_gram(G: np.ndarray, N: int):
    """A = G'G as the int8 engine forms the Gram matrix: one column
    representation of G on both sides, so A is the exactly rounded Gram
    matrix of that representation.  Returns (A, beta, e)."""
    G = np.asarray(G, np.float64)
    A, beta, ea, eb = crt_product(G.T, G, N)
    return A, beta, eb


def representation_error_bound(A: np.ndarray, B: np.ndarray, beta: int, ea, eb) -> np.ndarray:
    """Elementwise bound on |crt_product - A B| from the operand rounding:
    |a 2^(ea-beta) - A| <= 2^(ea-beta-1), likewise for B."""
    A = np.abs(np.asarray(A, np.float64))
    B = np.abs(np.asarray(B, np.float64))
    da = np.ldexp(np.ones(A.shape[0]), np.asarray(ea) - beta - 1)[:, None]
    db = np.ldexp(np.ones(B.shape[1]), np.asarray(eb) - beta - 1)[None, :]
    K = A.shape[1]
    return da * B.sum(axis=0)[None, :] + A.sum(axis=1)[:, None] * db + K * da * db
