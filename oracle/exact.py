"""Exact rational pseudoinverse for tiny integer matrices.

TEST INFRASTRUCTURE ONLY: a second, independent reference used to pin the
float64 oracle.  It does not follow the paper's algorithm.  It computes G^+
in exact rational arithmetic (``fractions.Fraction``) from the classical
full-rank factorization formula

    G = B C,  B (m x r) and C (r x n) of full rank r
    =>  G^+ = C' (C C')^-1 (B' B)^-1 B'

with B the greedily chosen independent columns of G (left to right) and C
the exact coordinates of every column of G in that basis.  In exact
arithmetic the paper's full-rank Cholesky accepts exactly these columns,
and its updated pivot d_k equals the squared distance of column k to the
span of the columns accepted before it; both are returned for the pins.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _frac_matrix(G):
    return [[Fraction(int(x)) if float(x).is_integer() else Fraction(x) for x in row] for row in G]


def _T(X):
    return [list(col) for col in zip(*X)] if X and X[0] else []


def _mm(X, Y):
    if not X or not Y or not Y[0]:
        return [[Fraction(0)] * (len(Y[0]) if Y and Y[0] else 0) for _ in X]
    YT = _T(Y)
    return [[sum((a * b for a, b in zip(row, col)), Fraction(0)) for col in YT] for row in X]


def _inv(X):
    """Exact inverse by Gauss-Jordan with nonzero pivot search."""
    n = len(X)
    aug = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(X)]
    for c in range(n):
        p = next((i for i in range(c, n) if aug[i][c] != 0), None)
        if p is None:
            raise ZeroDivisionError("singular matrix")
        aug[c], aug[p] = aug[p], aug[c]
        pv = aug[c][c]
        aug[c] = [v / pv for v in aug[c]]
        for i in range(n):
            if i != c and aug[i][c] != 0:
                f = aug[i][c]
                aug[i] = [a - f * b for a, b in zip(aug[i], aug[c])]
    return [row[n:] for row in aug]


def _sqdist_to_span(g, basis_cols):
    """Squared Euclidean distance of vector g to span(basis_cols), exactly."""
    gg = sum((x * x for x in g), Fraction(0))
    if not basis_cols:
        return gg
    B = _T(basis_cols)                 # m x s
    BtB = _mm(_T(B), B)
    Btg = [sum((b * x for b, x in zip(col, g)), Fraction(0)) for col in basis_cols]
    coef = [sum((a * b for a, b in zip(row, Btg)), Fraction(0)) for row in _inv(BtB)]
    proj = sum((c * x for c, x in zip(coef, Btg)), Fraction(0))
    return gg - proj


def exact_pinv(G):
    """Return (Y, rank, piv, d) for an integer/rational matrix G, exactly.

    Y is a list-of-lists of Fractions (n x m); piv the accepted column
    indices; d[k] the exact squared distance of column k to the span of the
    columns accepted before it (zero exactly for dependent columns).
    """
    G = _frac_matrix(np.asarray(G))
    m = len(G)
    n = len(G[0]) if m else 0
    cols = _T(G)
    piv, basis, d = [], [], []
    for k in range(n):
        dk = _sqdist_to_span(cols[k], basis)
        d.append(dk)
        if dk != 0:
            piv.append(k)
            basis.append(cols[k])
    r = len(piv)
    if r == 0:
        return [[Fraction(0)] * m for _ in range(n)], 0, piv, d
    B = _T(basis)                                   # m x r
    BtB_inv = _inv(_mm(_T(B), B))                   # r x r
    C = _mm(_mm(BtB_inv, _T(B)), G)                 # r x n, exact coordinates
    CCt_inv = _inv(_mm(C, _T(C)))
    Y = _mm(_mm(_mm(_T(C), CCt_inv), BtB_inv), _T(B))
    return Y, r, piv, d


def is_exact_pinv(G, Y) -> bool:
    """True iff Y satisfies the four Penrose conditions exactly for G."""
    G = _frac_matrix(np.asarray(G))
    GY, YG = _mm(G, Y), _mm(Y, G)
    return (_mm(GY, G) == G and _mm(YG, Y) == Y and _T(GY) == GY and _T(YG) == YG)


def to_float(Y) -> np.ndarray:
    return np.array([[float(x) for x in row] for row in Y], dtype=np.float64).reshape(len(Y), -1)
