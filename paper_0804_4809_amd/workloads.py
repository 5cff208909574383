"""Seeded synthetic workloads for the full-rank-Cholesky pseudoinverse.

Every matrix family used by the tests and the benchmark is generated here,
from ``numpy.random.default_rng(seed)``, in float64 (float32 where a family
is stored in single precision).  This module builds inputs only: it contains
none of the pseudoinverse method's arithmetic, and both the CPU reference
and the GPU library consume exactly the arrays it returns.

Families
--------
* ``lowrank_uv``  -- G = U V with Gaussian factors (exact rank r).
* ``rbf_design``  -- Gaussian radial-basis design matrix, the application of
  Section 4 of the paper: rows are inputs, columns are basis functions, and
  some centers are exact duplicates of earlier ones, so the matrix is rank
  deficient by construction.
* ``svd_family``  -- G = P diag(s) Q' with orthonormal P, Q and log-spaced s.
* ``table1``      -- the rank-deficient family of the timing experiment in
  Section 3 (n = 2^k, m = 2n, rank 7n/8, entries in [-1, 1]).
* ``batch_lowrank`` -- thousands of small uneven U V problems, float32.

All matrices are returned as C-contiguous ``float64`` arrays of shape
(rows, cols) unless stated otherwise; callers that need column-major storage
transpose-copy them.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# exact-rank Gaussian products
# ---------------------------------------------------------------------------
def lowrank_uv(m: int, n: int, r: int, seed: int, k: int = 0):
    """G = U V with U (m x r), V (r x n) i.i.d. N(0,1); F (m x k) N(0,1).

    Returns (G, F); F is None when k == 0.  rank(G) = min(r, m, n) with
    probability one.
    """
    g = _rng(seed)
    U = g.standard_normal((m, r))
    V = g.standard_normal((r, n))
    G = U @ V
    F = g.standard_normal((m, k)) if k > 0 else None
    return G, F


def c1_problem(seed: int = 0):
    """Plain CPU-sized case: 200 x 50, exact rank 40, F 200 x 3."""
    return lowrank_uv(200, 50, 40, seed, k=3)


# ---------------------------------------------------------------------------
# Gaussian RBF design matrices (Section 4 application)
# ---------------------------------------------------------------------------
def _center_order(n_unique: int, n_dup: int, g: np.random.Generator, interleave: bool):
    """Index list of length n_unique + n_dup into the unique centers.

    Duplicates copy a uniformly chosen unique center.  With ``interleave``
    each duplicate is inserted at a uniformly random position after its
    original; otherwise duplicates are appended at the end.
    """
    order = list(range(n_unique))
    srcs = g.integers(0, n_unique, size=n_dup)
    if not interleave:
        return np.array(order + [int(s) for s in srcs], dtype=np.int64)
    pos_of = np.arange(n_unique, dtype=np.int64)  # position of each original
    for s in srcs:
        p0 = int(pos_of[s]) + 1
        pos = int(g.integers(p0, len(order) + 1))
        order.insert(pos, int(s))
        pos_of[pos_of >= pos] += 1  # originals at or after pos shift right
    return np.array(order, dtype=np.int64)


def rbf_design(m: int, dim: int, n_unique: int, n_dup: int, sigma: float, seed: int,
               k: int = 0, interleave: bool = True, chunk_rows: int = 8192):
    """Gaussian RBF design matrix G_ij = exp(-|x_i - c_j|^2 / (2 sigma^2)).

    Inputs x_i are uniform in [0,1]^dim (m of them).  The first ``n_unique``
    centers are uniform in [0,1]^dim; ``n_dup`` more are exact copies of
    uniformly chosen unique centers.  F is (m x k) N(0,1).

    Returns (G, F, centers_index) where centers_index[j] names the unique
    center behind column j (duplicates share an index).
    """
    g = _rng(seed)
    X = g.uniform(0.0, 1.0, size=(m, dim))
    C_u = g.uniform(0.0, 1.0, size=(n_unique, dim))
    idx = _center_order(n_unique, n_dup, g, interleave)
    C = C_u[idx]
    n = C.shape[0]
    G = np.empty((m, n), dtype=np.float64)
    inv2s2 = 1.0 / (2.0 * sigma * sigma)

    def rows(r0):
        r1 = min(m, r0 + chunk_rows)
        d2 = np.zeros((r1 - r0, n), dtype=np.float64)
        diff = np.empty_like(d2)
        for t in range(dim):
            np.subtract(X[r0:r1, t][:, None], C[:, t][None, :], out=diff)
            np.multiply(diff, diff, out=diff)
            d2 += diff
        np.multiply(d2, -inv2s2, out=d2)
        np.exp(d2, out=G[r0:r1])

    # row blocks are independent and NumPy releases the GIL inside ufuncs;
    # the values do not depend on the number of threads
    starts = range(0, m, chunk_rows)
    workers = max(1, min(16, os.cpu_count() or 1, len(starts)))
    if workers > 1:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(rows, starts))
    else:
        for r0 in starts:
            rows(r0)
    F = g.standard_normal((m, k)) if k > 0 else None
    return G, F, idx


def c2_problem(seed: int = 1, m: int = 8192, n_unique: int = 1792, n_dup: int = 256):
    """RBF design, 8192 inputs in [0,1]^4, 2048 centers (256 duplicates), sigma 0.3, F 8192 x 8."""
    return rbf_design(m, 4, n_unique, n_dup, 0.3, seed, k=8)


def c5_problem(seed: int = 4, m: int = 131072, n_unique: int = 7000, n_dup: int = 1192):
    """Large RBF design: 131072 inputs in [0,1]^8, 8192 centers (1192 duplicates), sigma 0.5, F 131072 x 16."""
    return rbf_design(m, 8, n_unique, n_dup, 0.5, seed, k=16)


# ---------------------------------------------------------------------------
# G = P diag(s) Q' with orthonormal factors
# ---------------------------------------------------------------------------
def svd_family(m: int, n: int, r: int, smin: float, seed: int, k: int = 0):
    """G = P diag(s) Q', P (m x r), Q (n x r) orthonormal columns (QR of Gaussians),
    s log-spaced from 1 down to ``smin``.  Returns (G, F, P, s, Q)."""
    g = _rng(seed)
    P, _ = np.linalg.qr(g.standard_normal((m, r)))
    Q, _ = np.linalg.qr(g.standard_normal((n, r)))
    s = np.logspace(0.0, np.log10(smin), r)
    G = (P * s[None, :]) @ Q.T
    F = g.standard_normal((m, k)) if k > 0 else None
    return G, F, P, s, Q


def c3_problem(seed: int = 2, m: int = 32768, n: int = 4096, r: int = 3072):
    """Mixed-precision case: 32768 x 4096, rank 3072, s in [1e-3, 1]."""
    return svd_family(m, n, r, 1e-3, seed)


# ---------------------------------------------------------------------------
# Section 3 timing family
# ---------------------------------------------------------------------------
def table1(n: int, seed: int):
    """m = 2n rows, rank 7n/8, entries in [-1, 1].

    Column slots are split at random into 7n/8 base slots (slot 0 is always
    a base) and n/8 dependent slots.  Base columns are uniform in [-1, 1].
    A dependent column is a random combination (uniform [-1, 1] weights) of
    the base columns placed before it, rescaled to max-abs 1, so each one is
    exactly dependent on columns that precede it.  Requires n divisible by 8.
    """
    if n % 8:
        raise ValueError("n must be a multiple of 8")
    g = _rng(seed)
    m, r = 2 * n, 7 * n // 8
    dep = np.zeros(n, dtype=bool)
    dep[1 + g.choice(n - 1, size=n - r, replace=False)] = True
    G = np.empty((m, n), dtype=np.float64)
    base_cols = []
    for j in range(n):
        if not dep[j]:
            G[:, j] = g.uniform(-1.0, 1.0, size=m)
            base_cols.append(j)
        else:
            coef = g.uniform(-1.0, 1.0, size=len(base_cols))
            col = G[:, base_cols] @ coef
            G[:, j] = col / np.max(np.abs(col))
    return G


# ---------------------------------------------------------------------------
# batched small problems
# ---------------------------------------------------------------------------
@dataclass
class Batch:
    m: np.ndarray          # int32 [B]
    n: np.ndarray          # int32 [B]
    rank: np.ndarray       # int32 [B], construction rank
    G: list                # float32 (m_b x n_b) arrays
    F: list                # float32 (m_b x k) arrays
    k: int


def batch_lowrank(count: int, seed: int, k: int = 4, m_lo: int = 64, m_hi: int = 1024,
                  n_lo: int = 16, n_hi: int = 256):
    """``count`` problems with m ~ U[m_lo, m_hi], n ~ U[n_lo, min(n_hi, m//2)],
    r ~ U[n//2, n] (integer, inclusive); G_b = U_b V_b with N(0,1) factors,
    F_b (m x k) N(0,1); G_b and F_b are stored as float32."""
    g = _rng(seed)
    ms = np.empty(count, np.int32)
    ns = np.empty(count, np.int32)
    rs = np.empty(count, np.int32)
    Gs, Fs = [], []
    for b in range(count):
        m = int(g.integers(m_lo, m_hi + 1))
        n = int(g.integers(n_lo, min(n_hi, m // 2) + 1))
        r = int(g.integers(n // 2, n + 1))
        U = g.standard_normal((m, r))
        V = g.standard_normal((r, n))
        Gs.append((U @ V).astype(np.float32))
        Fs.append(g.standard_normal((m, k)).astype(np.float32))
        ms[b], ns[b], rs[b] = m, n, r
    return Batch(ms, ns, rs, Gs, Fs, k)


def c4_problem(seed: int = 3, count: int = 4096):
    """4096 uneven small least-squares problems, F_b with 4 columns."""
    return batch_lowrank(count, seed, k=4)
