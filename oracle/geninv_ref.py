"""Float64 CPU reference of the full-rank-Cholesky Moore-Penrose inverse.

TEST INFRASTRUCTURE ONLY.  This module is the oracle that the GPU library is
checked against.  Only the test-suite, the package smoke check and the CPU
baseline leg of the benchmark may import it; the library itself never does.
It shares no code with the GPU path.

It follows the paper (P. Courrieu, "Fast Computation of Moore-Penrose Inverse
Matrices") step by step, in plain NumPy float64, without blocking, fusion or
reordering:

1. transpose branch when m < n                      (Appendix, transpose test)
2. Gram matrix A = G'G                              (Section 2, Eq. (1))
3. tol = 1e-9 * (smallest positive diagonal of A)   (Appendix, tolerance)
4. full-rank Cholesky of A, column by column, that
   keeps column k only when its updated pivot is
   strictly above tol                               (Section 2, Theorem 4 of
                                                     its ref. [6]; Appendix)
5. M = (L'L)^-1                                     (Theorem 1; Appendix)
6. Y = L M M L' G'                                  (Theorem 1; Appendix)

and the least-squares use of the result, W = G^+ F, from Section 1.

Readings of points the paper leaves open are listed with each function.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg.lapack as _lapack

TOL_FACTOR = 1e-9  # Appendix: tolerance is 1e-9 times the smallest positive Gram diagonal


@dataclass
class GeninvResult:
    """Everything the oracle computes, kept for parity reports."""
    Y: np.ndarray            # n x m pseudoinverse (m x n input)
    rank: int
    piv: np.ndarray          # int64[rank]: 0-based pivot (accepted) column of each L column
    d: np.ndarray            # float64[n_eff]: updated pivot value d_k seen for every k
    tol: float | None        # None when the Gram has no positive diagonal
    L: np.ndarray            # n_eff x rank
    M: np.ndarray            # rank x rank, (L'L)^-1
    A: np.ndarray            # n_eff x n_eff Gram matrix actually factored
    transposed: bool = False
    extra: dict = field(default_factory=dict)


def gram(G: np.ndarray, row_blocks: int = 1) -> np.ndarray:
    """A = G'G (Section 2, Eq. (1); Appendix).

    ``row_blocks`` > 1 sums the Gram matrices of that many row blocks of G
    instead: the same matrix in exact arithmetic, a different rounding order.
    Used only to measure how far two correct float64 evaluations of the method
    can drift apart on a given input (its self-spread)."""
    G = np.asarray(G, dtype=np.float64)
    if row_blocks <= 1:
        return G.T @ G
    A = np.zeros((G.shape[1], G.shape[1]))
    for blk in np.array_split(G, row_blocks, axis=0):
        A += blk.T @ blk
    return A


def paper_tol(A: np.ndarray) -> float | None:
    """Default tolerance: 1e-9 times the smallest strictly positive diagonal
    entry of A (Appendix).  Returns None when no diagonal entry is positive:
    the paper's minimum over an empty set is empty, every pivot test then
    fails and the rank is 0."""
    dA = np.diag(A)
    pos = dA[dA > 0]
    if pos.size == 0:
        return None
    return float(pos.min()) * TOL_FACTOR


def full_rank_cholesky(A: np.ndarray, tol: float | None, *, matlab_stale: bool = False,
                       forced: np.ndarray | None = None):
    """Full-rank Cholesky factor L (n x r) with A = L L' (Section 2, Eq. (1)).

    Column k of A is processed in order k = 0..n-1 (Appendix):
        v = A[k:, k] - L[k:, :r] L[k, :r]'
        if v[0] > tol (strict): L[k, r] = sqrt(v[0]); L[k+1:, r] = v[1:] / L[k, r]; r += 1
        otherwise column k is dropped.

    Reading: a dropped column leaves nothing behind, so every L column is zero
    above its pivot row and L is the paper's factor S' with its zero rows
    removed.  ``matlab_stale=True`` instead keeps the rejected value v[0] in
    row k of the next column, as the printed listing's in-place update would.

    ``forced`` (bool[n], replay mode) takes the keep/drop decision of every
    column from the given mask instead of the tol test, with the arithmetic
    otherwise unchanged.  It lets a parity check reproduce another
    implementation's decisions when a pivot lies within rounding of tol.

    Returns (L, r, piv, d) where d[k] is the updated pivot value of column k.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n), dtype=np.float64)
    piv = []
    d = np.zeros(n, dtype=np.float64)
    r = 0
    for k in range(n):
        v = A[k:, k] - L[k:, :r] @ L[k, :r]
        d[k] = v[0]
        keep = (tol is not None and v[0] > tol) if forced is None else bool(forced[k])
        if keep:
            s = np.sqrt(v[0])
            L[k, r] = s
            L[k + 1:, r] = v[1:] / s
            piv.append(k)
            r += 1
        elif matlab_stale:
            L[k, r] = v[0]
    return L[:, :r].copy(), r, np.array(piv, dtype=np.int64), d


def spd_inverse(B: np.ndarray) -> np.ndarray:
    """M = B^-1 for symmetric positive definite B (Theorem 1: B = L'L).

    Reading: the inverse is taken through the Cholesky factor of B (LAPACK
    potrf then potri), which equals the general inverse in exact arithmetic
    and uses that B is SPD.  The result is symmetrised from its lower half.
    """
    r = B.shape[0]
    if r == 0:
        return np.zeros((0, 0))
    c, info = _lapack.dpotrf(np.asarray(B, dtype=np.float64), lower=1, clean=1)
    if info != 0:
        raise np.linalg.LinAlgError(f"L'L is not positive definite (potrf info={info})")
    inv, info = _lapack.dpotri(c, lower=1)
    if info != 0:
        raise np.linalg.LinAlgError(f"potri failed (info={info})")
    low = np.tril(inv)
    return low + np.tril(inv, -1).T


def geninv(G: np.ndarray, tol: float | None = None, *, matlab_stale: bool = False,
           gram_row_blocks: int = 1, forced: np.ndarray | None = None,
           A: np.ndarray | None = None) -> GeninvResult:
    """Moore-Penrose inverse Y = G^+ (n x m) of a real m x n matrix G.

    Follows the Appendix: if m < n the method factors A = G G' instead and
    returns Y = G' L M M L' (the transpose branch); otherwise A = G'G and
    Y = L M M L' G' (Theorem 1).

    ``tol``: None or <= 0 selects the paper's default (``paper_tol``); a
    positive value is used as given.
    The product chain is evaluated left to right, as written in the Appendix.
    ``forced``: replay mode of ``full_rank_cholesky``.  ``A``: use this Gram
    matrix instead of forming it (sensitivity studies).
    """
    G = np.asarray(G, dtype=np.float64)
    if G.ndim != 2:
        raise ValueError("G must be 2-D")
    m, n = G.shape
    transposed = m < n
    Gw = G.T if transposed else G          # work matrix with rows >= cols
    if A is None:
        A = gram(Gw, gram_row_blocks)
    t = paper_tol(A) if (tol is None or tol <= 0) else float(tol)
    L, r, piv, d = full_rank_cholesky(A, t, matlab_stale=matlab_stale, forced=forced)
    M = spd_inverse(L.T @ L)
    if r == 0:
        Y = np.zeros((n, m))
    elif transposed:
        Y = (((G.T @ L) @ M) @ M) @ L.T
    else:
        Y = (((L @ M) @ M) @ L.T) @ G.T
    return GeninvResult(Y=np.ascontiguousarray(Y), rank=r, piv=piv, d=d, tol=t, L=L, M=M, A=A,
                        transposed=transposed)


def lstsq(G: np.ndarray, F: np.ndarray, tol: float | None = None, *, gram_row_blocks: int = 1):
    """Minimum-norm least-squares weights W = G^+ F (Section 1).

    Reading: the printed "W = G^+ W" is a typo for W = G^+ F, the solution of
    min ||G W - F||^2 stated just before it.  Returns (W, result)."""
    res = geninv(G, tol, gram_row_blocks=gram_row_blocks)
    F = np.asarray(F, dtype=np.float64)
    return res.Y @ F, res


def decision_margins(res: GeninvResult) -> dict:
    """Smallest accepted and largest rejected pivot, relative to tol."""
    if res.tol is None or res.d.size == 0:
        return {"min_acc": None, "max_rej": None}
    acc = np.zeros(res.d.size, bool)
    acc[res.piv] = True
    a = res.d[acc] / res.tol
    j = res.d[~acc] / res.tol
    return {"min_acc": float(a.min()) if a.size else None,
            "max_rej": float(j.max()) if j.size else None}


def penrose_errors(G: np.ndarray, Y: np.ndarray) -> dict:
    """Max-abs entry of the four Penrose error matrices (Section 1 and the
    accuracy criterion of Section 3)."""
    G = np.asarray(G, np.float64)
    Y = np.asarray(Y, np.float64)
    GY = G @ Y
    YG = Y @ G
    return {
        "GYG-G": float(np.max(np.abs(GY @ G - G), initial=0.0)),
        "YGY-Y": float(np.max(np.abs(YG @ Y - Y), initial=0.0)),
        "(GY)'-GY": float(np.max(np.abs(GY.T - GY), initial=0.0)),
        "(YG)'-YG": float(np.max(np.abs(YG.T - YG), initial=0.0)),
    }


def gram_extended(G: np.ndarray) -> np.ndarray:
    """G'G accumulated in x87 extended precision (64-bit significand) and
    rounded to float64 once: the Gram matrix to within about one rounding.
    Plain O(m n^2) loops in NumPy longdouble; for small inputs only."""
    Gl = np.asarray(G, dtype=np.longdouble)
    return (Gl.T @ Gl).astype(np.float64)


def self_spread(G: np.ndarray, tol: float | None = None, base: GeninvResult | None = None,
                forced: np.ndarray | None = None, extended_limit: float = 3e8) -> float:
    """Rounding sensitivity of the method on this input.

    The relative Frobenius distance between the oracle's Y and the Y the
    same algorithm gives from a Gram matrix that differs only by rounding:
    the Gram summed in two row halves, and (when m n^2 <= extended_limit)
    the Gram accumulated in extended precision.  The largest distance is
    returned.  The method's forward error grows like cond(G)^4 u, so for
    ill-conditioned G no two float64 evaluations agree more closely than
    this.  ``forced`` replays given decisions in every run."""
    a = base if base is not None else geninv(G, tol, forced=forced)
    G = np.asarray(G, np.float64)
    variants = [dict(gram_row_blocks=2)]
    m, n = G.shape
    if m * min(m, n) ** 2 <= extended_limit:
        Gw = G.T if m < n else G
        variants.append(dict(A=gram_extended(Gw)))
    out = 0.0
    for kw in variants:
        b = geninv(G, tol, forced=forced if forced is not None else None, **kw)
        if forced is None and b.rank != a.rank:
            return float("inf")
        out = max(out, rel_fro(b.Y, a.Y))
    return out


def ambiguity_band(A: np.ndarray, tol: float, keep: np.ndarray | None = None, *, rel_eps: float | None = None,
                   trials: int = 2, safety: float = 4.0, seed: int = 0) -> np.ndarray:
    """Per-column half-width, relative to tol, of the pivot values whose
    keep/drop decision two correct float64 evaluations may take differently.

    Measured, not assumed: the factorization is replayed (same decisions,
    ``keep``, default the oracle's own) on ``trials`` copies of A whose
    entries carry independent random relative perturbations of size
    ``rel_eps`` (default 2 sqrt(n) u: a pivot value is the end of a chain of
    about n rounded updates, whose errors add up like a random walk), and
    the band is ``safety`` times the largest change of each pivot value,
    plus the Cholesky backward-error term 2 (n+1) u A_kk.  On well-conditioned inputs
    the band is tiny; on Gaussian RBF design matrices, whose pivots fall
    through ten orders of magnitude to tol, it reaches a few percent."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    u = np.finfo(np.float64).eps / 2
    eps = 2 * np.sqrt(max(n, 1)) * u if rel_eps is None else rel_eps
    L0, r0, piv0, d0 = full_rank_cholesky(A, tol)
    if keep is None:
        keep = np.zeros(n, bool)
        keep[piv0] = True
    else:
        L0, r0, piv0, d0 = full_rank_cholesky(A, tol, forced=keep)
    rng = np.random.default_rng(seed)
    spread = np.zeros(n)
    for _ in range(trials):
        E = rng.uniform(-1.0, 1.0, size=A.shape)
        E = np.tril(E) + np.tril(E, -1).T
        _, _, _, d1 = full_rank_cholesky(A * (1.0 + eps * E), tol, forced=keep)
        spread = np.maximum(spread, np.abs(d1 - d0))
    return (safety * spread + 2.0 * (n + 1) * u * np.abs(np.diag(A))) / tol


def newton_schulz_step(X: np.ndarray, G: np.ndarray) -> np.ndarray:
    """One Newton-Schulz step for the pseudoinverse, X <- X (2I - G X), in
    float64 with two plain matrix products (the refinement the mixed form
    applies; the iteration of Ben-Israel and Cohen for G^+).  X is n x m for
    an m x n G.  If I - G X restricted to the range of G has spectral radius
    below one and X starts in the row/column spaces of G', the iterates
    converge quadratically to G^+: the residual I - G X is squared by each
    step."""
    X = np.asarray(X, np.float64)
    G = np.asarray(G, np.float64)
    return 2.0 * X - (X @ G) @ X


def newton_schulz_factored_step(P: np.ndarray, A: np.ndarray) -> np.ndarray:
    """The same step written on P with X = P G' and A = G'G:
    P <- 2P - P A P, since X (2I - G X) = (2P - P G'G P) G'.  P and A are
    n x n and symmetric."""
    P = np.asarray(P, np.float64)
    A = np.asarray(A, np.float64)
    return 2.0 * P - (P @ A) @ P


def rel_fro(X: np.ndarray, Ref: np.ndarray) -> float:
    """||X - Ref||_F / ||Ref||_F (0 when both are zero)."""
    num = float(np.linalg.norm(np.asarray(X, np.float64) - Ref))
    den = float(np.linalg.norm(Ref))
    if den == 0.0:
        return num
    return num / den
