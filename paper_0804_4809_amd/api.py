"""Python entry points of libgeninv, same names as the C ABI.

Tensors are torch float64 tensors on a GPU.  Inputs may have any strides: a
column-major tensor (strides (1, ld)) is passed straight through, any other
layout is first copied to column-major (the paper's storage order).  Outputs
are returned as column-major tensors of the mathematical shape.  torch
supplies only device memory and the current stream; every step of the method
runs in libgeninv's HIP kernels.
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple
from dataclasses import dataclass

import torch

from ._lib import GENINV_EACCURACY, GeninvError, load

_ctxs: dict = {}


def _ctx(device: torch.device):
    """Per-device context, switched to torch's current stream on every call."""
    idx = device.index if device.index is not None else torch.cuda.current_device()
    lib = load()
    c = _ctxs.get(idx)
    if c is None:
        h = ctypes.c_void_p()
        st = lib.geninv_create(ctypes.byref(h), idx, ctypes.c_void_p(torch.cuda.current_stream(idx).cuda_stream))
        if st != 0:
            raise GeninvError(st, "geninv_create")
        c = h
        _ctxs[idx] = c
    lib.geninv_set_stream(c, ctypes.c_void_p(torch.cuda.current_stream(idx).cuda_stream))
    return c


def set_host_sync(enable: bool, device=None):
    """geninv_set_host_sync on the context of `device` (default: current)."""
    _check(load().geninv_set_host_sync(_ctx(_ctx_of(device)), 1 if enable else 0), "geninv_set_host_sync")


def _ctx_of(device):
    return torch.device("cuda", device if isinstance(device, int) else torch.cuda.current_device()) \
        if not isinstance(device, torch.device) else device


def set_workspace_limit(nbytes: int, device=None):
    """geninv_set_workspace_limit (0 = no cap) on the context of `device`."""
    _check(load().geninv_set_workspace_limit(_ctx(_ctx_of(device)), int(nbytes)), "geninv_set_workspace_limit")


def set_debug(flags: int, device=None):
    """geninv_set_debug (GENINV_DEBUG_POISON = 1) on the context of `device`."""
    _check(load().geninv_set_debug(_ctx(_ctx_of(device)), int(flags)), "geninv_set_debug")


def debug_poison(device=None):
    """geninv_debug_poison: NaN-fill the context's current workspace."""
    _check(load().geninv_debug_poison(_ctx(_ctx_of(device))), "geninv_debug_poison")


def _check(st: int, where: str):
    if st != 0:
        raise GeninvError(st, where)


def _dev(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU (libgeninv has no CPU path)")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")


def colmajor(t: torch.Tensor):
    """(tensor, ld) with column-major storage: copies only when needed."""
    r, c = t.shape
    if t.stride(0) == 1 and (c <= 1 or t.stride(1) >= max(1, r)):
        return t, max(1, t.stride(1) if c > 1 else r)
    cm = t.t().contiguous().t()
    return cm, max(1, r)


def empty_colmajor(rows: int, cols: int, device, dtype=torch.float64):
    return torch.empty_strided((rows, cols), (1, max(1, rows)), device=device, dtype=dtype)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def geninv(G: torch.Tensor, tol: float | None = None, *, return_piv: bool = False):
    """Y = G^+ (n x m) and the rank r (Theorem 1; Appendix).  Synchronizes to read r."""
    _dev(G, "G")
    m, n = G.shape
    Gc, ldg = colmajor(G)
    Y = empty_colmajor(n, m, G.device)
    piv = torch.empty(max(1, min(m, n)), dtype=torch.int32, device=G.device)
    r = ctypes.c_int(0)
    st = load().geninv_dgeninv(_ctx(G.device), m, n, _p(Gc), ldg, float(tol or 0.0), _p(Y), max(1, n),
                               ctypes.byref(r), _p(piv))
    _check(st, "geninv_dgeninv")
    if return_piv:
        return Y, r.value, piv[: r.value]
    return Y, r.value


ENGINES = {"bf16": 1, "int8": 2}


@dataclass
class MixedResult:
    Y: torch.Tensor
    rank: int
    piv: torch.Tensor
    err_est: float
    status: int          # 0, or the EACCURACY status when err_est exceeds the target


def mixed(G: torch.Tensor, tol: float | None = None, engine: str = "int8", gram_digits: int = 16,
          chain_digits: int = 16, ns_steps: int = 0, target: float = 0.0, *, return_result: bool = False):
    """Y = G^+ with the Gram matrix and Y = P G' on reduced-precision matrix
    cores (geninv_mixed): engine "int8" (digits = moduli, 16 give float64
    accuracy) or "bf16" (digits = 8-bit slices, at most 4); pivots, the
    factor and (L'L)^-1 in float64.  Returns (Y, r), or a MixedResult with
    the error estimate and status when return_result (then a missed target
    is reported in .status instead of raised)."""
    _dev(G, "G")
    m, n = G.shape
    Gc, ldg = colmajor(G)
    Y = empty_colmajor(n, m, G.device)
    piv = torch.empty(max(1, min(m, n)), dtype=torch.int32, device=G.device)
    r = ctypes.c_int(0)
    est = ctypes.c_double(0.0)
    st = load().geninv_mixed(_ctx(G.device), m, n, _p(Gc), ldg, float(tol or 0.0), ENGINES[engine],
                             int(gram_digits), int(chain_digits), int(ns_steps), float(target), _p(Y), max(1, n),
                             ctypes.byref(r), _p(piv), ctypes.byref(est))
    if return_result and st == GENINV_EACCURACY:
        return MixedResult(Y, r.value, piv[: r.value], est.value, st)
    _check(st, "geninv_mixed")
    if return_result:
        return MixedResult(Y, r.value, piv[: r.value], est.value, st)
    return Y, r.value


def mgemm(A: torch.Tensor, B: torch.Tensor, transA: bool = False, transB: bool = False, moduli: int = 16,
          lower: bool = False):
    """C = op(A) op(B) on the int8 modular engine (geninv_mgemm)."""
    _dev(A, "A")
    _dev(B, "B")
    Ac, lda = colmajor(A)
    Bc, ldb = colmajor(B)
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    if (B.shape[1] if transB else B.shape[0]) != K:
        raise ValueError("inner dimensions differ")
    C = empty_colmajor(M, N, A.device)
    if lower:
        C.zero_()
    if Ac.data_ptr() == Bc.data_ptr() and lda == ldb:
        Bc = Ac
    _check(load().geninv_mgemm(_ctx(A.device), int(transA), int(transB), M, N, K, _p(Ac), lda, _p(Bc), ldb,
                               int(moduli), int(lower), _p(C), max(1, M)), "geninv_mgemm")
    return C


def bslice(X: torch.Tensor, slices: int = 4, transposed: bool = False):
    """(planes, exponents): the 8-bit slices of X by column (or by row,
    transposed storage) as bfloat16 planes, and the exponents."""
    _dev(X, "X")
    rows, cols = X.shape
    Xc, ldx = colmajor(X)
    inner = cols if transposed else rows
    outer = rows if transposed else cols
    ldp = max(1, (inner + 63) // 64 * 64)
    planes = torch.empty((slices, outer, ldp), dtype=torch.bfloat16, device=X.device)
    e = torch.empty(max(1, outer), dtype=torch.int32, device=X.device)
    _check(load().geninv_bslice(_ctx(X.device), rows, cols, _p(Xc), ldx, int(slices), int(transposed), _p(planes),
                                ldp, _p(e)), "geninv_bslice")
    return planes, e[:outer]


def bgram(G: torch.Tensor, slices: int = 4):
    """Lower triangle (upper set to zero) of the sliced Gram matrix G_s'G_s."""
    _dev(G, "G")
    m, n = G.shape
    Gc, ldg = colmajor(G)
    A = empty_colmajor(n, n, G.device)
    A.zero_()
    _check(load().geninv_bgram(_ctx(G.device), m, n, _p(Gc), ldg, int(slices), _p(A), max(1, n)), "geninv_bgram")
    return A


class IncrementalLstsq:
    """Least squares W = G^+ F while columns are appended to G (Section 4's
    incremental learning): the Gram matrix G'G and G'F grow by the rows of
    the new columns (geninv_inc_gram), the full-rank Cholesky factor and
    (L'L)^-1 are extended rather than recomputed (geninv_inc_factor), and a
    solve applies them (geninv_factored_lstsq).  ``refactor=True`` instead
    runs the method from the Gram matrix on every solve
    (geninv_dlstsq_gram).  Column-major device buffers sized for ``nmax``
    columns are held here."""

    def __init__(self, nmax: int, k: int, device=None, tol: float | None = None, refactor: bool = False):
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.nmax, self.k, self.n = int(nmax), int(k), 0
        self.tol = float(tol or 0.0)
        self.refactor = refactor
        z = lambda: torch.zeros((self.nmax, self.nmax), dtype=torch.float64, device=self.device).t()
        self.A = z()
        self.B = torch.zeros((max(1, self.k), self.nmax), dtype=torch.float64, device=self.device).t()
        self.L, self.M = z(), z()
        self.piv = torch.zeros(self.nmax, dtype=torch.int32, device=self.device)
        self.dvals = torch.zeros(self.nmax, dtype=torch.float64, device=self.device)
        self.rank, self.tol_used, self.n_factored = 0, 0.0, 0

    def append(self, G: torch.Tensor, F: torch.Tensor):
        """G: m x n_total, the columns seen so far followed by the new ones; F: m x k."""
        _dev(G, "G")
        _dev(F, "F")
        m, n_total = G.shape
        if n_total > self.nmax or n_total < self.n or F.shape != (m, self.k):
            raise ValueError("G must hold the earlier columns first, at most nmax in all; F must be m x k")
        Gc, ldg = colmajor(G)
        Fc, ldf = colmajor(F)
        ctx = _ctx(self.device)
        _check(load().geninv_inc_gram(ctx, m, self.n, n_total - self.n, self.k, _p(Gc), ldg, _p(Fc),
                                      ldf, _p(self.A), self.nmax, _p(self.B), self.nmax), "geninv_inc_gram")
        self.n = n_total
        if not self.refactor:
            r = ctypes.c_int(self.rank)
            t = ctypes.c_double(self.tol_used)
            _check(load().geninv_inc_factor(ctx, self.n_factored, self.n - self.n_factored, _p(self.A), self.nmax,
                                            self.tol, _p(self.L), self.nmax, _p(self.piv), _p(self.dvals),
                                            _p(self.M), self.nmax, ctypes.byref(r), ctypes.byref(t)),
                   "geninv_inc_factor")
            self.rank, self.tol_used, self.n_factored = r.value, t.value, self.n

    def solve(self, tol: float | None = None):
        """(W, rank) for the columns appended so far."""
        W = empty_colmajor(self.n, self.k, self.device)
        if not self.refactor:
            _check(load().geninv_factored_lstsq(_ctx(self.device), self.n, self.rank, self.k, _p(self.L), self.nmax,
                                                _p(self.M), self.nmax, _p(self.B), self.nmax, _p(W), max(1, self.n)),
                   "geninv_factored_lstsq")
            return W, self.rank
        r = ctypes.c_int(0)
        _check(load().geninv_dlstsq_gram(_ctx(self.device), self.n, self.k, _p(self.A), self.nmax, _p(self.B),
                                         self.nmax, float(tol or self.tol or 0.0), _p(W), max(1, self.n),
                                         ctypes.byref(r)),
               "geninv_dlstsq_gram")
        return W, r.value

    def pivots(self):
        return self.piv[: self.rank]


def bchain(P: torch.Tensor, G: torch.Tensor, slices: int = 4):
    """Y = P G' as the mixed form's chain product (rows of P and G sliced)."""
    _dev(P, "P")
    _dev(G, "G")
    n, k = P.shape
    m = G.shape[0]
    if G.shape[1] != k:
        raise ValueError("P and G must have the same number of columns")
    Pc, ldp = colmajor(P)
    Gc, ldg = colmajor(G)
    Y = empty_colmajor(n, m, P.device)
    _check(load().geninv_bchain(_ctx(P.device), n, m, k, _p(Pc), ldp, _p(Gc), ldg, int(slices), _p(Y), max(1, n)),
           "geninv_bchain")
    return Y


def lstsq(G: torch.Tensor, F: torch.Tensor, tol: float | None = None):
    """W = G^+ F (n x k), minimum-norm least squares (Section 1); m < n
    takes the Appendix's transpose branch."""
    _dev(G, "G")
    _dev(F, "F")
    m, n = G.shape
    if F.shape[0] != m:
        raise ValueError("F must have as many rows as G")
    k = F.shape[1]
    Gc, ldg = colmajor(G)
    Fc, ldf = colmajor(F)
    W = empty_colmajor(n, k, G.device)
    r = ctypes.c_int(0)
    st = load().geninv_dlstsq(_ctx(G.device), m, n, k, _p(Gc), ldg, _p(Fc), ldf, float(tol or 0.0), _p(W),
                              max(1, n), ctypes.byref(r))
    _check(st, "geninv_dlstsq")
    return W, r.value


def gram(G: torch.Tensor, full: bool = True):
    """A = G'G (Section 2, Eq. (1)); lower triangle only when full=False (upper left unset)."""
    _dev(G, "G")
    m, n = G.shape
    Gc, ldg = colmajor(G)
    A = empty_colmajor(n, n, G.device)
    if not full:
        A.zero_()
    _check(load().geninv_dgram(_ctx(G.device), m, n, _p(Gc), ldg, _p(A), max(1, n), 1 if full else 0),
           "geninv_dgram")
    return A


@dataclass
class FrCholResult:
    L: torch.Tensor        # n x r
    rank: int
    piv: torch.Tensor      # int32 [r]
    d: torch.Tensor        # float64 [n], updated pivot values
    tol: float


def frchol(A: torch.Tensor, tol: float | None = None) -> FrCholResult:
    """Full-rank Cholesky with column dropping (Appendix loop) of the lower triangle of A."""
    _dev(A, "A")
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    Ac, lda = colmajor(A)
    L = empty_colmajor(n, n, A.device)
    piv = torch.empty(max(1, n), dtype=torch.int32, device=A.device)
    d = torch.empty(max(1, n), dtype=torch.float64, device=A.device)
    tu = torch.empty(1, dtype=torch.float64, device=A.device)
    r = ctypes.c_int(0)
    st = load().geninv_dfrchol(_ctx(A.device), n, _p(Ac), lda, float(tol or 0.0), _p(L), max(1, n), _p(piv),
                               _p(d), _p(tu), ctypes.byref(r))
    _check(st, "geninv_dfrchol")
    rv = r.value
    return FrCholResult(L[:, :rv], rv, piv[:rv], d[:n], float(tu.item()) if n else float("inf"))


def spd_inverse(B: torch.Tensor):
    """M = B^-1 for SPD B (Theorem 1, B = L'L), exactly symmetric."""
    _dev(B, "B")
    r = B.shape[0]
    Bc, ldb = colmajor(B)
    M = empty_colmajor(r, r, B.device)
    lib = load()
    c = _ctx(B.device)
    _check(lib.geninv_dspdinv(c, r, _p(Bc), ldb, _p(M), max(1, r)), "geninv_dspdinv")
    _check(lib.geninv_sync_status(c), "geninv_dspdinv (device status)")
    return M


def spd_inverse_ns(B: torch.Tensor, max_iter: int = 100):
    """(M, iterations, residual): M = B^-1 for SPD B by Newton-Schulz
    iteration on the matrix cores (geninv_dspdinv_ns)."""
    _dev(B, "B")
    r = B.shape[0]
    Bc, ldb = colmajor(B)
    M = empty_colmajor(r, r, B.device)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    _check(load().geninv_dspdinv_ns(_ctx(B.device), r, _p(Bc), ldb, _p(M), max(1, r), int(max_iter),
                                    ctypes.byref(it), ctypes.byref(res)), "geninv_dspdinv_ns")
    return M, it.value, res.value


def chain(L: torch.Tensor, M: torch.Tensor, G: torch.Tensor):
    """Y = L M M L' G' for given factors (Theorem 1)."""
    for t, nm in ((L, "L"), (M, "M"), (G, "G")):
        _dev(t, nm)
    m, n = G.shape
    r = L.shape[1]
    Lc, ldl = colmajor(L) if r > 0 else (L, max(1, n))
    Mc, ldm = colmajor(M) if r > 0 else (M, 1)
    Gc, ldg = colmajor(G)
    Y = empty_colmajor(n, m, G.device)
    _check(load().geninv_dchain(_ctx(G.device), m, n, r, _p(Lc), ldl, _p(Mc), ldm, _p(Gc), ldg, _p(Y), max(1, n)),
           "geninv_dchain")
    return Y


def dgemm(A: torch.Tensor, B: torch.Tensor, transA: bool = False, transB: bool = False, alpha: float = 1.0,
          beta: float = 0.0, C: torch.Tensor | None = None):
    """C = alpha op(A) op(B) + beta C with the library's float64 MFMA GEMM."""
    _dev(A, "A")
    _dev(B, "B")
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    Kb = B.shape[1] if transB else B.shape[0]
    if K != Kb:
        raise ValueError("inner dimensions differ")
    Ac, lda = colmajor(A)
    Bc, ldb = colmajor(B)
    if C is None:
        C = empty_colmajor(M, N, A.device)
        beta = 0.0
    else:
        _dev(C, "C")
        if C.stride(0) != 1:
            raise ValueError("C must be column-major")
    _check(load().geninv_dgemm(_ctx(A.device), int(transA), int(transB), M, N, K, float(alpha), _p(Ac), lda,
                               _p(Bc), ldb, float(beta), _p(C), max(1, C.stride(1) if N > 1 else M)),
           "geninv_dgemm")
    return C


def sync_status(device=None):
    """Wait for the stream; device-side status of the calls since the last check."""
    dev = torch.device("cuda", device if device is not None else torch.cuda.current_device())
    return load().geninv_sync_status(_ctx(dev))


class _PackedBatch:
    """G_b (m_b x n_b) and F_b (m_b x k), float32, packed column-major into
    two device buffers, with W_b (n_b x k, float64) and the ranks as outputs,
    and the C argument arrays (device pointers per problem, sizes) that the
    batched entry points take."""

    def __init__(self, Gs, Fs, device=None):
        import numpy as np
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.batch = len(Gs)
        if self.batch != len(Fs):
            raise ValueError("Gs and Fs differ in length")
        self.m = np.array([g.shape[0] for g in Gs], dtype=np.int32)
        self.n = np.array([g.shape[1] for g in Gs], dtype=np.int32)
        ks = {f.shape[1] for f in Fs}
        if len(ks) != 1:
            raise ValueError("every F_b needs the same number of columns")
        self.k = ks.pop()
        self.g_off = np.concatenate([[0], np.cumsum(self.m.astype(np.int64) * self.n)])
        self.f_off = np.concatenate([[0], np.cumsum(self.m.astype(np.int64) * self.k)])
        self.w_off = np.concatenate([[0], np.cumsum(self.n.astype(np.int64) * self.k)])
        self.Gbuf = torch.empty(int(self.g_off[-1]), dtype=torch.float32, device=self.device)
        self.Fbuf = torch.empty(int(self.f_off[-1]), dtype=torch.float32, device=self.device)
        self.Wbuf = torch.zeros(int(self.w_off[-1]), dtype=torch.float64, device=self.device)
        self.rank = torch.zeros(max(1, self.batch), dtype=torch.int32, device=self.device)
        self.load(Gs, Fs)
        vp = ctypes.c_void_p
        gb, fb, wb = self.Gbuf.data_ptr(), self.Fbuf.data_ptr(), self.Wbuf.data_ptr()
        self.Gp = (vp * self.batch)(*[gb + 4 * int(o) for o in self.g_off[:-1]])
        self.Fp = (vp * self.batch)(*[fb + 4 * int(o) for o in self.f_off[:-1]])
        self.Wp = (vp * self.batch)(*[wb + 8 * int(o) for o in self.w_off[:-1]])
        ci = ctypes.c_int * self.batch
        self.m_c, self.n_c = ci(*self.m.tolist()), ci(*self.n.tolist())

    def load(self, Gs, Fs):
        """Copy new G_b, F_b (same shapes) into the plan's packed buffers."""
        import numpy as np
        g = np.concatenate([np.asarray(x, np.float32).ravel(order="F") for x in Gs]) if self.batch else np.zeros(0)
        f = np.concatenate([np.asarray(x, np.float32).ravel(order="F") for x in Fs]) if self.batch else np.zeros(0)
        self.Gbuf.copy_(torch.from_numpy(g.astype(np.float32)))
        self.Fbuf.copy_(torch.from_numpy(f.astype(np.float32)))

    def W(self, b: int):
        o = int(self.w_off[b])
        n = int(self.n[b])
        return self.Wbuf[o:o + n * self.k].view(self.k, n).t()


class AutotuneResult(NamedTuple):
    nl: int
    grid: int
    ms: float
    from_cache: bool


class BatchPlan(_PackedBatch):
    """Batched least squares W_b = G_b^+ F_b (geninv_batch_plan_*).

    G_b (m_b x n_b) and F_b (m_b x k) are float32; they are packed
    column-major into two device buffers owned by the plan (``load`` refills
    them in place).  W_b (n_b x k, float64) and the ranks are outputs.
    """

    def __init__(self, Gs, Fs, tol: float | None = None, device=None):
        super().__init__(Gs, Fs, device)
        lib = load()
        h = ctypes.c_void_p()
        self._lib = lib
        self._ctx = _ctx(self.device)
        _check(lib.geninv_batch_plan_create(self._ctx, ctypes.byref(h), self.batch, self.m_c, self.n_c, self.k,
                                            self.Gp, self.m_c, self.Fp, self.m_c, self.Wp, self.n_c,
                                            float(tol or 0.0), _p(self.rank)),
               "geninv_batch_plan_create")
        self._plan = h

    def enable_pivots(self):
        """Allocate per-problem pivot outputs (geninv_batch_plan_set_pivots);
        piv(b) then returns the kept column indices of problem b."""
        import numpy as np
        self.p_off = np.concatenate([[0], np.cumsum(self.n.astype(np.int64))])
        self.Pbuf = torch.zeros(max(1, int(self.p_off[-1])), dtype=torch.int32, device=self.device)
        pb = self.Pbuf.data_ptr()
        self.Pp = (ctypes.c_void_p * self.batch)(*[pb + 4 * int(o) for o in self.p_off[:-1]])
        _check(self._lib.geninv_batch_plan_set_pivots(self._plan, self.Pp), "geninv_batch_plan_set_pivots")

    def piv(self, b: int):
        o = int(self.p_off[b])
        return self.Pbuf[o:o + int(self.rank[b])]

    def run(self, use_graph: bool = True):
        _ctx(self.device)   # follow torch's current stream
        _check(self._lib.geninv_batch_plan_run(self._plan, int(use_graph)), "geninv_batch_plan_run")

    def graph_fallbacks(self) -> int:
        """Runs that asked for the graph and launched directly
        (geninv_batch_plan_graph_fallbacks)."""
        return int(self._lib.geninv_batch_plan_graph_fallbacks(self._plan))

    def autotune(self, reps: int = 3, cache: str | None = None):
        """geninv_batch_plan_autotune: (nl, grid, ms, from_cache)."""
        _ctx(self.device)
        nl, grid, fc = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        ms = ctypes.c_double(0.0)
        path = None if cache is None else os.fsencode(cache)
        _check(self._lib.geninv_batch_plan_autotune(self._plan, reps, path, ctypes.byref(nl), ctypes.byref(grid),
                                                    ctypes.byref(ms), ctypes.byref(fc)), "geninv_batch_plan_autotune")
        return AutotuneResult(nl.value, grid.value, ms.value, bool(fc.value))

    def config(self, nl: int | None = None, grid: int | None = None):
        """Set (when nl and grid are given) and return the launch
        configuration (nl, grid)."""
        if nl is not None and grid is not None:
            _check(self._lib.geninv_batch_plan_config(self._plan, int(nl), int(grid)), "geninv_batch_plan_config")
        a, b = ctypes.c_int(0), ctypes.c_int(0)
        _check(self._lib.geninv_batch_plan_get_config(self._plan, ctypes.byref(a), ctypes.byref(b)),
               "geninv_batch_plan_get_config")
        return a.value, b.value

    def close(self):
        if getattr(self, "_plan", None):
            self._lib.geninv_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lstsq_batched(Gs, Fs, tol: float | None = None, device=None):
    """One-shot batched least squares (geninv_lstsq_batched): W_b = G_b^+ F_b
    for float32 G_b, F_b.  Synchronizes.  Returns (packed batch with ``W(b)``
    and ``rank``, device status word)."""
    pb = _PackedBatch(Gs, Fs, device)
    st = ctypes.c_int(0)
    _check(load().geninv_lstsq_batched(_ctx(pb.device), pb.batch, pb.m_c, pb.n_c, pb.k, pb.Gp, pb.m_c, pb.Fp,
                                       pb.m_c, float(tol or 0.0), pb.Wp, pb.n_c, _p(pb.rank), ctypes.byref(st)),
           "geninv_lstsq_batched")
    return pb, st.value
