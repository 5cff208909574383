"""The allocation-free least-squares entry point (geninv_dlstsq_noalloc)
against geninv_dlstsq, through the C ABI.

Both run the same kernels on the same workspace layout, the first in the
library's fixed device scratch array, the second in the context's
workspace, so W and the rank must agree bit for bit; two calls in a row
(the second smaller, so the array holds the first call's larger contents)
and the transpose branch; sizes beyond the array are refused before
anything is enqueued.
"""
import ctypes

import numpy as np
import pytest

from oracle import geninv_ref as o
from paper_0804_4809_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_0804_4809_amd import api  # noqa: E402
from paper_0804_4809_amd._lib import load  # noqa: E402

DEV = torch.device("cuda", 0)
ESCRATCH = -8


def _call(lib, ctx, fn, G, F):
    m, n = G.shape
    k = F.shape[1]
    Gc, ldg = api.colmajor(G)
    Fc, ldf = api.colmajor(F)
    W = api.empty_colmajor(n, k, DEV)
    W.fill_(float("nan"))
    r = ctypes.c_int(-1)
    st = getattr(lib, fn)(ctx, m, n, k, ctypes.c_void_p(Gc.data_ptr()), ldg, ctypes.c_void_p(Fc.data_ptr()), ldf,
                          0.0, ctypes.c_void_p(W.data_ptr()), n, ctypes.byref(r))
    torch.cuda.synchronize()
    return st, W, r.value


def test_noalloc_matches_dlstsq_two_calls_in_a_row():
    lib = load()
    ctx = ctypes.c_void_p()
    assert lib.geninv_create(ctypes.byref(ctx), 0, None) == 0     # a fresh context, empty workspace
    try:
        for m, n, k, r, seed in [(3000, 700, 4, 500, 1), (900, 129, 2, 100, 2), (300, 800, 3, 250, 3)]:
            print(f"[case] noalloc m={m} n={n} k={k} r={r}", flush=True)
            G, F = w.lowrank_uv(m, n, r, seed=seed, k=k)
            Gd = torch.from_numpy(G).to(DEV)
            Fd = torch.from_numpy(F).to(DEV)
            st, Wn, rn = _call(lib, ctx, "geninv_dlstsq_noalloc", Gd, Fd)
            assert st == 0, st
            st, Wr, rr = _call(lib, ctx, "geninv_dlstsq", Gd, Fd)
            assert st == 0, st
            assert rn == rr == r
            assert torch.equal(Wn, Wr)
            Wo, ref = o.lstsq(G, F)
            assert o.rel_fro(Wn.cpu().numpy(), Wo) <= max(1e-10, 10 * o.self_spread(G, base=ref))
    finally:
        lib.geninv_destroy(ctx)


def test_noalloc_refuses_sizes_beyond_the_scratch_array():
    lib = load()
    cap = lib.geninv_noalloc_capacity()
    assert cap == 256 << 20
    ctx = api._ctx(DEV)
    n = 4096                                  # four n x n float64 slots alone need 512 MiB
    assert lib.geninv_workspace_bytes(n, n, 1, 0, 0, 0, 0) > cap
    G = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    F = torch.zeros((n, 1), dtype=torch.float64, device=DEV)
    st, W, r = _call(lib, ctx, "geninv_dlstsq_noalloc", G, F)
    assert st == ESCRATCH
    assert torch.isnan(W).all()               # nothing was enqueued
