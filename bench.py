#!/usr/bin/env python3
"""Benchmark of the full-rank-Cholesky Moore-Penrose inverse on one MI355X.

One step = the whole float64 method on the large RBF design workload
(131072 inputs uniform in [0,1]^8, 8192 Gaussian centers with sigma 0.5 of
which 1192 are exact duplicates of earlier ones, F 131072 x 16): Gram
matrix, tolerance, full-rank Cholesky with column dropping, (L'L)^-1,
Y = L M M L' G', and the least-squares weights W = Y F.  Inputs are resident
in HBM before timing.  ``--workload c2`` times the 8192 x 2048 RBF design
(sigma 0.3, 256 duplicates, F 8192 x 8) instead.

Prints one JSON line.  `value` is algorithmic TFLOP/s of the step (the flop
model of `algorithmic_flops` below); `roofline` covers the kernel class that
takes the most time, timed with HIP events on the library's stream during the
timed steps; `cpu_baseline` is the float64 CPU oracle timed on a row sample
of the same design.  `forms` adds the mixed-precision form beside the
float64 one on the same input, the smaller RBF design with its accuracy
against the oracle, the mixed form on G = P diag(s) Q', the batched form,
the paper's Table 1 sweep, incremental least squares and the two inverses
of L'L.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--skip-forms] [--workload c5|c2]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

try:
    _CORES = len(os.sched_getaffinity(0))
except AttributeError:  # pragma: no cover
    _CORES = os.cpu_count() or 1
os.environ.setdefault("OPENBLAS_NUM_THREADS", str(_CORES))

METRIC = "geninv time & TFLOP/s, mixed vs FP64 at ≤1e-6 rel err; batched solves/sec"
FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def algorithmic_flops(m: int, n: int, r_before, r: int, k: int = 0) -> float:
    """Flops of the method as the paper states it (2 per multiply-add).

    Gram m n(n+1); Cholesky sum_k 2(n-k) r_k (+ n square roots/divisions
    ignored); L'L n r(r+1); inverse r^3; chain 2 n r^2 + n(n+1) r + 2 n^2 m;
    W = Y F 2 n m k.  r_before[k] is the rank before column k."""
    f = m * n * (n + 1.0)
    f += sum(2.0 * (n - kk) * rk for kk, rk in enumerate(r_before))
    f += n * r * (r + 1.0) + float(r) ** 3
    f += 2.0 * n * r * r + n * (n + 1.0) * r + 2.0 * n * n * m
    f += 2.0 * n * m * k
    return f


def lstsq_flops(m: int, n: int, r: int, k: int) -> float:
    """Least-squares variant of the model: the chain is replaced by
    (2mn + 4nr + 4r^2) k for W = L (M (M (L' (G'F)))); the Cholesky term uses
    r_k = min(k, r), exact for generic exact-rank inputs."""
    f = m * n * (n + 1.0)
    f += sum(2.0 * (n - kk) * min(kk, r) for kk in range(n))
    f += n * r * (r + 1.0) + float(r) ** 3
    f += (2.0 * m * n + 4.0 * n * r + 4.0 * r * r) * k
    return f


def _counter_traffic(kernel_class: str, tag: str):
    """HBM bytes per launch of `kernel_class` (FETCH_SIZE + WRITE_SIZE, scaled
    by a plain copy) from the committed counter summary of workload `tag`, or
    None when the summary has no such line or the kernel sources changed
    since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"fp64_{tag}_hbm_bytes.md")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    for line in lines:
        if not line.startswith(f"traffic {kernel_class} "):
            continue
        fields = dict(f.split("=", 1) for f in line.split()[2:] if "=" in f and not f.startswith('kernel'))
        h = hashlib.sha256()
        for src in fields["sources"].split(","):
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != fields["sha256_16"]:
            return None
        return int(fields["read_bytes"]) + int(fields["write_bytes"])
    return None


def _finite(x):
    """The report with non-finite numbers (e.g. an infinite rounding spread
    where a perturbed Gram matrix changes the rank) as null: strict JSON."""
    if isinstance(x, dict):
        return {k: _finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_finite(v) for v in x]
    if isinstance(x, float) and not math.isfinite(x):
        return None
    return x


def _timed(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) * 1e3 / steps


# mixed-form variants: (key, precision, gram digits, chain digits, Newton-Schulz steps)
# precision 1 = bfloat16 slices (digits = 8-bit slices), 2 = int8 residues
# (digits = moduli; 16 give float64-accurate products)
MIXED_C3 = [
    ("int8_m16", 2, 16, 16, 0),
    ("int8_m13", 2, 13, 13, 0),
    ("int8_g13_c10", 2, 13, 10, 0),
    ("int8_g10_c10", 2, 10, 10, 0),
    ("int8_m16_ns1", 2, 16, 16, 1),
    ("bf16_s4", 1, 4, 4, 0),
    ("bf16_s4_ns1", 1, 4, 4, 1),
]
MIXED_C5 = [
    ("int8_m16", 2, 16, 16, 0),
    ("int8_m16_ns1", 2, 16, 16, 1),
    ("bf16_s4", 1, 4, 4, 0),
]


def _mixed_call(lib, ctx, m, n, G, ldg, Y, variant, rank=None, est=None):
    _, prec, gd, cd, ns = variant
    return lib.geninv_mixed(ctx, m, n, ctypes.c_void_p(G.data_ptr()), ldg, 0.0, prec, gd, cd, ns, 0.0,
                            ctypes.c_void_p(Y.data_ptr()), n, rank, None, est)


def bench_mixed(lib, api, workloads, torch, np, steps, keep_host):
    """Mixed-precision form vs the float64 form on G = P diag(s) Q'
    (32768 x 4096, rank 3072, s log-spaced in [1e-3, 1]).  Returns the
    report and, with ``keep_host``, host copies of every Y for the oracle leg."""
    G, _, P, sv, Q = workloads.c3_problem()
    m, n = G.shape
    dev = torch.device("cuda", 0)
    Gd = torch.from_numpy(G).to(dev)
    Gc, ldg = api.colmajor(Gd)
    del Gd
    ctx = api._ctx(dev)
    vp = ctypes.c_void_p
    Y64 = api.empty_colmajor(n, m, dev)
    Ymx = api.empty_colmajor(n, m, dev)
    piv = torch.empty(n, dtype=torch.int32, device=dev)
    out = {"workload": "G = P diag(s) Q', m=32768, n=4096, rank 3072, s log-spaced from 1 to 1e-3"}
    host = {"G": G, "P": P, "sv": sv, "Q": Q, "Y": {}} if keep_host else None

    def run64():
        st = lib.geninv_dgeninv(ctx, m, n, vp(Gc.data_ptr()), ldg, 0.0, vp(Y64.data_ptr()), n, None, None)
        assert st == 0, st


    r_c = ctypes.c_int(0)
    lib.geninv_dgeninv(ctx, m, n, vp(Gc.data_ptr()), ldg, 0.0, vp(Y64.data_ptr()), n, ctypes.byref(r_c),
                       vp(piv.data_ptr()))
    r = r_c.value
    acc = np.zeros(n, bool)
    acc[piv[:r].cpu().numpy()] = True
    r_before = np.concatenate([[0], np.cumsum(acc)[:-1]])
    flops = algorithmic_flops(m, n, r_before, r)
    sync = torch.cuda.synchronize
    run64()
    t64 = _timed(run64, steps, sync)
    out["fp64"] = {"ms": round(t64, 3), "tflops": round(flops / t64 / 1e9, 3), "rank": r}
    if host is not None:
        host["Y"]["fp64"] = Y64.cpu().numpy()
    for variant in MIXED_C3:
        key = variant[0]

        def f():
            st = _mixed_call(lib, ctx, m, n, Gc, ldg, Ymx, variant)
            assert st == 0, st
        r2 = ctypes.c_int(0)
        est = ctypes.c_double(0.0)
        st = _mixed_call(lib, ctx, m, n, Gc, ldg, Ymx, variant, ctypes.byref(r2), ctypes.byref(est))
        assert st == 0, st
        t = _timed(f, steps, sync)
        out[key] = {"ms": round(t, 3), "tflops_fp64_equivalent": round(flops / t / 1e9, 3), "rank": r2.value,
                    "speedup_vs_fp64": round(t64 / t, 3), "err_est": est.value,
                    "relF_vs_fp64_gpu": float(torch.linalg.norm(Ymx - Y64) / torch.linalg.norm(Y64))}
        if host is not None:
            host["Y"][key] = Ymx.cpu().numpy()
    del Gc, Y64, Ymx
    torch.cuda.empty_cache()
    return out, host


def _incremental_run(api, torch, Gd, Fd, first, batch, steps):
    m, n = Gd.shape
    k = Fd.shape[1]
    sync = torch.cuda.synchronize
    # warm every path at the full size (the context's workspace grows to what
    # the largest factorization and the largest incremental step need, so no
    # timed call allocates): the first columns, then all of them in one append
    for refactor in (False, True):
        inc = api.IncrementalLstsq(n, k, refactor=refactor)
        inc.append(Gd[:, :first], Fd)
        inc.solve()
        inc.append(Gd, Fd)
        inc.solve()
    api.lstsq(Gd, Fd)
    incs = {False: api.IncrementalLstsq(n, k), True: api.IncrementalLstsq(n, k, refactor=True)}
    rows = []
    n_t = 0
    for n_new in [first] + list(range(first + batch, n + 1, batch)):
        Gv = Gd[:, :n_new]
        res = {}
        for refactor, inc in incs.items():
            sync()
            t0 = time.perf_counter()
            inc.append(Gv, Fd)
            Wi, ri = inc.solve()
            sync()
            res[refactor] = ((time.perf_counter() - t0) * 1e3, Wi, ri)
        one = []
        for _ in range(max(1, steps)):
            sync()
            t0 = time.perf_counter()
            W_one, r_one = api.lstsq(Gv, Fd)
            sync()
            one.append((time.perf_counter() - t0) * 1e3)
        t_one = sorted(one)[len(one) // 2]
        t_inc, W_inc, r_inc = res[False]
        t_ref, W_ref, r_ref = res[True]
        rows.append({"columns": n_new, "appended": n_new - n_t, "incremental_factor_ms": round(t_inc, 3),
                     "refactor_from_gram_ms": round(t_ref, 3), "one_shot_ms": round(t_one, 3),
                     "speedup_vs_one_shot": round(t_one / t_inc, 2),
                     "rank_incremental": r_inc, "rank_refactor": r_ref, "rank_one_shot": r_one,
                     "relF_W_incremental_vs_one_shot": float(torch.linalg.norm(W_inc - W_one) / torch.linalg.norm(W_one)),
                     "relF_W_refactor_vs_one_shot": float(torch.linalg.norm(W_ref - W_one) / torch.linalg.norm(W_one))})
        n_t = n_new
    return rows


def bench_incremental(lib, api, workloads, torch, np, steps):
    """Incremental least squares (appended Gram and G'F rows; the factor and
    (L'L)^-1 extended, or the method rerun from the Gram matrix) against
    geninv_dlstsq on the whole matrix so far, on the RBF design and on a tall
    low-rank matrix.  Times include each call's host synchronizations."""
    dev = torch.device("cuda", 0)
    out = {}
    G, F, _ = workloads.c2_problem()
    Gd = torch.from_numpy(G).to(dev).t().contiguous().t()
    Fd = torch.from_numpy(F).to(dev).t().contiguous().t()
    out["rbf_8192x2048"] = {"workload": "RBF design 8192 x 2048 (sigma 0.3, 256 duplicate centers), F 8192 x 8: "
                                        "1536 centers, then 4 x 128 appended",
                            "steps": _incremental_run(api, torch, Gd, Fd, 1536, 128, steps)}
    del Gd, Fd
    G, F = workloads.lowrank_uv(131072, 1024, 896, seed=5, k=8)
    Gd = torch.from_numpy(G).to(dev).t().contiguous().t()
    Fd = torch.from_numpy(F).to(dev).t().contiguous().t()
    del G, F
    out["tall_131072x1024"] = {"workload": "G = U V, 131072 x 1024 of rank 896 (N(0,1) factors), F 131072 x 8: "
                                           "768 columns, then 2 x 128 appended",
                               "steps": _incremental_run(api, torch, Gd, Fd, 768, 128, steps)}
    del Gd, Fd
    torch.cuda.empty_cache()
    return out


def bench_spd_inverse(lib, api, workloads, torch, np, steps):
    """The inverse of L'L two ways on the GPU: the Gauss-Jordan sweep of the
    method's path (geninv_dspdinv) and Newton-Schulz iteration on the matrix
    cores (geninv_dspdinv_ns), on the L'L of the RBF (8192 x 2048) and SVD
    family (32768 x 4096) workloads."""
    dev = torch.device("cuda", 0)
    sync = torch.cuda.synchronize
    out = {}
    for name, G in (("rbf_8192x2048", workloads.c2_problem()[0]), ("svd_32768x4096", workloads.c3_problem()[0])):
        Gd = torch.from_numpy(G).to(dev)
        del G
        A = api.gram(Gd)
        del Gd
        fr = api.frchol(A)
        L = fr.L
        B = api.dgemm(L, L, transA=True)
        del A, fr
        M_gj = api.spd_inverse(B)
        t_gj = _timed(lambda: api.spd_inverse(B), steps, sync)
        M_ns, iters, resid = api.spd_inverse_ns(B)
        t_ns = _timed(lambda: api.spd_inverse_ns(B), max(1, steps // 2), sync)
        r = B.shape[0]
        eye = torch.eye(r, dtype=torch.float64, device=dev)
        res_gj = float(torch.linalg.norm(eye - B @ M_gj) / r ** 0.5)
        out[name] = {"r": r, "gauss_jordan_ms": round(t_gj, 3), "newton_schulz_ms": round(t_ns, 3),
                     "newton_schulz_iterations": iters, "residual_newton_schulz": resid,
                     "residual_gauss_jordan": res_gj,
                     "relF_between": float(torch.linalg.norm(M_ns - M_gj) / torch.linalg.norm(M_gj))}
        del B, L, M_gj, M_ns, eye
    torch.cuda.empty_cache()
    return out


def bench_table1(lib, api, workloads, torch, np, steps):
    """The paper's timing family (Section 3, Table 1): m = 2n, rank 7n/8,
    entries in [-1, 1], float64 geninv on the GPU, with the four Penrose
    error matrices checked against the paper's 2e-10 bound.  The paper's own
    geninv times (Matlab 6.5.1 on a personal computer) are quoted beside."""
    with open(os.path.join(ROOT, "tests", "golden", "paper_table1.json")) as fh:
        paper = json.load(fh)
    dev = torch.device("cuda", 0)
    ctx = api._ctx(dev)
    vp = ctypes.c_void_p
    rows = []
    for n in [32, 64, 128, 256, 512, 1024, 2048]:
        G = workloads.table1(n, n)
        m = G.shape[0]
        Gd = torch.from_numpy(G).to(dev).t().contiguous().t()
        Y = torch.empty((n, m), dtype=torch.float64, device=dev).t().contiguous().t()
        r = ctypes.c_int(0)

        def f():
            st = lib.geninv_dgeninv(ctx, m, n, vp(Gd.data_ptr()), m, 0.0, vp(Y.data_ptr()), n, None, None)
            assert st == 0, st

        st = lib.geninv_dgeninv(ctx, m, n, vp(Gd.data_ptr()), m, 0.0, vp(Y.data_ptr()), n, ctypes.byref(r), None)
        assert st == 0, st
        times = []
        for _ in range(max(3, steps)):
            times.append(_timed(f, 1, torch.cuda.synchronize))
        ms = sorted(times)[len(times) // 2]
        GY, YG = Gd @ Y, Y @ Gd
        pen = max(float((GY @ Gd - Gd).abs().max()), float((YG @ Y - Y).abs().max()),
                  float((GY.t() - GY).abs().max()), float((YG.t() - YG).abs().max()))
        row = {"n": n, "m": m, "rank": r.value, "rank_expected": 7 * n // 8, "gpu_ms": round(ms, 3),
               "penrose_max_abs": pen}
        if str(n) in paper["geninv_seconds"]:
            row["paper_geninv_s"] = paper["geninv_seconds"][str(n)]
        rows.append(row)
        del Gd, Y, GY, YG
    return {"workload": paper["workload"], "penrose_bound": paper["penrose_max_abs_bound"],
            "paper_hardware": "Matlab 6.5.1 on an unnamed personal computer (Section 3); context, not a target",
            "rows": rows}


def bench_batched(api, workloads, torch, np, steps, keep_host):
    """4096 uneven float32 least-squares problems in one persistent launch,
    replayed from a HIP graph after autotuning."""
    B = workloads.c4_problem()
    plan = api.BatchPlan(B.G, B.F)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tuned = plan.autotune(reps=2)
        plan.run(use_graph=True)
        stream.synchronize()
        t = _timed(lambda: plan.run(use_graph=True), steps, stream.synchronize)
    ranks = plan.rank.cpu().numpy()
    flops = sum(lstsq_flops(int(B.m[b]), int(B.n[b]), int(ranks[b]), B.k) for b in range(len(B.G)))
    out = {"workload": "4096 problems, m ~ U[64,1024], n ~ U[16, min(256, m/2)], rank ~ U[n/2, n], G = U V and "
                       "F (m x 4) stored in float32, float64 accumulation and pivots",
           "ms": round(t, 3), "solves_per_s": round(len(B.G) / (t * 1e-3), 1), "tflops": round(flops / t / 1e9, 3),
           "autotuned": {"lds_threshold": tuned.nl, "workgroups": tuned.grid, "ms": round(tuned.ms, 3)},
           "rank_equals_construction": int((ranks == B.rank).sum())}
    # the same 4096 problems through the plain float64 form, one geninv_dlstsq
    # call per problem on the library's stream (float32 inputs widened exactly)
    lib = api.load()
    dev = torch.device("cuda", 0)
    ctx = api._ctx(dev)
    vp = ctypes.c_void_p
    Gs = [torch.from_numpy(g.astype(np.float64)).to(dev).t().contiguous().t() for g in B.G]
    Fs = [torch.from_numpy(f.astype(np.float64)).to(dev).t().contiguous().t() for f in B.F]
    Ws = [torch.empty((int(B.n[b]), B.k), dtype=torch.float64, device=dev).t().contiguous().t()
          for b in range(len(B.G))]

    def run64():
        for b in range(len(B.G)):
            m_b, n_b = int(B.m[b]), int(B.n[b])
            st = lib.geninv_dlstsq(ctx, m_b, n_b, B.k, vp(Gs[b].data_ptr()), m_b, vp(Fs[b].data_ptr()), m_b, 0.0,
                                   vp(Ws[b].data_ptr()), n_b, None)
            assert st == 0, st

    # the float64 form reads each problem's rank back to the host once per
    # call by default (geninv_set_host_sync); timed both with that
    # synchronization and without it (later launches sized for n_b)
    run64()
    t64_sync = _timed(run64, 2, torch.cuda.synchronize)
    api.set_host_sync(False, dev)
    try:
        run64()
        t64 = _timed(run64, 2, torch.cuda.synchronize)
    finally:
        api.set_host_sync(True, dev)
    rel = np.array([float(torch.linalg.norm(plan.W(b) - Ws[b]) / torch.linalg.norm(Ws[b]))
                    for b in range(len(B.G))])
    # ranks of the float64 form (one synchronous call per problem, untimed)
    r64 = np.zeros(len(B.G), dtype=np.int64)
    rc = ctypes.c_int(0)
    for b in range(len(B.G)):
        m_b, n_b = int(B.m[b]), int(B.n[b])
        st = lib.geninv_dlstsq(ctx, m_b, n_b, B.k, vp(Gs[b].data_ptr()), m_b, vp(Fs[b].data_ptr()), m_b, 0.0,
                               vp(Ws[b].data_ptr()), n_b, ctypes.byref(rc))
        assert st == 0, st
        r64[b] = rc.value
    same = r64 == ranks
    out["fp64_form"] = {"ms": round(t64, 3), "solves_per_s": round(len(B.G) / (t64 * 1e-3), 1),
                        "ms_with_rank_readback": round(t64_sync, 3),
                        "note": "geninv_dlstsq once per problem on the library's stream, float64 inputs; 'ms' "
                                "with geninv_set_host_sync(0) (no host synchronization inside or between "
                                "calls), 'ms_with_rank_readback' with the default one rank read-back per call"}
    out["speedup_vs_fp64_form"] = round(t64 / t, 2)
    out["speedup_vs_fp64_form_with_rank_readback"] = round(t64_sync / t, 2)
    out["rank_equals_fp64_form"] = int(same.sum())
    out["relF_vs_fp64_form_same_rank"] = {"median": float(np.median(rel[same])), "max": float(rel[same].max()),
                                          "above_1e-6": int((rel[same] > 1e-6).sum())}

    host = None
    if keep_host:
        rng = np.random.default_rng(0)
        sample = [int(b) for b in rng.choice(len(B.G), size=16, replace=False)]
        # same-rank problems where the two GPU forms differ by more than
        # 1e-6: both against the oracle in the oracle leg
        outl = [int(b) for b in np.nonzero(same & (rel > 1e-6))[0][:16]]
        host = {"B": B, "sample": {b: plan.W(b).cpu().numpy() for b in sample},
                "outliers": {b: (plan.W(b).cpu().numpy(), Ws[b].cpu().numpy()) for b in outl},
                "rank_batched": ranks.copy(), "rank_fp64": r64, "differs": [int(b) for b in np.nonzero(~same)[0]]}
    del Gs, Fs, Ws
    plan.close()
    return out, host


WORKLOADS = {
    "c5": ("rbf_131072x8192",
           "float64 geninv + W = G^+ F on a Gaussian RBF design matrix: m=131072 inputs uniform in [0,1]^8, "
           "n=8192 centers (7000 uniform + 1192 exact duplicates), sigma=0.5, F 131072x16"),
    "c2": ("rbf_8192x2048",
           "float64 geninv + W = G^+ F on a Gaussian RBF design matrix: m=8192 inputs uniform in [0,1]^4, "
           "n=2048 centers (1792 uniform + 256 exact duplicates), sigma=0.3, F 8192x8"),
}


def _generate(workloads, key):
    if key == "c5":
        G, F, _ = workloads.c5_problem()
    else:
        G, F, _ = workloads.c2_problem()
    return G, F


def _upload_colmajor(torch, X, dev):
    """Host row-major array -> device column-major tensor (copy through a
    transposed device view, no second host copy)."""
    T = torch.from_numpy(X).to(dev)
    C = T.t().contiguous().t()
    del T
    return C


def _gpu_quality(torch, Gd, Y, Fd, W):
    """Backward-stable figures of merit of a pseudoinverse on the GPU:
    ||G Y G - G||_F / ||G||_F and the least-squares residual ||G W - F|| / ||F||
    (products in torch, outside any timed region)."""
    YG = Y @ Gd
    gyg = float(torch.linalg.norm(Gd @ YG - Gd) / torch.linalg.norm(Gd))
    del YG
    ls = float(torch.linalg.norm(Gd @ W - Fd) / torch.linalg.norm(Fd))
    return {"gyg_minus_g_relF": gyg, "ls_residual": ls}


class Fp64Step:
    """The timed step: geninv_dgeninv (Y, rank, pivots) then W = Y F with the
    library's GEMM, on device-resident inputs."""

    def __init__(self, lib, api, torch, np, G, F, dev):
        self.lib, self.torch, self.np = lib, torch, np
        self.m, self.n = G.shape
        self.k = F.shape[1]
        self.Gd = _upload_colmajor(torch, G, dev)
        self.Fd = _upload_colmajor(torch, F, dev)
        self.Y = api.empty_colmajor(self.n, self.m, dev)
        self.W = api.empty_colmajor(self.n, self.k, dev)
        self.piv = torch.empty(self.n, dtype=torch.int32, device=dev)
        self.ctx = api._ctx(dev)

    def __call__(self, rank=None):
        vp = ctypes.c_void_p
        st = self.lib.geninv_dgeninv(self.ctx, self.m, self.n, vp(self.Gd.data_ptr()), self.m, 0.0,
                                     vp(self.Y.data_ptr()), self.n, rank, vp(self.piv.data_ptr()))
        if st != 0:
            raise RuntimeError(f"geninv_dgeninv failed: {st}")
        st = self.lib.geninv_dgemm(self.ctx, 0, 0, self.n, self.k, self.m, 1.0, vp(self.Y.data_ptr()), self.n,
                                   vp(self.Fd.data_ptr()), self.m, 0.0, vp(self.W.data_ptr()), self.n)
        if st != 0:
            raise RuntimeError(f"geninv_dgemm failed: {st}")

    def rank_and_flops(self):
        r_c = ctypes.c_int(0)
        self(ctypes.byref(r_c))
        r = r_c.value
        pv = self.piv[:r].cpu().numpy()
        acc = self.np.zeros(self.n, bool)
        acc[pv] = True
        r_before = self.np.concatenate([[0], self.np.cumsum(acc)[:-1]])
        return r, pv, algorithmic_flops(self.m, self.n, r_before, r, self.k)

    def free(self):
        del self.Gd, self.Fd, self.Y, self.W, self.piv


def measure_fp64(lib, step, steps, warmup, torch, tag):
    """Warm-up, rank and flops, one step with every kernel class timed (the
    dominant class), then `steps` timed steps with event timers on that class
    only.  Returns (report, roofline, per-class ms of one step)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    r, pv, flops = step.rank_and_flops()
    ctx = step.ctx
    ncls = lib.geninv_prof_classes()
    names = [lib.geninv_prof_name(c).decode() for c in range(ncls)]
    lib.geninv_prof_enable(ctx, (1 << ncls) - 1)
    step()
    torch.cuda.synchronize()
    per_class = {}
    for c in range(ncls):
        t = ctypes.c_double(0.0)
        cnt = ctypes.c_long(0)
        fl = ctypes.c_double(0.0)
        lib.geninv_prof_read(ctx, c, ctypes.byref(t), ctypes.byref(cnt), ctypes.byref(fl))
        per_class[names[c]] = (t.value, cnt.value, fl.value)
    dom = max(per_class, key=lambda name: per_class[name][0])
    dom_idx = names.index(dom)
    lib.geninv_prof_enable(ctx, 1 << dom_idx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps
    dt = ctypes.c_double(0.0)
    dcnt = ctypes.c_long(0)
    dfl = ctypes.c_double(0.0)
    lib.geninv_prof_read(ctx, dom_idx, ctypes.byref(dt), ctypes.byref(dcnt), ctypes.byref(dfl))
    lib.geninv_prof_enable(ctx, 0)
    avg_ms = dt.value / max(1, dcnt.value)
    m, n = step.m, step.n
    # algorithmic work per launch of the dominant class
    if dom == "chain_y":
        unit_flops = 2.0 * n * n * m
    elif dom == "gram":
        unit_flops = m * n * (n + 1.0)
    else:
        unit_flops = dfl.value / max(1, dcnt.value)
    achieved = unit_flops / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    roofline = {
        "kernel": dom,
        "bound": "mfma",
        "achieved": round(achieved, 3),
        "peak": FP64_MFMA_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
        "traffic": _counter_traffic(dom, tag),
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "algorithmic_flops_per_launch": unit_flops,
        "avg_launch_ms": round(avg_ms, 4),
        "launches_per_step": dcnt.value / steps,
    }
    rep = {"ms_per_step": round(ms_per_step, 4), "tflops": round(flops / (ms_per_step * 1e-3) / 1e12, 4),
           "rank": r, "flops_per_step": flops}
    breakdown = {name: round(v[0], 4) for name, v in per_class.items() if v[1] > 0}
    return rep, roofline, breakdown, pv


def bench_mixed_same_input(lib, api, torch, step, steps, variants):
    """The mixed-precision form beside the float64 one on the headline's
    device-resident G: time, rank, and the backward-stable figures of each
    (the float64 form's Y and W are the step's last outputs)."""
    m, n, k = step.m, step.n, step.k
    vp = ctypes.c_void_p
    dev = step.Gd.device
    sync = torch.cuda.synchronize
    t64 = None
    out = {"fp64": dict(_gpu_quality(torch, step.Gd, step.Y, step.Fd, step.W))}
    Ymx = api.empty_colmajor(n, m, dev)
    for variant in variants:
        key = variant[0]

        def f(rank=None, est=None):
            st = _mixed_call(lib, step.ctx, m, n, step.Gd, m, Ymx, variant, rank, est)
            if st != 0:
                raise RuntimeError(f"geninv_mixed failed: {st}")
        rm = ctypes.c_int(0)
        est = ctypes.c_double(0.0)
        f(ctypes.byref(rm), ctypes.byref(est))
        t = _timed(f, steps, sync)
        Wmx = Ymx @ step.Fd
        rep = {"ms": round(t, 3), "rank": rm.value, "speedup_vs_fp64": None, "err_est": est.value,
               "relF_Y_vs_fp64_gpu": float(torch.linalg.norm(Ymx - step.Y) / torch.linalg.norm(step.Y)),
               "relF_W_vs_fp64_gpu": float(torch.linalg.norm(Wmx - step.W) / torch.linalg.norm(step.W))}
        rep.update(_gpu_quality(torch, step.Gd, Ymx, step.Fd, Wmx))
        out[key] = rep
        del Wmx
    del Ymx
    return out


def cpu_oracle_leg(workloads, np, headline_key, flops_fn, c2_host, mixed_host, batched_host, forms):
    """Everything that runs the CPU oracle: its timing on a row sample of the
    headline workload (cpu_baseline), and the reference results that the
    other forms' accuracy figures are stated against."""
    from oracle import geninv_ref as o
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        threads = int(os.environ.get("OPENBLAS_NUM_THREADS", "1"))
    G, F = _generate(workloads, headline_key)
    m, n = G.shape
    rows = min(m, 16384)
    Gs = np.ascontiguousarray(G[:rows])
    Fs = np.ascontiguousarray(F[:rows])
    del G, F
    times = []
    budget = 25.0
    while not times or (sum(times) + times[-1] < budget and len(times) < 3):
        c0 = time.perf_counter()
        W, res = o.lstsq(Gs, Fs)
        times.append(time.perf_counter() - c0)
    med = sorted(times)[len(times) // 2]
    acc = np.zeros(res.d.size, bool)
    acc[res.piv] = True
    r_before = np.concatenate([[0], np.cumsum(acc)[:-1]])
    flops = flops_fn(rows, n, r_before, res.rank, Fs.shape[1])
    cpu = {"value": round(flops / med / 1e12, 5), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"whole float64 oracle (Gram, tol, column-by-column full-rank Cholesky, (L'L)^-1, "
                     f"chain, W = Y F) on the first {rows} of the {m} rows of the same design (all {n} "
                     f"columns), median of {len(times)} run(s), {med:.2f} s each; rank {res.rank}; "
                     f"TFLOP/s by the same flop model as value",
           "seconds": round(med, 3)}
    del Gs, Fs, W, res

    def relf(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    if c2_host is not None:
        co = forms["fp64_rbf_8192x2048"]
        Gc, Fc = c2_host["G"], c2_host["F"]
        ref = o.geninv(Gc)
        acc = co["accuracy"]
        acc["oracle_rank"] = ref.rank
        acc["relF_Y_vs_oracle"] = relf(c2_host["Y"], ref.Y)
        acc["oracle_self_spread"] = o.self_spread(Gc, base=ref)
        Wref = ref.Y @ Fc
        acc["relF_W_vs_oracle"] = relf(c2_host["W"], Wref)
        acc["oracle_gyg_minus_g_relF"] = relf(Gc @ (ref.Y @ Gc), Gc)
        acc["oracle_ls_residual"] = float(np.linalg.norm(Gc @ Wref - Fc) / np.linalg.norm(Fc))
        acc["oracle_penrose_max_abs"] = max(o.penrose_errors(Gc, ref.Y).values())
        acc["penrose_max_abs"] = max(o.penrose_errors(Gc, c2_host["Y"]).values())
        same = np.array_equal(np.sort(ref.piv), np.sort(c2_host["piv"]))
        acc["pivots_equal_oracle"] = bool(same)
    if mixed_host is not None:
        mo = forms["mixed_vs_fp64"]
        Gm = mixed_host["G"]
        c0 = time.perf_counter()
        ref = o.geninv(Gm)
        mo["oracle_seconds"] = round(time.perf_counter() - c0, 2)
        mo["oracle_rank"] = ref.rank
        Ytrue = (mixed_host["Q"] / mixed_host["sv"]) @ mixed_host["P"].T
        # the oracle on the 32-bit column-sliced representation G_s that the
        # mixed Gram matrix is exact for: separates representation error
        # from arithmetic error
        from oracle import ozaki_ref as z
        Ssl, esl = z.slice_columns(Gm, 4)
        Gsl = z.reconstruct(Ssl, esl)
        del Ssl
        ref_s = o.geninv(Gsl).Y
        del Gsl
        mo["oracle_on_sliced_G_relF_vs_oracle"] = relf(ref_s, ref.Y)
        mo["oracle_relF_vs_closed_form"] = relf(ref.Y, Ytrue)
        for key, Y in mixed_host["Y"].items():
            mo[key]["relF_vs_oracle"] = relf(Y, ref.Y)
            mo[key]["relF_vs_closed_form"] = relf(Y, Ytrue)
            if key != "fp64":
                mo[key]["relF_vs_oracle_on_sliced_G"] = relf(Y, ref_s)
    if batched_host is not None:
        bo = forms["batched"]
        B = batched_host["B"]
        worst = 0.0
        for b, Wg in batched_host["sample"].items():
            Wr, _ = o.lstsq(B.G[b].astype(np.float64), B.F[b].astype(np.float64))
            worst = max(worst, relf(Wg, Wr))
        bo["sampled_16_max_relF_vs_oracle"] = worst
        # problems whose rank differs from the float64 form: the oracle's
        # rank from its own Gram and from an extended-precision Gram
        diffs = []
        for b in batched_host["differs"][:16]:
            Gb = B.G[b].astype(np.float64)
            diffs.append({"problem": b, "rank_batched": int(batched_host["rank_batched"][b]),
                          "rank_fp64": int(batched_host["rank_fp64"][b]), "rank_oracle": o.geninv(Gb).rank,
                          "rank_oracle_extended_gram": o.geninv(Gb, A=o.gram_extended(Gb)).rank})
        bo["rank_differs_from_fp64_form"] = diffs
        # same-rank problems where the batched and float64 forms disagree by
        # more than 1e-6: both forms against the oracle, its own rounding
        # spread, and the least-squares residuals
        outl = []
        for b, (Wg, W64) in batched_host["outliers"].items():
            Gb = B.G[b].astype(np.float64)
            Fb = B.F[b].astype(np.float64)
            ref = o.geninv(Gb)
            Wr = ref.Y @ Fb
            nf = float(np.linalg.norm(Fb))
            outl.append({"problem": b, "m": int(Gb.shape[0]), "n": int(Gb.shape[1]), "rank_oracle": ref.rank,
                         "relF_batched_vs_oracle": relf(Wg, Wr), "relF_fp64_form_vs_oracle": relf(W64, Wr),
                         "oracle_self_spread_Y": o.self_spread(Gb, base=ref),
                         "ls_residual": {"batched": float(np.linalg.norm(Gb @ Wg - Fb)) / nf,
                                         "fp64_form": float(np.linalg.norm(Gb @ W64 - Fb)) / nf,
                                         "oracle": float(np.linalg.norm(Gb @ Wr - Fb)) / nf}})
        bo["same_rank_outliers_vs_oracle"] = outl
    return cpu


def bench_c2_form(lib, api, workloads, torch, np, steps, keep_host):
    """The float64 form on the 8192 x 2048 RBF design: time, rank, and the
    figures its accuracy is stated with (host copies for the oracle leg)."""
    G, F = _generate(workloads, "c2")
    dev = torch.device("cuda", 0)
    step = Fp64Step(lib, api, torch, np, G, F, dev)
    rep, roof, breakdown, pv = measure_fp64(lib, step, steps, 2, torch, WORKLOADS["c2"][0])
    rep["workload"] = WORKLOADS["c2"][1]
    rep["dominant_kernel"] = {k: roof[k] for k in ("kernel", "achieved", "frac", "avg_launch_ms")}
    rep["kernel_ms_one_step"] = breakdown
    rep["accuracy"] = _gpu_quality(torch, step.Gd, step.Y, step.Fd, step.W)
    host = None
    if keep_host:
        host = {"G": G, "F": F, "Y": step.Y.cpu().numpy(), "W": step.W.cpu().numpy(), "piv": pv}
    step.free()
    torch.cuda.empty_cache()
    return rep, host


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c5",
                    help="headline workload: c5 (131072 x 8192 RBF design, default) or c2 (8192 x 2048)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-forms", action="store_true", help="only the headline float64 workload")
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle checks of the other forms")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for hardware byte counters) and exit")
    ap.add_argument("--only-batched", action="store_true",
                    help="only run the 4096-problem batch `steps` times (direct launches, LDS threshold 48, 512 "
                         "workgroups) "
                         "and exit (for hardware counter runs)")
    ap.add_argument("--only-mixed", metavar="KEY",
                    help="only run one mixed-form variant (e.g. int8_m16) on the headline workload `steps` "
                         "times and exit (for hardware counter runs)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0804_4809_amd import api, workloads
    from paper_0804_4809_amd._lib import load

    lib = load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    tag, desc = WORKLOADS[args.workload]
    if args.only_batched:
        B = workloads.c4_problem()
        plan = api.BatchPlan(B.G, B.F)
        plan.config(48, 512)
        for _ in range(args.warmup):
            plan.run(use_graph=False)
        t = _timed(lambda: plan.run(use_graph=False), args.steps, torch.cuda.synchronize)
        print(json.dumps({"workload": "4096 batched problems (C4)", "config": plan.config(), "ms": round(t, 3),
                          "steps": args.steps}), flush=True)
        plan.close()
        return

    c0 = time.perf_counter()
    G, F = _generate(workloads, args.workload)
    gen_s = time.perf_counter() - c0
    step = Fp64Step(lib, api, torch, np, G, F, dev)
    m, n, k = step.m, step.n, step.k
    del G, F
    print(f"[bench] {tag} generated in {gen_s:.1f} s, uploaded", file=sys.stderr, flush=True)
    if args.only_mixed:
        variant = {v[0]: v for v in MIXED_C5 + MIXED_C3}[args.only_mixed]
        Ymx = api.empty_colmajor(n, m, dev)
        for _ in range(args.warmup):
            _mixed_call(lib, step.ctx, m, n, step.Gd, m, Ymx, variant)
        t = _timed(lambda: _mixed_call(lib, step.ctx, m, n, step.Gd, m, Ymx, variant), args.steps,
                   torch.cuda.synchronize)
        print(json.dumps({"workload": desc, "variant": variant, "ms": round(t, 3), "steps": args.steps}), flush=True)
        return
    rep, roofline, breakdown, _ = measure_fp64(lib, step, args.steps, args.warmup, torch, tag)
    print(f"[bench] {tag} float64: {rep['ms_per_step']} ms/step", file=sys.stderr, flush=True)

    oracle_on = not args.no_cpu_baseline and not args.no_oracle
    forms = {}
    mixed_host = batched_host = c2_host = None
    if not args.skip_forms:
        fsteps = max(2, min(args.steps, 3)) if args.workload == "c5" else max(2, min(args.steps, 5))
        mo = bench_mixed_same_input(lib, api, torch, step, fsteps, MIXED_C5 if args.workload == "c5" else MIXED_C3)
        mo["fp64"]["ms"] = rep["ms_per_step"]
        for key, v in mo.items():
            if isinstance(v, dict) and v.get("speedup_vs_fp64", 0) is None:
                v["speedup_vs_fp64"] = round(rep["ms_per_step"] / v["ms"], 3)
        forms["mixed_vs_fp64_same_input"] = mo
        forms["mixed_vs_fp64_same_input"]["workload"] = desc.replace("float64 geninv + W = G^+ F on ", "")
    headline_quality = _gpu_quality(torch, step.Gd, step.Y, step.Fd, step.W)
    step.free()
    del step
    torch.cuda.empty_cache()
    if not args.skip_forms:
        print("[bench] forms", file=sys.stderr, flush=True)
        def note(what):
            print(f"[bench] form {what}", file=sys.stderr, flush=True)

        if args.workload != "c2":
            note("fp64_rbf_8192x2048")
            forms["fp64_rbf_8192x2048"], c2_host = bench_c2_form(lib, api, workloads, torch, np, 20, oracle_on)
        fsteps = max(2, min(args.steps, 5))
        note("mixed_vs_fp64")
        forms["mixed_vs_fp64"], mixed_host = bench_mixed(lib, api, workloads, torch, np, fsteps, oracle_on)
        note("batched")
        forms["batched"], batched_host = bench_batched(api, workloads, torch, np, max(3, min(args.steps, 10)),
                                                       oracle_on)
        note("table1_sweep")
        forms["table1_sweep"] = bench_table1(lib, api, workloads, torch, np, 5)
        note("incremental_lstsq")
        forms["incremental_lstsq"] = bench_incremental(lib, api, workloads, torch, np, 3)
        note("spd_inverse")
        forms["spd_inverse_gj_vs_newton_schulz"] = bench_spd_inverse(lib, api, workloads, torch, np, 3)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] oracle leg", file=sys.stderr, flush=True)
        cpu = cpu_oracle_leg(workloads, np, args.workload, algorithmic_flops, c2_host if oracle_on else None,
                             mixed_host if oracle_on else None, batched_host if oracle_on else None, forms)
    del mixed_host, batched_host, c2_host

    out = {
        "metric": METRIC,
        "value": rep["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rep["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "m": m, "n": n, "k": k, "rank": rep["rank"], "flops_per_step": rep["flops_per_step"],
            "generate_s": round(gen_s, 1),
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": headline_quality,
        "kernel_ms_one_step": breakdown,
        "forms": forms,
    }
    print(json.dumps(_finite(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
