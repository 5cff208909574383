"""GPU parity of libgeninv (float64 form) against the CPU oracle.

Every case feeds identical seeded inputs to both sides.  Integer results
(rank, pivot columns) must match exactly; floating-point results within the
float64 tolerance 1e-10 relative Frobenius, except where the input itself
is so ill-conditioned that two correct float64 evaluations differ by more:
then the bound is 10x the oracle's own self-spread (the oracle with the Gram
summed in a different order), and backward-stable quantities (Penrose
residual, least-squares residual) are checked as well.
"""
import numpy as np
import pytest

from oracle import geninv_ref as o
from paper_0804_4809_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_0804_4809_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)
FP64_TOL = 1e-10


def up(X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(DEV)


def down(T):
    torch.cuda.synchronize()
    return T.detach().cpu().numpy().astype(np.float64)


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


# ---------------------------------------------------------------------------
# GEMM, the contraction every step uses
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("M,N,K,tA,tB", [
    (64, 64, 64, 0, 0), (200, 130, 77, 0, 0), (130, 200, 77, 1, 0), (77, 61, 300, 0, 1),
    (300, 50, 1000, 1, 1), (1, 1, 1, 0, 0), (5, 7, 0, 0, 0), (3000, 2900, 300, 0, 1),
])
def test_dgemm_parity(M, N, K, tA, tB):
    _print_case("dgemm", M=M, N=N, K=K, tA=tA, tB=tB)
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((K, M) if tA else (M, K))
    B = rng.standard_normal((N, K) if tB else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = 0.5 * ((A.T if tA else A) @ (B.T if tB else B)) - 2.0 * C0
    Cg = api.empty_colmajor(M, N, DEV)
    Cg.copy_(up(C0))
    out = down(api.dgemm(up(A), up(B), bool(tA), bool(tB), alpha=0.5, beta=-2.0, C=Cg))
    bound = 2 * max(K, 1) * 2.2e-16 * (0.5 * (np.abs(A.T if tA else A) @ np.abs(B.T if tB else B)) + 2 * np.abs(C0))
    assert np.all(np.abs(out - ref) <= bound + 1e-300)


# ---------------------------------------------------------------------------
# individual steps on identical inputs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n", [(200, 50), (1000, 300), (513, 129), (4096, 1000)])
def test_gram_parity(m, n):
    _print_case("gram", m=m, n=n)
    G = np.random.default_rng(m + n).standard_normal((m, n))
    ref = o.gram(G)
    A = down(api.gram(up(G), full=True))
    assert o.rel_fro(A, ref) <= 1e-14 * np.sqrt(m)
    Al = down(api.gram(up(G), full=False))
    assert np.array_equal(np.tril(Al), np.tril(A))


def _frchol_case(G):
    A = o.gram(G)
    tol = o.paper_tol(A)
    Lr, r, piv, d = o.full_rank_cholesky(A, tol)
    res = api.frchol(up(A))
    return A, tol, Lr, r, piv, d, res


@pytest.mark.parametrize("name", ["c1", "ragged_lowrank", "table1_256", "rbf_small", "zero_cols"])
def test_frchol_parity_same_gram(name):
    _print_case("frchol", name=name)
    if name == "c1":
        G, _ = w.c1_problem(0)
    elif name == "ragged_lowrank":
        G, _ = w.lowrank_uv(700, 333, 201, seed=21)
    elif name == "table1_256":
        G = w.table1(256, seed=3)
    elif name == "rbf_small":
        G, _, _ = w.rbf_design(2000, 3, 300, 60, 0.35, seed=8)
    else:
        G, _ = w.lowrank_uv(300, 150, 90, seed=5)
        G[:, [0, 7, 64, 65, 149]] = 0.0
    A, tol, Lr, r, piv, d, res = _frchol_case(G)
    assert res.rank == r
    assert np.array_equal(down(res.piv).astype(np.int64), piv)
    assert res.tol == pytest.approx(tol, rel=1e-15)
    Lg = down(res.L)
    assert o.rel_fro(Lg, Lr) <= 1e-9 if name == "rbf_small" else o.rel_fro(Lg, Lr) <= 1e-11
    # exactly zero above each pivot
    for c in range(r):
        assert not Lg[: piv[c], c].any()
    acc = np.zeros(len(d), bool)
    acc[piv] = True
    dg = down(res.d)
    assert np.allclose(dg[acc], d[acc], rtol=1e-6, atol=0)


def test_spdinv_parity():
    _print_case("spdinv")
    rng = np.random.default_rng(4)
    for r in (1, 17, 64, 65, 200, 333):
        X = rng.standard_normal((r + 5, r))
        B = X.T @ X
        ref = o.spd_inverse(B)
        M = down(api.spd_inverse(up(B)))
        assert np.array_equal(M, M.T)
        cond = np.linalg.cond(B)
        assert o.rel_fro(M, ref) <= 50 * cond * 2.2e-16 * r, r


def test_chain_parity_same_factors():
    _print_case("chain")
    G, _ = w.lowrank_uv(900, 260, 170, seed=31)
    res = o.geninv(G)
    Y = down(api.chain(up(res.L), up(res.M), up(G)))
    assert o.rel_fro(Y, res.Y) <= 1e-11


# ---------------------------------------------------------------------------
# whole method
# ---------------------------------------------------------------------------
def _compare(G, tol=None, check_penrose=None):
    ref = o.geninv(G, tol)
    Y, r, piv = api.geninv(up(G), tol, return_piv=True)
    Yg = down(Y)
    assert r == ref.rank
    assert np.array_equal(down(piv).astype(np.int64), ref.piv)
    err = o.rel_fro(Yg, ref.Y)
    if check_penrose is not None:
        assert max(o.penrose_errors(G, Yg).values()) <= check_penrose
    return err, ref, Yg


def test_geninv_c1():
    _print_case("geninv", cfg="c1 200x50 rank 40")
    G, F = w.c1_problem(0)
    err, ref, Yg = _compare(G)
    assert err <= FP64_TOL
    assert o.rel_fro(Yg, np.linalg.pinv(G, rcond=1e-10)) <= FP64_TOL


@pytest.mark.parametrize("m,n,r,seed", [(1000, 300, 200, 1), (777, 129, 129, 2), (65, 64, 63, 3),
                                        (130, 1, 1, 4), (1, 1, 1, 5), (300, 700, 120, 6), (64, 200, 64, 7)])
def test_geninv_lowrank_ragged(m, n, r, seed):
    _print_case("geninv", m=m, n=n, r=r, seed=seed)
    G, _ = w.lowrank_uv(m, n, r, seed)
    err, ref, Yg = _compare(G)
    assert err <= FP64_TOL


@pytest.mark.parametrize("n", [64, 256, 512])
def test_geninv_table1_family_penrose(n):
    _print_case("geninv", cfg=f"table1 n={n}")
    G = w.table1(n, seed=n + 1)
    err, ref, Yg = _compare(G, check_penrose=2e-10)
    assert ref.rank == 7 * n // 8
    assert err <= FP64_TOL


def test_geninv_user_tol_and_strictness():
    _print_case("geninv", cfg="strict tol")
    G = np.diag([3.0, 2.0, 5.0])
    Y, r = api.geninv(up(G), tol=4.0)     # A = diag(9, 4, 25): the pivot equal to tol is dropped
    assert r == 2
    assert np.allclose(down(Y), np.diag([1 / 3, 0.0, 0.2]), rtol=1e-15, atol=0)


def test_geninv_zero_and_empty():
    _print_case("geninv", cfg="zero/empty")
    for shape in [(50, 20), (20, 50)]:
        Y, r = api.geninv(up(np.zeros(shape)))
        assert r == 0 and not down(Y).any()
    Y, r = api.geninv(torch.zeros((0, 5), dtype=torch.float64, device=DEV))
    assert r == 0 and Y.shape == (5, 0)


def test_geninv_nonfinite_reports_error():
    _print_case("geninv", cfg="nan")
    G = np.ones((40, 10))
    G[3, 4] = np.nan
    with pytest.raises(api.GeninvError) as e:
        api.geninv(up(G))
    assert e.value.status == -4
    # the context is usable afterwards
    G2, _ = w.c1_problem(0)
    err, _, _ = _compare(G2)
    assert err <= FP64_TOL


def test_geninv_duplicate_columns_rejected():
    _print_case("geninv", cfg="rbf duplicates")
    G, _, idx = w.rbf_design(3000, 4, 400, 100, 0.3, seed=12)
    ref = o.geninv(G)
    Y, r, piv = api.geninv(up(G), return_piv=True)
    assert r == ref.rank
    seen, dups = set(), []
    for j, c in enumerate(idx):
        if c in seen:
            dups.append(j)
        seen.add(c)
    assert not set(dups) & set(down(piv).astype(int).tolist())


def test_lstsq_c1():
    _print_case("lstsq", cfg="c1")
    G, F = w.c1_problem(0)
    Wr, ref = o.lstsq(G, F)
    W, r = api.lstsq(up(G), up(F))
    assert r == 40
    assert o.rel_fro(down(W), Wr) <= FP64_TOL


@pytest.mark.parametrize("m,n,k,r", [(3000, 257, 5, 180), (700, 64, 1, 64), (9000, 130, 16, 100)])
def test_lstsq_ragged(m, n, k, r):
    _print_case("lstsq", m=m, n=n, k=k, r=r)
    G, F = w.lowrank_uv(m, n, r, seed=m + k, k=k)
    Wr, ref = o.lstsq(G, F)
    W, rg = api.lstsq(up(G), up(F))
    assert rg == ref.rank
    assert o.rel_fro(down(W), Wr) <= FP64_TOL


def test_geninv_c2_full_size():
    """RBF design 8192 x 2048 (256 duplicate centers) at the benchmark's size."""
    _print_case("geninv", cfg="c2 rbf 8192x2048")
    G, F, idx = w.c2_problem()
    ref = o.geninv(G)
    spread = o.self_spread(G, base=ref)
    margins = o.decision_margins(ref)
    Y, r, piv = api.geninv(up(G), return_piv=True)
    Yg = down(Y)
    print(f"  oracle r={ref.rank} gpu r={r} margins={margins} self_spread={spread:.3e}", flush=True)
    assert r == ref.rank
    assert np.array_equal(down(piv).astype(np.int64), ref.piv)
    err = o.rel_fro(Yg, ref.Y)
    print(f"  relF(Y)={err:.3e} bound={max(FP64_TOL, 10 * spread):.3e}", flush=True)
    assert err <= max(FP64_TOL, 10 * spread)
    # backward-stable checks: G Y G = G and least-squares residuals agree
    GYG = G @ (Yg @ G)
    ref_res = o.rel_fro(G @ (ref.Y @ G), G)
    assert o.rel_fro(GYG, G) <= max(1e-6, 10 * ref_res)
    Wg, _ = api.lstsq(up(G), up(F))
    Wg = down(Wg)
    Wr = ref.Y @ F
    rg = np.linalg.norm(G @ Wg - F)
    rr = np.linalg.norm(G @ Wr - F)
    assert abs(rg - rr) <= 1e-8 * rr
