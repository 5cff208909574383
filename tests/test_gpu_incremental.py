"""GPU parity of the incremental least-squares form (Section 4's incremental
learning): Gram rows appended per batch of new columns, the full-rank
Cholesky factor and (L'L)^-1 extended (geninv_inc_factor) or the method
rerun from the Gram matrix, against the oracle on the whole matrix seen so
far: identical decisions (pivot columns), W within the float64 bound.
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
U = 2.0 ** -53


def up(X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(DEV)


def down(T):
    return T.detach().cpu().numpy()


def _case(**kw):
    print("[case] " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("m,steps,k", [(3000, [200, 250, 250], 3), (777, [1, 63, 64, 1, 130], 2), (2000, [700], 1)])
def test_appended_gram_rows_equal_the_gram_matrix(m, steps, k):
    """After every append, the lower triangle of A is G'G and B is G'F for the
    columns so far, within the rounding of an m-term float64 sum."""
    _case(test="inc_gram", m=m, steps=steps, k=k)
    n = sum(steps)
    rng = np.random.default_rng(m + n)
    G = rng.standard_normal((m, n))
    F = rng.standard_normal((m, k))
    inc = api.IncrementalLstsq(n, k)
    n_t = 0
    for p in steps:
        n_t += p
        inc.append(up(G[:, :n_t]), up(F))
        A = down(inc.A)[:n_t, :n_t]
        B = down(inc.B)[:n_t, :k]
        Gt = G[:, :n_t]
        bound_a = 2 * m * U * (np.abs(Gt).T @ np.abs(Gt))
        bound_b = 2 * m * U * (np.abs(Gt).T @ np.abs(F))
        assert np.all(np.tril(np.abs(A - Gt.T @ Gt) - bound_a) <= 0)
        assert np.all(np.abs(B - Gt.T @ F) <= bound_b)


@pytest.mark.parametrize("refactor", [False, True])
@pytest.mark.parametrize("m,n,r,k,steps", [(2000, 300, 200, 4, [100, 120, 80]), (1500, 129, 129, 2, [64, 65]),
                                           (900, 200, 60, 3, [50, 50, 50, 50]), (3000, 700, 500, 2, [300, 1, 399]),
                                           # 128 appended columns all combinations of the 896 before them: the
                                           # new rows of L dominate L'L (the direct inverse, not Woodbury)
                                           (20000, 1024, 896, 2, [896, 128])])
def test_incremental_lstsq_matches_oracle_after_every_append(m, n, r, k, steps, refactor):
    """W from the appended Gram rows equals the oracle's W = G^+ F on the
    columns seen so far (same pivot columns, relF within the float64 bound)."""
    _case(test="inc_lstsq", m=m, n=n, r=r, k=k, steps=steps, refactor=refactor)
    G, F = w.lowrank_uv(m, n, r, seed=m + r, k=k)
    inc = api.IncrementalLstsq(n, k, refactor=refactor)
    n_t = 0
    for p in steps:
        n_t += p
        inc.append(up(G[:, :n_t]), up(F))
        W, rank = inc.solve()
        Wr, ref = o.lstsq(G[:, :n_t], F)
        assert rank == ref.rank
        if not refactor:
            assert np.array_equal(down(inc.pivots()).astype(np.int64), ref.piv)
        bound = max(FP64_TOL, 10 * o.self_spread(G[:, :n_t], base=ref))
        assert o.rel_fro(down(W), Wr) <= bound


def test_incremental_rbf_design_appends():
    """The RBF design of the benchmark (8192 x 2048, sigma 0.3, 256 duplicate
    centers), 1536 centers then 4 x 128: decisions equal the oracle's (or a
    rounding-band replay) and W within 10x the oracle's own spread."""
    from parity_rules import decisions_or_replay
    _case(test="inc_rbf")
    G, F, _ = w.c2_problem()
    inc = api.IncrementalLstsq(2048, F.shape[1])
    for n_t in (1536, 1664, 1792, 1920, 2048):
        inc.append(up(G[:, :n_t]), up(F))
        W, rank = inc.solve()
        ref0 = o.geninv(G[:, :n_t])
        ref, amb = decisions_or_replay(G[:, :n_t], ref0, down(inc.pivots()).astype(np.int64))
        forced = np.isin(np.arange(n_t), down(inc.pivots())) if amb else None
        err = o.rel_fro(down(W), ref.Y @ F)
        bound = max(FP64_TOL, 10 * o.self_spread(G[:, :n_t], base=ref, forced=forced))
        print(f"  {n_t} columns: rank {rank} (oracle {ref0.rank}), relF(W) {err:.3e}, bound {bound:.3e}", flush=True)
        assert err <= bound


def test_incremental_threshold_falls_and_refactors():
    """A new column with a much smaller diagonal lowers the paper's default
    threshold below an earlier dropped pivot: that column is now kept, as in
    the oracle on the whole matrix (the call refactors)."""
    _case(test="inc_tol_falls")
    rng = np.random.default_rng(31)
    m = 400
    a = rng.standard_normal(m)
    c = rng.standard_normal(m)
    base = rng.standard_normal((m, 20))
    G = np.column_stack([a, base, a + 1e-5 * c, 1e-3 * rng.standard_normal(m)])
    F = rng.standard_normal((m, 2))
    inc = api.IncrementalLstsq(G.shape[1], 2)
    inc.append(up(G[:, :22]), up(F))
    _, r1 = inc.solve()
    assert r1 == o.geninv(G[:, :22]).rank == 21        # a + 1e-5 c dropped at the first threshold
    inc.append(up(G), up(F))
    W, r2 = inc.solve()
    ref = o.geninv(G)
    assert r2 == ref.rank == 23                          # kept once the threshold falls
    assert np.array_equal(down(inc.pivots()).astype(np.int64), ref.piv)
    assert o.rel_fro(down(W), ref.Y @ F) <= max(FP64_TOL, 10 * o.self_spread(G, base=ref))


def test_incremental_equals_one_shot_lstsq():
    """The incremental path and geninv_dlstsq on the whole matrix agree (same
    decisions; the Gram sums are grouped differently, so within rounding)."""
    _case(test="inc_vs_one_shot")
    G, F = w.lowrank_uv(4000, 512, 400, seed=7, k=8)
    inc = api.IncrementalLstsq(512, 8)
    for n_t in (128, 256, 512):
        inc.append(up(G[:, :n_t]), up(F))
    W_inc, r_inc = inc.solve()
    W_one, r_one = api.lstsq(up(G), up(F))
    assert r_inc == r_one == 400
    assert o.rel_fro(down(W_inc), down(W_one)) <= 1e-10


def test_zero_new_columns_is_a_no_op_and_empty_solve():
    inc = api.IncrementalLstsq(10, 2)
    W, r = inc.solve()
    assert r == 0 and W.shape == (0, 2)
    G = np.arange(20.0).reshape(10, 2)
    inc.append(up(G[:, :0]), up(np.ones((10, 2))))
    assert inc.n == 0
