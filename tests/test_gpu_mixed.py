"""GPU parity of the mixed-precision form (sliced bfloat16 products).

* slicing is integer work: planes and exponents must be bit-identical to
  the oracle's;
* the sliced Gram matrix must equal the exactly rounded Gram matrix of the
  sliced representation up to the float64 rounding of the pair/chunk totals
  (bit-exact when every partial sum is exact);
* the whole mixed method must give the oracle's rank and Y within 1e-6
  relative Frobenius (the accuracy target of the mixed form).
"""
import numpy as np
import pytest

from oracle import geninv_ref as o
from oracle import ozaki_ref as z
from paper_0804_4809_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_0804_4809_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)
MIXED_TOL = 1e-6


def up(X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(DEV)


def down(T):
    torch.cuda.synchronize()
    return T.detach().cpu().numpy()


def _case(label, **kw):
    print(f"[case] {label} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("rows,cols,s", [(100, 7, 4), (257, 33, 3), (64, 64, 6), (1, 5, 2), (1000, 130, 4)])
def test_slice_columns_bit_exact(rows, cols, s):
    _case("bslice cols", rows=rows, cols=cols, s=s)
    rng = np.random.default_rng(rows + cols)
    X = rng.standard_normal((rows, cols)) * 10.0 ** rng.uniform(-5, 5, size=cols)
    X[:, 0] = 0.0
    S, e = z.slice_columns(X, s)
    planes, eg = api.bslice(up(X), s)
    eg = down(eg).astype(np.int64)
    assert np.array_equal(eg, e)
    P = down(planes.float()).astype(np.float64)          # (s, cols, ldp)
    assert np.array_equal(P[:, :, :rows], np.transpose(S, (0, 2, 1)).astype(np.float64))
    assert not P[:, :, rows:].any()


@pytest.mark.parametrize("rows,cols,s", [(100, 7, 4), (33, 257, 3), (64, 64, 5)])
def test_slice_rows_transposed_bit_exact(rows, cols, s):
    _case("bslice rows", rows=rows, cols=cols, s=s)
    rng = np.random.default_rng(rows * cols)
    X = rng.standard_normal((rows, cols)) * 10.0 ** rng.uniform(-4, 4, size=(rows, 1))
    S, e = z.slice_columns(X.T.copy(), s)               # row slicing = column slicing of X'
    planes, eg = api.bslice(up(X), s, transposed=True)
    assert np.array_equal(down(eg).astype(np.int64), e)
    P = down(planes.float()).astype(np.float64)          # (s, rows, ldp): planes[t][i][k]
    assert np.array_equal(P[:, :, :cols], np.transpose(S, (0, 2, 1)).astype(np.float64))
    assert not P[:, :, cols:].any()


def test_sliced_gram_integer_input_bit_exact():
    _case("bgram exact integers")
    rng = np.random.default_rng(9)
    G = rng.integers(-100, 101, size=(777, 70)).astype(np.float64)
    A = down(api.bgram(up(G), 4))
    ref = G.T @ G          # exact: integer sums below 2^53
    assert np.array_equal(np.tril(A), np.tril(ref))


@pytest.mark.parametrize("m,n,s", [(300, 40, 4), (513, 129, 3), (2000, 200, 4), (12000, 150, 4), (64, 200, 2),
                                   (100, 7, 1)])
def test_sliced_gram_matches_exact_representation_gram(m, n, s):
    """The GPU sliced Gram is the exact Gram matrix of the sliced representation
    up to the float64 rounding of its class totals (12000 x 150 goes through
    the split-K path)."""
    _case("bgram", m=m, n=n, s=s)
    G, _ = w.lowrank_uv(m, n, max(1, n // 2), seed=m)
    S, e = z.slice_columns(G, s)
    Gs = z.reconstruct(S, e)
    A = np.tril(down(api.bgram(up(G), s)))
    ref = np.tril(z.sliced_gram(G, s))
    # float64 totals: 2s - 1 weight classes per 32-deep stage, plus the
    # split-K sum and one final scaling
    nterms = (2 * s - 1) * ((m + 31) // 32) + 18
    bound = nterms * 2.0 ** -53 * np.tril(np.abs(Gs).T @ np.abs(Gs))
    assert np.all(np.abs(A - ref) <= bound + 1e-300)


@pytest.mark.parametrize("n,m,k,s", [(40, 300, 100, 4), (129, 513, 257, 3), (150, 2000, 600, 4), (7, 100, 33, 1),
                                     (64, 70, 200, 2), (33, 65, 1, 4)])
def test_sliced_chain_matches_exact_truncated_product(n, m, k, s):
    """The GPU chain product Y = P G' is the exact sum of the slice pairs
    t + u <= s of the row-sliced operands, up to the float64 rounding of its
    class totals."""
    _case("bchain", n=n, m=m, k=k, s=s)
    rng = np.random.default_rng(n * 1000 + k)
    P = rng.standard_normal((n, k)) * np.exp(rng.uniform(-3, 3, (n, 1)))
    G = rng.standard_normal((m, k))
    Y = down(api.bchain(up(P), up(G), s))
    SA, ea = z.slice_columns(P.T.copy(), s)
    SB, eb = z.slice_columns(G.T.copy(), s)
    ref = z.sliced_product_exact(SA, ea, SB, eb, max_class=min(s, 2 * s - 2))
    nterms = (s + 1) * ((k + 31) // 32) + 18
    bound = nterms * 2.0 ** -53 * (np.abs(z.reconstruct(SA, ea)).T @ np.abs(z.reconstruct(SB, eb)))
    assert np.all(np.abs(Y - ref) <= bound + 1e-300)


def test_sliced_chain_empty_inner_dimension_is_zero():
    Y = down(api.bchain(up(np.zeros((5, 0))), up(np.zeros((9, 0))), 4))
    assert Y.shape == (5, 9) and not Y.any()


def test_sliced_gram_rejects_five_slices():
    with pytest.raises(api.GeninvError) as e:
        api.bgram(up(np.ones((10, 3))), 5)
    assert e.value.status == -1


def test_mixed_c1_matches_oracle():
    _case("mixed", cfg="c1")
    G, F = w.c1_problem(0)
    ref = o.geninv(G)
    res = api.mixed(up(G), engine="bf16", gram_digits=4, chain_digits=4, return_result=True)
    Y, r, piv = res.Y, res.rank, res.piv
    assert r == ref.rank
    assert np.array_equal(down(piv).astype(np.int64), ref.piv)
    assert o.rel_fro(down(Y), ref.Y) <= MIXED_TOL


@pytest.mark.parametrize("chain_slices,ns", [(4, 0), (0, 0), (4, 1)])
def test_mixed_svd_family(chain_slices, ns):
    """G = P diag(s) Q', 8192 x 1024, rank 768, s in [1e-3, 1]: the mixed-form
    workload at reduced size."""
    _case("mixed", cfg="svd 8192x1024 r768", chain_slices=chain_slices, ns=ns)
    G, _, P, sv, Q = w.svd_family(8192, 1024, 768, 1e-3, seed=2)
    ref = o.geninv(G)
    res = api.mixed(up(G), engine="bf16", gram_digits=4, chain_digits=chain_slices, ns_steps=ns, return_result=True)
    Y, r, piv = res.Y, res.rank, res.piv
    Yg = down(Y)
    err = o.rel_fro(Yg, ref.Y)
    print(f"  rank gpu {r} oracle {ref.rank}; relF(Y) vs oracle {err:.3e}; "
          f"vs closed form {o.rel_fro(Yg, (Q / sv) @ P.T):.3e}", flush=True)
    assert r == ref.rank == 768
    assert np.array_equal(down(piv).astype(np.int64), ref.piv)
    assert err <= MIXED_TOL


@pytest.mark.parametrize("kind,m,n,r,slices,chain_slices,ns", [
    ("uv", 3001, 517, 300, 4, 4, 0),     # ragged against the 128 x 64 tiles and the 64-deep K padding
    ("uv", 2000, 2000, 1500, 4, 4, 0),   # square
    ("svd", 5000, 300, 300, 4, 3, 0),    # full column rank, cond 2, 3-slice chain (pairs t + u <= 3)
    ("uv", 4000, 256, 200, 4, 4, 2),     # two Newton-Schulz steps
])
def test_mixed_more_shapes(kind, m, n, r, slices, chain_slices, ns):
    """G = U V (N(0,1) factors) of exact rank r, or P diag(s) Q' with s in
    [0.5, 1]: the mixed form's decisions equal the oracle's and Y is within
    the mixed tolerance."""
    _case("mixed", kind=kind, m=m, n=n, r=r, slices=slices, chain_slices=chain_slices, ns=ns)
    if kind == "uv":
        G, _ = w.lowrank_uv(m, n, r, seed=m + n)
    else:
        G = w.svd_family(m, n, r, 0.5, seed=m + n)[0]
    ref = o.geninv(G)
    res = api.mixed(up(G), engine="bf16", gram_digits=slices, chain_digits=chain_slices, ns_steps=ns,
                    return_result=True)
    Y, rg, piv = res.Y, res.rank, res.piv
    err = o.rel_fro(down(Y), ref.Y)
    # 4 chain slices: the 1e-6 target.  3 chain slices represent P and G with
    # 24 bits: an entry of Y = P G' (n terms of random sign) then carries
    # about sqrt(n) 2^-23 relative error, which the target does not cover
    tol = MIXED_TOL if chain_slices == 4 else 4 * np.sqrt(n) * 2.0 ** -23
    print(f"  rank gpu {rg} oracle {ref.rank}; relF(Y) {err:.3e} (bound {tol:.1e})", flush=True)
    assert rg == ref.rank == r
    assert np.array_equal(down(piv).astype(np.int64), ref.piv)
    assert err <= tol


def test_mixed_transpose_branch():
    """m < n: the Appendix's transpose branch, G G' factored and Y = G' P."""
    _case("mixed", cfg="wide 300 x 900, rank 200", engine="bf16")
    G, _ = w.lowrank_uv(300, 900, 200, seed=77)
    ref = o.geninv(G)
    res = api.mixed(up(G), engine="bf16", gram_digits=4, chain_digits=4, return_result=True)
    assert res.rank == ref.rank == 200
    assert np.array_equal(down(res.piv).astype(np.int64), ref.piv)
    assert o.rel_fro(down(res.Y), ref.Y) <= MIXED_TOL


def test_mixed_rejects_bad_digits():
    G = up(np.ones((5, 3)))
    for kw in (dict(engine="bf16", gram_digits=5), dict(engine="bf16", gram_digits=0),
               dict(engine="int8", gram_digits=17), dict(engine="int8", chain_digits=-1)):
        with pytest.raises(api.GeninvError) as e:
            api.mixed(G, **kw)
        assert e.value.status == -1
