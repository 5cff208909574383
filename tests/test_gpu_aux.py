"""Failure handling and debug aids, forced from the host (every kernel exits
normally):

* the workspace cap: a call that needs more returns ENOMEM before anything
  is enqueued, and the context keeps working once the cap is lifted;
* NaN poisoning of the workspace between two calls: the second call's
  results are bit-identical to the first's, so no step reads memory that an
  earlier call (rather than an earlier step of the same call) wrote;
* a batched plan asked for its graph on a stream that the caller is already
  capturing launches directly into the caller's graph and counts the
  fallback; every replay of the caller's graph matches the eager run;
* a least-squares call captured on the caller's stream replays the eager
  result.
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


def up(X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(DEV)


def down(T):
    torch.cuda.synchronize()
    return T.detach().cpu().numpy().astype(np.float64)


def _case(label, **kw):
    print(f"[case] {label} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def test_workspace_cap_gives_enomem_and_the_context_recovers():
    _case("workspace cap")
    G, F = w.lowrank_uv(1000, 300, 200, 1, k=3)
    Gd, Fd = up(G), up(F)
    try:
        api.set_workspace_limit(1 << 20, DEV)
        with pytest.raises(api.GeninvError) as e:
            api.geninv(Gd)
        assert e.value.status == -2
        with pytest.raises(api.GeninvError) as e:
            api.lstsq(Gd, Fd)
        assert e.value.status == -2
    finally:
        api.set_workspace_limit(0, DEV)
    Y, r = api.geninv(Gd)
    ref = o.geninv(G)
    assert r == ref.rank == 200
    assert o.rel_fro(down(Y), ref.Y) <= 1e-10


def test_debug_flags_are_checked():
    with pytest.raises(api.GeninvError) as e:
        api.set_debug(6, DEV)
    assert e.value.status == -1
    api.set_debug(1, DEV)
    api.set_debug(0, DEV)


@pytest.mark.parametrize("form", ["geninv", "geninv_wide", "lstsq", "lstsq_wide", "mixed_int8"])
def test_results_do_not_depend_on_stale_workspace(form):
    _case("poisoned workspace", form=form)
    wide = form.endswith("_wide")
    m, n, r = (300, 1100, 150) if wide else (3000, 700, 500)
    G, F = w.lowrank_uv(m, n, r, seed=17, k=4)
    Gd, Fd = up(G), up(F)

    def run():
        if form.startswith("geninv"):
            Y, _ = api.geninv(Gd)
            return down(Y)
        if form.startswith("lstsq"):
            W, _ = api.lstsq(Gd, Fd)
            return down(W)
        Y, _ = api.mixed(Gd, engine="int8", gram_digits=16, chain_digits=16)
        return down(Y)

    first = run()
    api.debug_poison(DEV)
    second = run()
    assert np.isfinite(second).all()
    assert np.array_equal(first, second)


def test_batched_run_inside_a_caller_capture_falls_back_to_direct_launches():
    _case("batched graph fallback")
    rng = np.random.default_rng(5)
    Gs, Fs = [], []
    for _ in range(24):
        m = int(rng.integers(64, 400))
        n = int(rng.integers(8, min(120, m // 2) + 1))
        r = int(rng.integers(n // 2, n + 1))
        Gs.append((rng.standard_normal((m, r)) @ rng.standard_normal((r, n))).astype(np.float32))
        Fs.append(rng.standard_normal((m, 4)).astype(np.float32))
    plan = api.BatchPlan(Gs, Fs)
    plan.run(use_graph=False)
    torch.cuda.synchronize()
    ref = [plan.W(b).clone() for b in range(len(Gs))]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(use_graph=True)
    assert plan.graph_fallbacks() == 1
    for rep in range(3):
        for b in range(len(Gs)):
            plan.W(b).fill_(0.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for b in range(len(Gs)):
            assert torch.equal(plan.W(b), ref[b]), (rep, b)
        _ = (torch.ones(1000, device=DEV) * rep).sum().item()   # eager work between replays
    # outside any capture the plan captures and replays its own graph
    plan.run(use_graph=True)
    torch.cuda.synchronize()
    assert plan.graph_fallbacks() == 1
    for b in range(len(Gs)):
        assert torch.equal(plan.W(b), ref[b])
    plan.close()


def test_lstsq_captured_into_a_caller_graph_replays_the_eager_result():
    """geninv_dlstsq without host synchronization, captured on the caller's
    stream (the factorization then keeps to that one stream) and replayed
    three times with eager work in between: every replay gives the same W,
    equal to the eager call's (which runs the trailing updates on the second
    stream) up to the summation order of the split update."""
    _case("lstsq in a caller graph", m=3000, n=700)
    import ctypes
    G, F = w.lowrank_uv(3000, 700, 500, seed=71, k=4)
    Gd, Fd = up(G), up(F)
    Gc, ldg = api.colmajor(Gd)
    Fc, ldf = api.colmajor(Fd)
    lib = api.load()
    vp = ctypes.c_void_p
    try:
        api.set_host_sync(False, DEV)
        W0 = api.empty_colmajor(700, 4, DEV)
        ctx = api._ctx(DEV)
        assert lib.geninv_dlstsq(ctx, 3000, 700, 4, vp(Gc.data_ptr()), ldg, vp(Fc.data_ptr()), ldf, 0.0,
                                 vp(W0.data_ptr()), 700, None) == 0
        torch.cuda.synchronize()
        W = api.empty_colmajor(700, 4, DEV)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx = api._ctx(DEV)
            st = lib.geninv_dlstsq(ctx, 3000, 700, 4, vp(Gc.data_ptr()), ldg, vp(Fc.data_ptr()), ldf, 0.0,
                                   vp(W.data_ptr()), 700, None)
        assert st == 0
        first = None
        for rep in range(3):
            W.fill_(0.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            if first is None:
                first = W.clone()
            assert torch.equal(W, first), rep
            _ = (torch.ones(1000, device=DEV) * rep).sum().item()   # eager work between replays
        assert float(torch.linalg.norm(first - W0) / torch.linalg.norm(W0)) <= 1e-10
    finally:
        api.set_host_sync(True, DEV)
