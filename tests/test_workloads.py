"""Seeded generators: shapes, determinism and construction properties."""
import numpy as np

from paper_0804_4809_amd import workloads as w


def test_seeded_determinism():
    a, fa = w.c1_problem(0)
    b, fb = w.c1_problem(0)
    assert np.array_equal(a, b) and np.array_equal(fa, fb)
    c, _ = w.c1_problem(1)
    assert not np.array_equal(a, c)


def test_c1_shape_and_rank():
    G, F = w.c1_problem(0)
    assert G.shape == (200, 50) and F.shape == (200, 3)
    assert np.linalg.matrix_rank(G) == 40


def test_rbf_duplicates_follow_their_original():
    G, F, idx = w.rbf_design(300, 4, 50, 20, 0.3, seed=3, k=2)
    assert G.shape == (300, 70) and F.shape == (300, 2)
    first = {}
    for j, c in enumerate(idx):
        if c in first:
            assert np.array_equal(G[:, j], G[:, first[c]])
        else:
            first[c] = j
    assert len(first) == 50
    assert np.all((G > 0) & (G <= 1))


def test_table1_family():
    G = w.table1(64, seed=2)
    assert G.shape == (128, 64)
    assert np.abs(G).max() <= 1.0
    assert np.linalg.matrix_rank(G) == 56


def test_svd_family_singular_values():
    G, _, P, s, Q = w.svd_family(200, 60, 40, 1e-3, seed=1)
    sv = np.linalg.svd(G, compute_uv=False)
    assert np.allclose(sv[:40], s, rtol=1e-10)
    assert sv[40] < 1e-12


def test_batch_ranges():
    B = w.batch_lowrank(200, seed=5)
    assert np.all((B.m >= 64) & (B.m <= 1024))
    assert np.all((B.n >= 16) & (B.n <= np.minimum(256, B.m // 2)))
    assert np.all((B.rank >= B.n // 2) & (B.rank <= B.n))
    for b in range(5):
        assert B.G[b].dtype == np.float32 and B.G[b].shape == (B.m[b], B.n[b])
        assert B.F[b].shape == (B.m[b], 4)
