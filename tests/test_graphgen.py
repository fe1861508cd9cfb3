"""Seeded input generators: determinism, Laplacian structure, family shapes."""
import numpy as np

from paper_1311_1695_amd import graphgen as gg


def _is_laplacian(L):
    G = L.to_scipy()
    assert (G - G.T).nnz == 0
    assert np.allclose(np.asarray(G.sum(axis=1)).ravel(), 0.0)
    off = G.copy()
    off.setdiag(0)
    assert off.data.max(initial=0.0) <= 0.0
    for i in range(L.n):
        seg = L.col[L.rowptr[i]:L.rowptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_determinism_and_structure():
    a = gg.workload("pa5k", 42)
    b = gg.workload("pa5k", 42)
    c = gg.workload("pa5k", 43)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert not (a.col.shape == c.col.shape and np.array_equal(a.col, c.col))
    _is_laplacian(a)
    # preferential attachment with m = 3: nnz = n + 2m_edges, min degree 3
    assert a.n == 5000 and a.nnz == 5000 + 2 * (6 + 3 * (5000 - 4))
    assert a.degrees().min() == 3


def test_chung_lu_shape_like_internet():
    L = gg.workload("cl30k", 1001)
    _is_laplacian(L)
    st = L.stats()
    # largest component of a gamma = 2.2, mean-degree-4 Chung-Lu graph
    assert 20000 < st["n"] < 28000
    assert 5.0 < st["anzr"] < 7.0
    assert st["leaf_frac"] > 0.2
    assert 200 < st["d_max"] < 600


def test_weighted_and_closed_forms():
    L = gg.workload("cl30k_w", 3)
    _is_laplacian(L)
    off = -L.val[L.val < 0]
    assert np.all(off == np.round(off)) and off.min() >= 1.0
    for g in [gg.path_graph(5), gg.cycle_graph(5), gg.star_graph(5), gg.complete_graph(5),
              gg.complete_bipartite_graph(2, 3), gg.hypercube_graph(3), gg.grid_graph(3, 4)]:
        _is_laplacian(g)
    u = gg.disjoint_union(gg.path_graph(3), gg.cycle_graph(4))
    assert u.n == 7 and u.nnz == 3 + 4 + 2 * (2 + 4)


def test_triadic_closure_adds_triangles():
    u, v = gg.chung_lu_edges(5000, 2.3, 7.0, 5)
    u2, v2 = gg.triadic_closure(5000, u, v, 0.3, 6)
    assert len(u2) > len(u)
    # every original edge survives, in order
    assert np.array_equal(u2[:len(u)], u) and np.array_equal(v2[:len(v)], v)


def test_pa_batch_sizes():
    graphs = gg.pa_batch(4, 9, n_lo=1000, n_hi=2000)
    assert len(graphs) == 4
    for g in graphs:
        assert 1000 <= g.n <= 2000
        _is_laplacian(g)


def test_pa_batch_member_is_the_batch_graph():
    graphs = gg.pa_batch(5, 17)
    for g in range(5):
        one = gg.pa_batch_member(g, 5, 17)
        assert one.n == graphs[g].n
        assert np.array_equal(one.rowptr, graphs[g].rowptr) and np.array_equal(one.col, graphs[g].col)
