"""Pins of the consumers' reference (oracle/consumers.py) against what
Section 2 and the mathematics fix: the pseudo-inverse G^+ from LAPACK, the
identity between the paper's two expressions of S^(k), the projector
identity G T^(k) = sum_{j<=k} v_j v_j', the closed form of the relaxed
bisection optimum, and brute force over every balanced partition of small
graphs (the relaxed optimum bounds every cut of those sizes from below)."""
import itertools

import numpy as np
import pytest

from oracle import consumers as cs
from paper_1311_1695_amd import graphgen as gg


def _small_graphs():
    u, v = gg.chung_lu_edges(120, 2.2, 4.0, 5)
    w = gg.integer_weights(u.shape[0], 6)
    n, u, v, w = gg.largest_component(120, u, v, w)
    return [gg.path_graph(30), gg.grid_graph(5, 7),
            gg.laplacian_from_edges(n, u, v, w, name="cl120w"),
            gg.disjoint_union(gg.cycle_graph(9), gg.star_graph(7))]


@pytest.mark.parametrize("L", _small_graphs(), ids=lambda g: g.name[:16])
def test_T_full_spectrum_is_the_pseudo_inverse(L):
    G = L.dense()
    w, V = np.linalg.eigh(G)
    w[np.abs(w) < 1e-10] = 0.0
    X = np.random.default_rng(1).standard_normal((L.n, 3))
    assert np.allclose(cs.pinv_T(w, V, X), np.linalg.pinv(G) @ X, rtol=1e-9, atol=1e-9 * np.abs(X).max())


@pytest.mark.parametrize("L", _small_graphs(), ids=lambda g: g.name[:16])
@pytest.mark.parametrize("k", [2, 5, 9])
def test_S_second_form_equals_the_first(L, k):
    G = L.dense()
    w, V = np.linalg.eigh(G)
    w[np.abs(w) < 1e-10] = 0.0
    k = max(k, int((w == 0).sum()) + 1)
    sigma = 0.5 * (w[k - 1] + w[-1])
    X = np.random.default_rng(2).standard_normal((L.n, 2))
    # first form: T^(k) + (1/sigma) sum_{j > k} v_j v_j' (needs the whole spectrum)
    first = cs.pinv_T(w[:k], V[:, :k], X) + V[:, k:] @ (V[:, k:].T @ X) / sigma
    assert np.allclose(cs.pinv_S(w[:k], V[:, :k], sigma, X), first, rtol=1e-10, atol=1e-10 * np.abs(first).max())


def test_T_projector_identity():
    L = _small_graphs()[2]
    G = L.dense()
    w, V = np.linalg.eigh(G)
    w[np.abs(w) < 1e-10] = 0.0
    X = np.random.default_rng(3).standard_normal((L.n, 4))
    k = 7
    P = V[:, 1:k] @ V[:, 1:k].T
    assert np.allclose(G @ cs.pinv_T(w[:k], V[:, :k], X), P @ X, atol=1e-10)


def test_bisect_path_and_barbell():
    # the Fiedler vector of a path is monotone: the halves split at the middle edge
    P = gg.path_graph(12)
    w, V = np.linalg.eigh(P.dense())
    part, cut = cs.bisect(P, V[:, 1], 6)
    assert cut == 1.0 and (part[:6] == part[0]).all() and (part[6:] != part[0]).all()
    # two K5 joined by one edge: the bridge is the cut
    K = gg.complete_graph(5)
    iu, ju = np.triu_indices(5, 1)
    u = np.concatenate([iu, iu + 5, [4]])
    v = np.concatenate([ju, ju + 5, [5]])
    B = gg.laplacian_from_edges(10, u, v)
    w, V = np.linalg.eigh(B.dense())
    part, cut = cs.bisect(B, V[:, 1], 5)
    assert cut == 1.0 and part.sum() == 5
    # ties go by index
    part, _ = cs.bisect(P, np.zeros(12), 4)
    assert part.tolist() == [0] * 4 + [1] * 8


def test_relaxed_optimum_closed_form():
    L = _small_graphs()[2]
    G = L.dense()
    w, V = np.linalg.eigh(G)
    n = L.n
    for n1 in (1, n // 3, n // 2):
        x, val = cs.relaxed_optimum(n1, n, w[1], V[:, 1])
        assert np.isclose(x @ x, n / 4, rtol=1e-12)
        assert np.isclose(x.sum(), (n1 - (n - n1)) / 2, rtol=1e-12, atol=1e-12)
        assert np.isclose(x @ G @ x, val, rtol=1e-10)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bisection_bound_by_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 12
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < 0.35
    u, v = iu[keep], ju[keep]
    n2, u, v, _ = gg.largest_component(n, u, v)
    L = gg.laplacian_from_edges(n2, u, v, rng.integers(1, 4, size=u.size).astype(float))
    G = L.dense()
    w, V = np.linalg.eigh(G)
    n = L.n
    n1 = n // 2
    best = min(sum(-G[i, j] for i in S for j in range(n) if j not in S)
               for S in map(set, itertools.combinations(range(n), n1)))
    part, cut = cs.bisect(L, V[:, 1], n1)
    bound = n1 * (n - n1) * w[1] / n
    assert best >= bound - 1e-9
    assert cut >= best - 1e-12
    x = np.where(part == 0, -0.5, 0.5)
    assert np.isclose(x @ G @ x, cut)  # the cut size is x'Gx, eq. (1)
