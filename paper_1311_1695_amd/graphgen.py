"""Seeded synthetic graph generators and Laplacian CSR assembly.

This module only builds *inputs*: edge lists of undirected simple graphs and
the CSR of their Laplacian G = D - A (Section 2: D holds the generalized
degrees, A the weighted adjacency).  It contains none of the eigensolver's
arithmetic and is shared by the CPU oracle's tests and by the GPU path's
tests and benchmark.  Every random draw goes through
``numpy.random.Generator(PCG64(seed))`` so a (generator, parameters, seed)
triple always yields the same graph.

Graph families (the paper's four networks are not redistributable; these
stand in for their shapes, Section 4, Table 1):
  * ``pa_edges``        preferential attachment (Barabasi-Albert), the
                        small protein-like case and the batch members;
  * ``chung_lu_edges``  power-law expected-degree graphs (internet-, www-
                        and dblp-like shapes);
  * ``triadic_closure`` adds collaboration-style triangles (dblp-like);
  * closed-form families (path, cycle, star, complete, complete bipartite,
    hypercube, grid, disjoint unions) used to pin the oracle.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

__all__ = [
    "LaplacianCSR", "laplacian_from_edges", "largest_component",
    "pa_edges", "chung_lu_edges", "triadic_closure", "integer_weights",
    "path_graph", "cycle_graph", "star_graph", "complete_graph",
    "complete_bipartite_graph", "hypercube_graph", "grid_graph",
    "disjoint_union", "workload", "WORKLOADS", "pa_batch", "collaboration",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclasses.dataclass
class LaplacianCSR:
    """CSR of L = D - A with the diagonal stored, columns sorted per row.

    rowptr: int32 (n+1); col: int32 (nnz); val: float64 (nnz).
    nnz = n + 2m for a graph with m edges and no isolated vertex.
    """
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def degrees(self) -> np.ndarray:
        """Number of off-diagonal entries per row (unweighted degree)."""
        counts = np.diff(self.rowptr).astype(np.int64)
        diag_present = np.zeros(self.n, dtype=np.int64)
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        diag_present[rows[self.col == rows]] = 1
        return counts - diag_present

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    def stats(self) -> dict:
        deg = self.degrees()
        return {
            "n": self.n, "nnz": self.nnz, "anzr": self.nnz / max(self.n, 1),
            "d_max": int(deg.max()) if self.n else 0,
            "leaf_frac": float((deg == 1).mean()) if self.n else 0.0,
        }


def _canonical_edges(u: np.ndarray, v: np.ndarray, n: int):
    """Drop self-loops and duplicate undirected edges, keeping the first
    occurrence (generation order is preserved)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a, b = np.minimum(u, v), np.maximum(u, v)
    key = a * n + b
    _, first = np.unique(key, return_index=True)
    first.sort()
    return u[first], v[first]


def laplacian_from_edges(n: int, u, v, w=None, name: str = "") -> LaplacianCSR:
    """Assemble the CSR of G = D - A from an undirected simple edge list.

    Edge k joins u[k] and v[k] with weight w[k] > 0 (1 when ``w`` is None).
    D(i,i) is the generalized degree, the sum of the incident weights.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if w is None:
        w = np.ones(u.shape[0], dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    deg = np.zeros(n, dtype=np.float64)
    np.add.at(deg, u, w)
    np.add.at(deg, v, w)
    diag = np.arange(n, dtype=np.int64)
    rows = np.concatenate([u, v, diag])
    cols = np.concatenate([v, u, diag])
    vals = np.concatenate([-w, -w, deg])
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return LaplacianCSR(n=n, rowptr=m.indptr.astype(np.int32),
                        col=m.indices.astype(np.int32),
                        val=m.data.astype(np.float64), name=name)


def largest_component(n: int, u, v, w=None):
    """Restrict an edge list to its largest connected component, relabelling
    the kept vertices 0..n'-1 in their original order."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    adj = sp.coo_matrix((np.ones(u.shape[0]), (u, v)), shape=(n, n))
    ncomp, labels = csgraph.connected_components(adj, directed=False)
    if ncomp == 1:
        return n, u, v, w
    sizes = np.bincount(labels, minlength=ncomp)
    big = int(np.argmax(sizes))
    keep = labels == big
    newid = -np.ones(n, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    ek = keep[u]
    w2 = None if w is None else np.asarray(w)[ek]
    return int(keep.sum()), newid[u[ek]], newid[v[ek]], w2


# --------------------------------------------------------------------------
# Random families
# --------------------------------------------------------------------------

def pa_edges(n: int, m: int, seed: int):
    """Preferential attachment: start from the complete graph on m+1 nodes;
    each later node t joins m distinct earlier nodes, each drawn uniformly
    from the list of all edge endpoints so far (so proportionally to degree),
    redrawing duplicates.  Connected by construction."""
    if n <= m:
        raise ValueError("pa_edges needs n > m")
    rng = _rng(seed)
    us, vs = [], []
    ends = np.empty(2 * (m * (m + 1) // 2 + m * (n - m - 1)), dtype=np.int64)
    ne = 0
    for a in range(m + 1):
        for b in range(a + 1, m + 1):
            us.append(b); vs.append(a)
            ends[ne] = a; ends[ne + 1] = b; ne += 2
    # pre-draw uniforms in chunks; each pick consumes one
    buf = rng.random(4 * m * n + 64)
    bi = 0
    for t in range(m + 1, n):
        chosen = []
        while len(chosen) < m:
            if bi >= buf.shape[0]:
                buf = rng.random(4 * m * n + 64); bi = 0
            x = int(ends[int(buf[bi] * ne)]); bi += 1
            if x not in chosen:
                chosen.append(x)
        for x in chosen:
            us.append(t); vs.append(x)
            ends[ne] = t; ends[ne + 1] = x; ne += 2
    return np.asarray(us, dtype=np.int64), np.asarray(vs, dtype=np.int64)


def chung_lu_weights(n: int, gamma: float, mean_deg: float, w_max: float) -> np.ndarray:
    """Expected degrees w_i = c (i0 + i)^(-1/(gamma-1)), i = 0..n-1, with
    c and i0 fixed by w_0 = w_max and mean(w) = mean_deg."""
    alpha = 1.0 / (gamma - 1.0)
    idx = np.arange(n, dtype=np.float64)
    if w_max <= mean_deg:
        raise ValueError("w_max must exceed the mean degree")

    def mean_for(i0):
        return w_max * np.mean((1.0 + idx / i0) ** (-alpha))

    lo, hi = 1e-6, 1e12
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) < mean_deg:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    return w_max * (1.0 + idx / i0) ** (-alpha)


def chung_lu_edges(n: int, gamma: float, mean_deg: float, seed: int, w_max: float | None = None):
    """Chung-Lu graph: Poisson(sum(w)/2) endpoint pairs drawn i.i.d. with
    probability proportional to w, self-loops and duplicates dropped.
    The default cutoff w_max = sqrt(n * mean_deg) is the structural one."""
    if w_max is None:
        w_max = math.sqrt(n * mean_deg)
    w = chung_lu_weights(n, gamma, mean_deg, w_max)
    rng = _rng(seed)
    S = float(w.sum())
    M = int(rng.poisson(S / 2.0))
    cdf = np.cumsum(w / S)
    cdf[-1] = 1.0
    ends = np.searchsorted(cdf, rng.random(2 * M), side="right")
    ends = np.minimum(ends, n - 1)
    return _canonical_edges(ends[0::2], ends[1::2], n)


def triadic_closure(n: int, u, v, p: float, seed: int):
    """For every edge (u, v), in generation order, with probability p pick a
    neighbour x of v uniformly (in the graph before closure) and add (u, x)
    when x != u; duplicates collapse."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    rng = _rng(seed)
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    order = np.argsort(rows, kind="stable")
    rows, cols = rows[order], cols[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    pick = rng.random(u.shape[0]) < p
    r2 = rng.random(u.shape[0])
    uu, vv = u[pick], v[pick]
    deg_v = rowptr[vv + 1] - rowptr[vv]
    x = cols[rowptr[vv] + np.minimum((r2[pick] * deg_v).astype(np.int64), deg_v - 1)]
    return _canonical_edges(np.concatenate([u, uu]), np.concatenate([v, x]), n)


def integer_weights(num_edges: int, seed: int) -> np.ndarray:
    """Integer edge weights 1, 2, 3, ... with P(w = j) = 2^-j (publication
    counts of a collaboration network)."""
    return _rng(seed).geometric(0.5, size=num_edges).astype(np.float64)


# --------------------------------------------------------------------------
# Closed-form families
# --------------------------------------------------------------------------

def path_graph(n: int) -> LaplacianCSR:
    i = np.arange(n - 1)
    return laplacian_from_edges(n, i, i + 1, name=f"path{n}")


def cycle_graph(n: int) -> LaplacianCSR:
    i = np.arange(n)
    return laplacian_from_edges(n, i, (i + 1) % n, name=f"cycle{n}")


def star_graph(n: int) -> LaplacianCSR:
    """Hub 0 joined to n-1 leaves."""
    i = np.arange(1, n)
    return laplacian_from_edges(n, np.zeros(n - 1, dtype=np.int64), i, name=f"star{n}")


def complete_graph(n: int) -> LaplacianCSR:
    a, b = np.triu_indices(n, 1)
    return laplacian_from_edges(n, a, b, name=f"K{n}")


def complete_bipartite_graph(a: int, b: int) -> LaplacianCSR:
    x, y = np.meshgrid(np.arange(a), a + np.arange(b), indexing="ij")
    return laplacian_from_edges(a + b, x.ravel(), y.ravel(), name=f"K{a},{b}")


def hypercube_graph(d: int) -> LaplacianCSR:
    n = 1 << d
    us, vs = [], []
    for bit in range(d):
        i = np.arange(n)
        j = i ^ (1 << bit)
        keep = i < j
        us.append(i[keep]); vs.append(j[keep])
    return laplacian_from_edges(n, np.concatenate(us), np.concatenate(vs), name=f"Q{d}")


def grid_graph(a: int, b: int) -> LaplacianCSR:
    idx = np.arange(a * b).reshape(a, b)
    us = [idx[:-1, :].ravel(), idx[:, :-1].ravel()]
    vs = [idx[1:, :].ravel(), idx[:, 1:].ravel()]
    return laplacian_from_edges(a * b, np.concatenate(us), np.concatenate(vs), name=f"grid{a}x{b}")


def disjoint_union(*graphs: LaplacianCSR) -> LaplacianCSR:
    us, vs, ws = [], [], []
    off = 0
    for g in graphs:
        rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
        mask = g.col > rows
        us.append(rows[mask] + off); vs.append(g.col[mask].astype(np.int64) + off)
        ws.append(-g.val[mask])
        off += g.n
    return laplacian_from_edges(off, np.concatenate(us), np.concatenate(vs), np.concatenate(ws),
                                name="+".join(g.name for g in graphs))


# --------------------------------------------------------------------------
# The named workloads (synthetic stand-ins for the paper's networks)
# --------------------------------------------------------------------------

def _pa_lcc(n, m, seed, name):
    u, v = pa_edges(n, m, seed)
    n2, u, v, _ = largest_component(n, u, v)
    return laplacian_from_edges(n2, u, v, name=name)


def _cl_lcc(n, gamma, dbar, seed, name, w_max=None, triadic=None, weighted=False):
    u, v = chung_lu_edges(n, gamma, dbar, seed, w_max)
    if triadic:
        u, v = triadic_closure(n, u, v, triadic, seed + 7919)
    w = integer_weights(u.shape[0], seed + 104729) if weighted else None
    n2, u, v, w = largest_component(n, u, v, w)
    return laplacian_from_edges(n2, u, v, w, name=name)


def collaboration(n: int, seed: int, weighted: bool = False) -> LaplacianCSR:
    """The collaboration-like family of the warm-start workload (Chung-Lu
    exponent 2.3, mean degree 7, triadic closure 0.3, largest component) at
    any size: the graphs the warm-start network is trained on."""
    return _cl_lcc(n, 2.3, 7.0, seed, f"collab{n}", triadic=0.3, weighted=weighted)


WORKLOADS = {
    # name: (builder, default k, description)
    "pa5k": (lambda seed: _pa_lcc(5000, 3, seed, "pa5k"), 10,
             "preferential attachment n=5000 m=3, LCC"),
    "cl30k": (lambda seed: _cl_lcc(30000, 2.2, 4.0, seed, "cl30k"), 10,
              "Chung-Lu gamma=2.2 n=30000 mean degree 4, LCC"),
    "cl330k": (lambda seed: _cl_lcc(330000, 2.1, 9.0, seed, "cl330k", w_max=1.35e4), 20,
               "Chung-Lu gamma=2.1 n=330000 mean degree 9, max degree ~1e4, LCC"),
    "cl1m_tc": (lambda seed: _cl_lcc(1100000, 2.3, 7.0, seed, "cl1m_tc", triadic=0.3), 10,
                "Chung-Lu gamma=2.3 n=1.1M mean degree 7 + triadic closure p=0.3, LCC"),
    "cl30k_w": (lambda seed: _cl_lcc(30000, 2.2, 4.0, seed, "cl30k_w", weighted=True), 10,
                "cl30k with integer weights 1+Geometric(1/2)"),
}


def workload(name: str, seed: int) -> LaplacianCSR:
    return WORKLOADS[name][0](seed)


def _pa_batch_sizes(num, seed, n_lo, n_hi, ms):
    rng = _rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=num)
    mm = rng.choice(np.asarray(ms), size=num)
    return ns, mm


def pa_batch(num: int, seed: int, n_lo: int = 1000, n_hi: int = 20000, ms=(2, 3, 4)):
    """A batch of uneven preferential-attachment graphs: graph g has
    n ~ U{n_lo..n_hi}, m ~ U(ms), and its own seed derived from ``seed``."""
    ns, mm = _pa_batch_sizes(num, seed, n_lo, n_hi, ms)
    return [_pa_lcc(int(ns[g]), int(mm[g]), seed * 1000 + g, f"pa_b{g}") for g in range(num)]


def pa_batch_member(g: int, num: int, seed: int, n_lo: int = 1000, n_hi: int = 20000, ms=(2, 3, 4)):
    """Graph g of pa_batch(num, seed, ...) alone."""
    ns, mm = _pa_batch_sizes(num, seed, n_lo, n_hi, ms)
    return _pa_lcc(int(ns[g]), int(mm[g]), seed * 1000 + g, f"pa_b{g}")
