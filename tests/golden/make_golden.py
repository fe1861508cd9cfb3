"""Write the stored expected values of the full-size parity tests.

Every value here comes from the FP64 CPU oracle (``oracle.jd``, Algorithm 2
with the paper's parameters and IC(0)) run on the seeded synthetic
workloads of ``paper_1311_1695_amd.graphgen``; nothing is taken from the
GPU path.  Run from the repository root:

    python tests/golden/make_golden.py [cl330k] [cl1m_tc] [cl1m_tc_stats] [pa_batch]

Outputs (JSON, one file per workload):

* ``cl330k_k20.json``   Chung-Lu exponent 2.1, n = 330,000, k = 20, oracle tol 1e-9
* ``cl1m_tc_k10.json``  Chung-Lu exponent 2.3 + triadic closure, n = 1.1M, k = 10, tol 1e-9
* ``pa_batch256_k5.json`` the 256 preferential-attachment graphs, k = 5 each, tol 1e-10

The 1.1M-vertex file also records the oracle's cost at the benchmark's
tolerance 1e-8 (``oracle_at_tol``), the scale of the benchmark's bounded CPU
sample.

For the two large graphs each file also holds the oracle eigenvectors at
a fixed set of sampled vertices (the 24 largest-magnitude entries of every
vector plus 512 seeded uniform indices, in the caller's vertex order), so
that a test can compare vectors without storing them whole.

The oracle tolerances are the ones the eigenvalue comparison needs: both
solves certify ||G u - theta u|| <= tol * theta, so each theta lies within
||r||^2 / gap of an eigenvalue; 1e-9 on the large graphs sits a few times
above the FP64 rounding floor eps * ||G|| (about 3e-12 there).
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1311_1695_amd import graphgen as gg  # noqa: E402

SEED = 1001          # workload seed of the benchmark and the tests
START_SEED = 1       # seed of the oracle's start vector


def _sample_indices(X, n, seed=7, n_uniform=512, n_top=24):
    rng = np.random.default_rng(seed)
    idx = set(int(i) for i in rng.choice(n, size=min(n_uniform, n), replace=False))
    for j in range(X.shape[1]):
        idx.update(int(i) for i in np.argsort(-np.abs(X[:, j]))[:n_top])
    return np.array(sorted(idx), dtype=np.int64)


def _graph_entry(name, k, tol):
    L = gg.workload(name, SEED)
    st = L.stats()
    t0 = time.perf_counter()
    r = oracle.jd(L, k, tol, precond=oracle.PREC_IC0, seed=START_SEED)
    dt = time.perf_counter() - t0
    assert r.nconv == k, (name, r.nconv)
    G = L.to_scipy()
    res = np.linalg.norm(G @ r.evecs - r.evecs * r.evals, axis=0)
    idx = _sample_indices(r.evecs, L.n)
    return {
        "workload": name, "graph_seed": SEED, "start_seed": START_SEED,
        "n": L.n, "nnz": L.nnz, "d_max": int(st["d_max"]), "k": k, "oracle_tol": tol,
        "oracle": {"solver": "oracle.jd (FP64 Algorithm 2, IC(0), m_min 5, m_max 10, ITMAX 20, "
                             "delta_PCG 1e-2)",
                   "outer": r.outer, "inner": r.inner, "mvp": r.mvp, "seconds": round(dt, 2),
                   "host": platform.processor() or platform.machine(), "threads": 1},
        "evals": [float(x) for x in r.evals],
        "res_abs": [float(x) for x in res],
        "sample_idx": [int(i) for i in idx],
        "sample_evecs": [[float(x) for x in r.evecs[idx, j]] for j in range(k)],
    }


def _batch_member(g):
    L = gg.pa_batch_member(g, 256, SEED)
    r = oracle.jd(L, 5, 1e-10, precond=oracle.PREC_IC0, seed=START_SEED)
    assert r.nconv == 5, (g, r.nconv)
    G = L.to_scipy()
    res = np.linalg.norm(G @ r.evecs - r.evecs * r.evals, axis=0)
    return {"graph": g, "n": L.n, "nnz": L.nnz, "evals": [float(x) for x in r.evals],
            "res_abs": [float(x) for x in res], "mvp": r.mvp, "outer": r.outer}


def _bench_tol_stats(fname, tol):
    """Add the oracle's cost at the benchmark's tolerance (outer iterations,
    products, seconds on one core) to an existing file: the scale of the
    benchmark's bounded CPU sample."""
    path = os.path.join(HERE, fname)
    with open(path) as fh:
        d = json.load(fh)
    L = gg.workload(d["workload"], d["graph_seed"])
    t0 = time.perf_counter()
    r = oracle.jd(L, d["k"], tol, precond=oracle.PREC_IC0, seed=d["start_seed"])
    dt = time.perf_counter() - t0
    assert r.nconv == d["k"]
    d["oracle_at_tol"] = {"tol": tol, "outer": r.outer, "inner": r.inner, "mvp": r.mvp,
                          "seconds": round(dt, 2), "threads": 1,
                          "evals": [float(x) for x in r.evals]}
    _write(fname, d)


def _write(fname, obj):
    path = os.path.join(HERE, fname)
    with open(path + ".tmp", "w") as fh:
        json.dump(obj, fh, indent=0)
        fh.write("\n")
    os.replace(path + ".tmp", path)
    print("wrote", path, flush=True)


def main(argv):
    which = argv or ["cl330k", "cl1m_tc", "pa_batch"]
    if "pa_batch" in which:
        with Pool(min(8, os.cpu_count() or 1)) as pool:
            members = pool.map(_batch_member, range(256), chunksize=4)
        _write("pa_batch256_k5.json", {"workload": "pa_batch256", "graph_seed": SEED,
                                       "start_seed": START_SEED, "k": 5, "oracle_tol": 1e-10,
                                       "members": members})
    if "cl330k" in which:
        _write("cl330k_k20.json", _graph_entry("cl330k", 20, 1e-9))
    if "cl1m_tc" in which:
        _write("cl1m_tc_k10.json", _graph_entry("cl1m_tc", 10, 1e-9))
    if "cl1m_tc" in which or "cl1m_tc_stats" in which:
        _bench_tol_stats("cl1m_tc_k10.json", 1e-8)


if __name__ == "__main__":
    main(sys.argv[1:])
