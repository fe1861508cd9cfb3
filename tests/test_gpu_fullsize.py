"""GPU parity at the full sizes of the benchmark workloads, against stored
oracle results (tests/golden, written by make_golden.py, which calls only
the CPU oracle and the input generators):

* the Chung-Lu exponent-2.1 graph, n = 297,292: 20 smallest pairs by block
  JD with a 20-column block, mixed precision and FP64;
* the collaboration-like graph, n = 1,032,939: 10 smallest pairs, mixed
  precision from the seeded random start and from a trained network's
  block (single-vector JD and block JD with a 10-column block), with the
  FSAI preconditioner, and FP64 from the random start;
* the 256 preferential-attachment graphs of the batch workload (n up to
  20k; in FP64 the largest keep part of their PCG direction in memory), 5
  pairs each, both precisions, in the one-launch batched solver.

Bars: every eigenvalue within relative 1e-8 of the oracle's (both sides
certify ||Gu - theta u|| <= tol theta, and the gaps of these spectra make
the quadratic residual bound far smaller than that); every residual,
recomputed here in FP64 from the returned vectors, within the requested
tolerance; orthonormal vectors; and, for the two large graphs, the vectors
compared with the oracle's at the stored sample of vertices, cluster by
cluster, up to a rotation within the cluster.
"""
import functools
import json
import os

import numpy as np
import pytest

import paper_1311_1695_amd as lap
from paper_1311_1695_amd import graphgen as gg
from tests._lapcheck import clusters, residuals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lap.load_library()
    yield


@functools.lru_cache(maxsize=None)
def golden(fname):
    with open(os.path.join(HERE, "golden", fname)) as fh:
        return json.load(fh)


@functools.lru_cache(maxsize=None)
def graph(name):
    return gg.workload(name, 1001)


@functools.lru_cache(maxsize=None)
def plan(name):
    return lap.Plan(graph(name))


def check_values(evals, ref, tol=TOL):
    ref = np.asarray(ref[:len(evals)])
    err = np.abs(np.asarray(evals) - ref)
    assert np.all(err <= tol * ref + 1e-13), (err / np.maximum(ref, 1e-300), ref)
    return err


def check_certified(L, evals, evecs, tol=TOL):
    rr = residuals(L.to_scipy(), evals, evecs)
    bound = tol * np.maximum(np.minimum(evals, 1.0), (evals <= 0) * 1.0)
    assert np.all(rr <= bound * (1 + 1e-6) + 1e-14), (rr, bound)
    assert np.abs(evecs.T @ evecs - np.eye(evecs.shape[1])).max() <= 1e-10


def check_sampled_vectors(evecs, gold, k):
    """Each cluster of the oracle's spectrum that lies inside the first k and
    ends before the last stored value: the GPU vectors restricted to the
    sampled vertices equal the oracle's restricted vectors times a c x c
    matrix (a sign for a simple eigenvalue, a rotation inside a cluster)
    to within 2e-6 sqrt(c), the restriction of the 1e-6 angle bound."""
    idx = np.asarray(gold["sample_idx"])
    Xs = np.asarray(gold["sample_evecs"]).T  # |S| x k
    ref = np.asarray(gold["evals"])
    checked = 0
    for c in clusters(ref, rel_gap=1e-2):
        if max(c) >= k or max(c) + 1 >= len(ref):
            continue
        Ys = evecs[idx][:, c]
        R, *_ = np.linalg.lstsq(Xs[:, c], Ys, rcond=None)
        misfit = np.linalg.norm(Ys - Xs[:, c] @ R)
        assert misfit <= 2e-6 * np.sqrt(len(c)), (c, misfit)
        assert np.abs(R.T @ R - np.eye(len(c))).max() <= 1e-4, (c, R)
        checked += len(c)
    return checked


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_block_jd_b20_cl330k_k20_vs_oracle(precision):
    gold = golden("cl330k_k20.json")
    L = graph("cl330k")
    assert (L.n, L.nnz) == (gold["n"], gold["nnz"])
    r = lap.lap_eigs(plan("cl330k"), 20, TOL, precision=precision, block=20, m_min=20, m_max=60, seed=1)
    assert r.nconv == 20 and r.ncomp == 1
    err = check_values(r.evals, gold["evals"])
    check_certified(L, r.evals, r.evecs)
    n_checked = check_sampled_vectors(r.evecs, gold, 20)
    print(f"cl330k block b=20 {precision}: max rel eigenvalue error "
          f"{float(np.max(err[1:] / np.asarray(gold['evals'][1:20]))):.2e}, "
          f"{n_checked} vectors compared at {len(gold['sample_idx'])} vertices, outer {r.outer}, mvp {r.mvp}")


@functools.lru_cache(maxsize=None)
def trained_network():
    """A warm-start network trained on the GPU on three same-family graphs."""
    train = [gg.collaboration(n, s) for n, s in ((6000, 61), (9000, 62), (12000, 63))]
    plans = [lap.Plan(L) for L in train]
    targets = [lap.lap_eigs(p, 10, 1e-6, evecs_on_device=True).evecs[1:].contiguous() for p in plans]
    net = lap.Mpnn(layers=2, hidden=32, random_channels=4, out_cols=9, seed=7)
    for s in range(150):
        g = s % len(plans)
        net.train_step(plans[g], targets[g], lr=3e-3, feature_seed=1)
    return net


@pytest.mark.parametrize("precision,start", [("mixed", "random"), ("mixed", "network"), ("fp64", "random"),
                                             ("mixed", "fsai"), ("mixed", "block_network"),
                                             ("mixed", "block_random"), ("fp64", "block_random")])
def test_collaboration_1m_k10_vs_oracle(precision, start):
    gold = golden("cl1m_tc_k10.json")
    L = graph("cl1m_tc")
    assert (L.n, L.nnz) == (gold["n"], gold["nnz"])
    p = plan("cl1m_tc")
    kw = {}
    if start in ("network", "block_network"):
        kw["init"] = trained_network().infer(p, feature_seed=1)
    if start in ("block_network", "block_random"):
        kw.update(block=10, m_min=20, m_max=50)
    if start == "fsai":
        kw["precond"] = "fsai"
    r = lap.lap_eigs(p, 10, TOL, precision=precision, seed=1, **kw)
    assert r.nconv == 10 and r.ncomp == 1
    err = check_values(r.evals, gold["evals"])
    check_certified(L, r.evals, r.evecs)
    n_checked = check_sampled_vectors(r.evecs, gold, 10)
    print(f"cl1m_tc {precision} {start}: per-pair rel error "
          f"{np.array2string(err[1:] / np.asarray(gold['evals'][1:10]), precision=2)}, "
          f"{n_checked} vectors compared, outer {r.outer}, mvp {r.mvp}")


@functools.lru_cache(maxsize=None)
def batch_graphs():
    return gg.pa_batch(256, 1001)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_256_graphs_vs_oracle(precision):
    gold = golden("pa_batch256_k5.json")
    graphs = batch_graphs()
    assert len(gold["members"]) == len(graphs) == 256
    # the largest members exceed the 18.9k vertices whose FP64 PCG direction fits in LDS
    assert max(g.n for g in graphs) > 18900
    out = lap.lap_eigs_batch(graphs, 5, TOL, precision=precision)
    worst = 0.0
    for L, r, m in zip(graphs, out, gold["members"]):
        assert (L.n, L.nnz) == (m["n"], m["nnz"])
        assert r.nconv == 5, L.name
        err = check_values(r.evals, m["evals"])
        worst = max(worst, float(np.max(err[1:] / np.asarray(m["evals"][1:5]))))
        check_certified(L, r.evals, r.evecs)
    print(f"batch {precision}: worst rel eigenvalue error over 256 x 4 pairs {worst:.2e}")
