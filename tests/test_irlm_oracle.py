"""Pins of the IRLM reference (oracle/irlm.py, Algorithm 1 right with PCG
inner solves and thick restarts): closed forms (path), LAPACK's dense
spectrum with cluster-aware vectors, disconnected graphs (zero pairs from
the components), both preconditioners of the inner solves, and the
certificate on every returned pair."""
import numpy as np
import pytest

import oracle
from oracle import irlm
from paper_1311_1695_amd import graphgen as gg
from tests._lapcheck import check_against_reference, residuals


def test_irlm_path_closed_form():
    L = gg.path_graph(120)
    ev, X, info = irlm.irlm(L, 6, 1e-9)
    exact = 2 - 2 * np.cos(np.pi * np.arange(6) / 120)
    assert np.allclose(ev, exact, rtol=1e-9, atol=1e-13)
    assert info["restarts"] >= 0 and info["lanczos_steps"] >= 15


@pytest.mark.parametrize("name", ["grid", "pa", "union", "weighted"])
@pytest.mark.parametrize("precond", [oracle.PREC_JACOBI, oracle.PREC_IC0])
def test_irlm_vs_dense(name, precond):
    if name == "grid":
        L, k = gg.grid_graph(18, 25), 7
    elif name == "pa":
        u, v = gg.pa_edges(1500, 3, 9)
        L, k = gg.laplacian_from_edges(1500, u, v, name="pa1500"), 6
    elif name == "union":
        L, k = gg.disjoint_union(gg.grid_graph(10, 12), gg.path_graph(30), gg.cycle_graph(11)), 6
    else:
        u, v = gg.chung_lu_edges(2000, 2.2, 4.0, 3)
        w = gg.integer_weights(u.shape[0], 4)
        n, u, v, w = gg.largest_component(2000, u, v, w)
        L, k = gg.laplacian_from_edges(n, u, v, w, name="cl2000w"), 6
    ev, X, info = irlm.irlm(L, k, 1e-8, precond=precond)
    w, V = np.linalg.eigh(L.dense())
    check_against_reference(ev, X, w[:30], V[:, :30], val_rtol=1e-8, angle_tol=1e-6)
    rr = residuals(L.to_scipy(), ev, X)
    assert np.all(rr <= 1e-8 * np.maximum(np.minimum(ev, 1.0), (ev <= 0) * 1.0) * (1 + 1e-6) + 1e-13)
