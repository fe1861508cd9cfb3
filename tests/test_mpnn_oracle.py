"""Pins of the FP64 reference of the warm-start network (oracle/mpnn_oracle.py)
against things other than itself: central finite differences of its loss for
every parameter, hand examples of the aggregation, the adjoint identity of
the aggregation and its transpose, the invariances of the subspace loss, and
the scalar SplitMix64 of the C oracle (itself pinned to published values)."""
import math

import numpy as np
import pytest

import oracle
from oracle import mpnn_oracle as mo
from paper_1311_1695_amd import graphgen as gg


def _orthonormal_target(gr, k, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((gr.n, k))
    X -= gr.Z @ (gr.Z.T @ X)
    return np.linalg.qr(X)[0]


@pytest.mark.parametrize("seed", [0, 7, 123456789])
def test_splitmix_matches_the_c_oracle(seed):
    idx = np.array([0, 1, 2, 17, 1000, 2 ** 40 + 3], dtype=np.uint64)
    got = mo.splitmix_unit(seed, idx)
    ref = np.array([oracle.start_value(seed, int(i)) for i in idx])
    assert np.array_equal(got, ref)


def test_aggregation_hand_examples():
    # star: the centre averages its leaves, each leaf takes the centre
    L = gg.star_graph(6)  # centre 0, leaves 1..5
    gr = mo.Graph(L)
    h = np.arange(6, dtype=float)
    a = gr.agg(h)
    assert a[0] == pytest.approx(np.mean(h[1:]))
    assert np.all(a[1:] == h[0])
    # weighted path 0 -(2)- 1 -(1)- 2: the middle vertex weighs its neighbours 2:1
    u, v, w = np.array([0, 1]), np.array([1, 2]), np.array([2.0, 1.0])
    gr = mo.Graph(gg.laplacian_from_edges(3, u, v, w))
    a = gr.agg(np.array([3.0, 0.0, 6.0]))
    assert a[1] == pytest.approx((2 * 3 + 1 * 6) / 3)
    assert a[0] == 0.0 and a[2] == 0.0


def test_aggregation_transpose_is_its_adjoint():
    gr = mo.Graph(gg.laplacian_from_edges(50, *gg.pa_edges(50, 2, 3)))
    rng = np.random.default_rng(1)
    U, V = rng.standard_normal((50, 4)), rng.standard_normal((50, 4))
    assert np.sum(gr.agg(U) * V) == pytest.approx(np.sum(U * gr.agg_t(V)), rel=1e-12)


def test_features_on_a_path():
    gr = mo.Graph(gg.path_graph(4))  # degrees 1 2 2 1
    cfg = mo.Config(layers=1, hidden=2, random_channels=2, out_cols=1)
    f = mo.features(cfg, gr, seed=5)
    l1, l2 = math.log(2.0), math.log(3.0)
    assert np.allclose(f[:, 0], 1.0)
    assert np.allclose(f[:, 1], [l1, l2, l2, l1])
    assert np.allclose(f[:, 2], [l2, (l1 + l2) / 2, (l1 + l2) / 2, l2])
    assert np.allclose(f[:, 3:], math.sqrt(3) * mo.splitmix_unit(5, np.arange(8).reshape(4, 2)))


def test_subspace_loss_invariances():
    rng = np.random.default_rng(2)
    n, k, p = 200, 3, 5
    X = np.linalg.qr(rng.standard_normal((n, k)))[0]
    Yc = np.concatenate([X @ rng.standard_normal((k, k)), rng.standard_normal((n, p - k))], axis=1)
    loss, grad = mo.subspace_loss(Yc, X)
    assert abs(loss) < 1e-12 and np.abs(grad).max() < 1e-10  # span Y contains span X
    Y = rng.standard_normal((n, p))
    R = rng.standard_normal((p, p)) + 3 * np.eye(p)
    l1, _ = mo.subspace_loss(Y, X)
    l2, _ = mo.subspace_loss(Y @ R, X)
    assert l1 == pytest.approx(l2, rel=1e-10) and 0.0 < l1 < 1.0
    Yo = Y - X @ (X.T @ Y)  # orthogonal to X
    assert mo.subspace_loss(Yo, X)[0] == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_matches_central_differences(weighted):
    rng = np.random.default_rng(11)
    n = 40
    u, v = gg.pa_edges(n, 2, 4)
    w = rng.integers(1, 4, size=len(u)).astype(float) if weighted else None
    gr = mo.Graph(gg.laplacian_from_edges(n, u, v, w))
    cfg = mo.Config(layers=2, hidden=5, random_channels=2, out_cols=3)
    params = mo.init_params(cfg, 99) + 0.05 * rng.standard_normal(cfg.num_params())
    X = _orthonormal_target(gr, 2, 5)
    loss, grad = mo.loss_and_grad(cfg, params, gr, 3, X)
    assert 0.0 < loss < 1.0
    h = 1e-6
    fd = np.empty_like(params)
    for j in range(params.size):
        e = np.zeros_like(params)
        e[j] = h
        fd[j] = (mo.loss_and_grad(cfg, params + e, gr, 3, X)[0] - mo.loss_and_grad(cfg, params - e, gr, 3, X)[0]) / (2 * h)
    assert np.abs(grad - fd).max() <= 1e-6 * max(np.abs(fd).max(), 1e-3)


def test_output_is_orthogonal_to_the_zero_space():
    L = gg.disjoint_union(gg.path_graph(10), gg.star_graph(7))
    gr = mo.Graph(L)
    cfg = mo.Config(layers=1, hidden=4, random_channels=1, out_cols=3)
    Yh, _ = mo.forward(cfg, mo.init_params(cfg, 1), gr, 2)
    assert gr.Z.shape[1] == 2
    assert np.abs(gr.Z.T @ Yh).max() < 1e-12


def test_adam_closed_forms():
    """Pins of the Adam reference (Kingma & Ba 2015, Algorithm 1) that do not
    restate its code: the first step from zero moments and every step under a
    constant gradient move by lr * g / (|g| + eps) (the bias corrections make
    the corrected moments g and g^2 exactly), zero gradient only decays the
    moments, and a two-step hand example."""
    rng = np.random.default_rng(11)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50) * np.logspace(-3, 2, 50)
    lr = 0.01
    p1, m1, v1 = mo.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # constant gradient: the same step every time
    pt, mt, vt = p, np.zeros(50), np.zeros(50)
    for t in range(1, 40):
        prev = pt
        pt, mt, vt = mo.adam_step(pt, g, mt, vt, t, lr)
        assert np.allclose(pt - prev, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-16)
    # zero gradient: the moments decay by beta1 and beta2
    p2, m2, v2 = mo.adam_step(pt, np.zeros(50), mt, vt, 40, lr)
    assert np.allclose(m2, 0.9 * mt, rtol=1e-15) and np.allclose(v2, 0.999 * vt, rtol=1e-15)
    # hand example, g = +1 then -1, lr = 1, eps = 0:
    #   step 1: m = 0.1, v = 0.001, m_hat = 1, v_hat = 1 -> move -1
    #   step 2: m = 0.09 - 0.1 = -0.01, v = 0.000999 + 0.001 = 0.001999,
    #           m_hat = -0.01 / 0.19, v_hat = 0.001999 / 0.001999 = 1 -> move +1/19
    q1, a1, b1 = mo.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, 1.0, eps=0.0)
    assert abs(q1[0] + 1.0) < 1e-15 and abs(a1[0] - 0.1) < 1e-16 and abs(b1[0] - 0.001) < 1e-18
    q2, a2, b2 = mo.adam_step(q1, -np.ones(1), a1, b1, 2, 1.0, eps=0.0)
    assert abs(a2[0] + 0.01) < 1e-16 and abs(b2[0] - 0.001999) < 1e-17
    assert abs(q2[0] - (-1.0 + 1.0 / 19.0)) < 1e-14
    # the step opposes the gradient and is invariant to scaling g and eps together
    s1, _, _ = mo.adam_step(p, 1e3 * g, np.zeros(50), np.zeros(50), 1, lr, eps=1e-5)
    assert np.allclose(s1, p1, rtol=0, atol=1e-14)
    assert np.all(np.sign(p1 - p) == -np.sign(g))
