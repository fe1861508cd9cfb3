"""GPU tests of the warm-start network (lap_mpnn_*): its forward pass, loss
and every gradient entry against the FP64 reference of oracle/mpnn_oracle.py
on the same parameters and inputs; training on the GPU lowers the loss;
and a trained network's start block leaves lap_eigs' certified answer
unchanged while the iteration count it saves (or costs) is reported."""
import functools

import numpy as np
import pytest

from oracle import mpnn_oracle as mo
import paper_1311_1695_amd as lap
from paper_1311_1695_amd import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lap.load_library()
    yield


def chung_lu_tc(n, seed, weighted=False):
    """The collaboration-like family (Chung-Lu exponent 2.3, mean degree 7,
    triadic closure 0.3, largest component)."""
    return gg.collaboration(n, seed, weighted)


@functools.lru_cache(maxsize=None)
def small_case(weighted):
    L = chung_lu_tc(2500, 7 + weighted, weighted)
    G = L.dense()
    w, V = np.linalg.eigh(G)
    return L, V[:, 1:5]  # four smallest nontrivial eigenvectors (connected graph)


def _tensor(X):
    return torch.tensor(np.ascontiguousarray(X.T), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("weighted", [False, True])
def test_loss_and_gradient_match_the_fp64_reference(weighted):
    L, X = small_case(weighted)
    cfg = mo.Config(layers=2, hidden=16, random_channels=4, out_cols=5)
    net = lap.Mpnn(layers=2, hidden=16, random_channels=4, out_cols=5, seed=3)
    assert net.num_params == cfg.num_params()
    rng = np.random.default_rng(4)
    params = (mo.init_params(cfg, 21) + 0.02 * rng.standard_normal(cfg.num_params())).astype(np.float32)
    net.set_params(params)
    assert np.array_equal(net.get_params(), params)
    plan = lap.Plan(L)
    gr = mo.Graph(L)
    loss_ref, g_ref = mo.loss_and_grad(cfg, params.astype(np.float64), gr, 9, X)
    loss, g = net.loss_grad(plan, _tensor(X), feature_seed=9)
    assert abs(loss - loss_ref) <= 1e-4 * max(loss_ref, 1e-3), (loss, loss_ref)
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert err <= 2e-3, err
    # every weight matrix and bias separately
    at = 0
    for r, c in cfg.shapes():
        for size in (r * c, c):
            seg = slice(at, at + size)
            assert np.linalg.norm(g[seg] - g_ref[seg]) <= 5e-3 * np.linalg.norm(g_ref[seg]) + 1e-7
            at += size
    # the forward output itself
    Yh, _ = mo.forward(cfg, params.astype(np.float64), gr, 9)
    V = net.infer(plan, feature_seed=9).cpu().numpy().T
    assert np.linalg.norm(V - Yh) <= 1e-4 * np.linalg.norm(Yh)


def test_adam_step_matches_the_fp64_reference():
    """k_adam against oracle/mpnn_oracle.adam_step: three consecutive
    training steps, each fed the gradient the GPU computed for the current
    parameters (read back through loss_grad, which leaves the Adam state
    alone), the moments carried on the reference side in FP64."""
    L, X = small_case(False)
    cfg = mo.Config(layers=2, hidden=16, random_channels=4, out_cols=5)
    net = lap.Mpnn(layers=2, hidden=16, random_channels=4, out_cols=5, seed=3)
    plan = lap.Plan(L)
    Xt = _tensor(X)
    lr = 5e-3
    p = net.get_params().astype(np.float64)
    m = np.zeros(cfg.num_params())
    v = np.zeros(cfg.num_params())
    for step in range(1, 4):
        _, g = net.loss_grad(plan, Xt, feature_seed=9)
        net.train_step(plan, Xt, lr=lr, feature_seed=9)
        got = net.get_params().astype(np.float64)
        ref, m, v = mo.adam_step(p, g.astype(np.float64), m, v, step, lr)
        # FP32 update: rounding of w (2^-24 |w|) plus a few ulps of the step (<= lr)
        err = np.abs(got - ref)
        assert np.all(err <= 2e-7 * np.abs(ref) + 2e-6 * lr), (step, float(err.max()),
                                                              float(np.max(err / (np.abs(ref) + lr))))
        assert np.abs(got - p).max() > 0.5 * lr  # the parameters did move
        p = got


def test_save_and_load_round_trip(tmp_path):
    """lap_mpnn_save then lap_mpnn_load: the same configuration, parameters
    bit for bit, the same inferred block, and the same Adam state (one more
    training step on each gives the same parameters)."""
    L, X = small_case(False)
    plan = lap.Plan(L)
    Xt = _tensor(X)
    net = lap.Mpnn(layers=2, hidden=16, random_channels=3, out_cols=5, seed=11)
    for _ in range(3):
        net.train_step(plan, Xt, lr=4e-3, feature_seed=2)
    path = str(tmp_path / "net.lapmpnn")
    net.save(path)
    other = lap.Mpnn.load(path)
    assert (other.cfg.layers, other.cfg.hidden, other.cfg.random_channels, other.cfg.out_cols, other.cfg.seed) == \
        (2, 16, 3, 5, 11)
    assert np.array_equal(other.get_params(), net.get_params())
    assert torch.equal(other.infer(plan, feature_seed=2), net.infer(plan, feature_seed=2))
    net.train_step(plan, Xt, lr=4e-3, feature_seed=2)
    other.train_step(plan, Xt, lr=4e-3, feature_seed=2)
    assert np.array_equal(other.get_params(), net.get_params())
    # the file is what lapeig.h documents: magic, JSON header, 3 x num_params floats
    import json
    with open(path, "rb") as fh:
        assert fh.readline() == b"LAPEIG-MPNN\n"
        hdr = json.loads(fh.readline())
        payload = fh.read()
    assert hdr["format"] == 1 and hdr["num_params"] == net.num_params and hdr["adam_step"] == 3
    assert len(payload) == hdr["payload_bytes"] == 12 * net.num_params
    assert np.array_equal(np.frombuffer(payload[:4 * net.num_params], dtype="<f4"),
                          lap.Mpnn.load(path).get_params())


def test_training_on_the_gpu_lowers_the_loss():
    graphs = [chung_lu_tc(3000, s) for s in (31, 32, 33)]
    plans = [lap.Plan(L) for L in graphs]
    targets = []
    for p in plans:
        r = lap.lap_eigs(p, 7, 1e-6, precision="mixed", evecs_on_device=True)
        targets.append(r.evecs[1:].contiguous())  # (6, n): the nontrivial eigenvectors
    net = lap.Mpnn(layers=2, hidden=32, random_channels=4, out_cols=8, seed=5)
    first = [net.loss_grad(p, X, feature_seed=1, want_grad=False)[0] for p, X in zip(plans, targets)]
    for step in range(150):
        g = step % len(plans)
        net.train_step(plans[g], targets[g], lr=3e-3, feature_seed=1)
    last = [net.loss_grad(p, X, feature_seed=1, want_grad=False)[0] for p, X in zip(plans, targets)]
    print("loss before", np.round(first, 4), "after", np.round(last, 4))
    assert np.mean(last) < 0.9 * np.mean(first)


def test_start_block_changes_iterations_not_the_answer():
    train = [chung_lu_tc(4000, s) for s in (41, 42, 43, 44)]
    plans = [lap.Plan(L) for L in train]
    targets = [lap.lap_eigs(p, 10, 1e-6, evecs_on_device=True).evecs[1:].contiguous() for p in plans]
    net = lap.Mpnn(layers=2, hidden=32, random_channels=4, out_cols=9, seed=6)
    untrained = lap.Mpnn(layers=2, hidden=32, random_channels=4, out_cols=9, seed=6)
    for step in range(200):
        g = step % len(plans)
        net.train_step(plans[g], targets[g], lr=3e-3, feature_seed=2)
    test_graph = chung_lu_tc(8000, 45)
    plan = lap.Plan(test_graph)
    V0 = net.infer(plan, feature_seed=2)
    cold = lap.lap_eigs(plan, 10, 1e-8, precision="mixed")
    warm = lap.lap_eigs(plan, 10, 1e-8, precision="mixed", init=V0)
    print(f"held-out n={test_graph.n}: random start outer {cold.outer} mvp {cold.mvp}; "
          f"network start outer {warm.outer} mvp {warm.mvp}")
    # what training gains on a graph it never saw: the block it proposes
    # holds more of the true eigenspace (subspace loss 1 - ||X'Q||_F^2 / k)
    # than the same network before training
    X = lap.lap_eigs(plan, 10, 1e-8, evecs_on_device=True).evecs[1:].contiguous()
    l_trained = net.loss_grad(plan, X, feature_seed=2, want_grad=False)[0]
    l_untrained = untrained.loss_grad(plan, X, feature_seed=2, want_grad=False)[0]
    print(f"held-out subspace loss: untrained {l_untrained:.4f}, trained {l_trained:.4f}")
    assert l_trained < 0.85 * l_untrained
    assert cold.nconv == warm.nconv == 10
    assert np.allclose(cold.evals, warm.evals, rtol=1e-7, atol=1e-12)
    G = test_graph.to_scipy()
    for r in (cold, warm):
        res = np.linalg.norm(G @ r.evecs - r.evecs * r.evals, axis=0)
        assert np.all(res[1:] <= 1e-8 * np.minimum(r.evals[1:], 1.0) * (1 + 1e-6))


def test_network_argument_errors():
    with pytest.raises(lap.LapError):
        lap.Mpnn(hidden=33)
    with pytest.raises(lap.LapError):
        lap.Mpnn(out_cols=32)
    L, X = small_case(False)
    net = lap.Mpnn(out_cols=30)
    plan = lap.Plan(L)
    with pytest.raises(lap.LapError) as e:
        net.loss_grad(plan, _tensor(X))  # 30 + 4 columns > 32
    assert e.value.code == -1
    disconnected = gg.disjoint_union(gg.path_graph(20), gg.star_graph(9))
    pd = lap.Plan(disconnected)
    net2 = lap.Mpnn(out_cols=3)
    Xd = np.linalg.qr(np.random.default_rng(0).standard_normal((disconnected.n, 2)))[0]
    with pytest.raises(lap.LapError) as e:
        net2.loss_grad(pd, _tensor(Xd))
    assert e.value.code == -6
    V = net2.infer(pd)  # inference works on any graph
    assert V.shape == (3, disconnected.n) and torch.isfinite(V).all()
