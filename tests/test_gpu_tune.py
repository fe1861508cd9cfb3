"""GPU tests of the row-class layouts and their autotuner (lap_plan_set_layout,
lap_plan_autotune): whatever thresholds are chosen, the product on integer
vectors stays equal bit for bit to the oracle's (every partial sum exact),
and the eigensolver's answer stays within the parity bar."""
import functools
import json

import numpy as np
import pytest

import oracle
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


@functools.lru_cache(maxsize=None)
def graph(name):
    if name == "star9000":
        return gg.star_graph(9000)
    return gg.workload(name, 1001)


def _spmv_exact(plan, L, dtype="f32", b=1, seed=11):
    rng = np.random.default_rng(seed)
    lim = 64 if dtype == "f32" else 1 << 20
    tdt = torch.float32 if dtype == "f32" else torch.float64
    if b == 1:
        x = rng.integers(-lim, lim, size=L.n).astype(np.float64)
        ref = oracle.spmv(L, x)
        X = torch.tensor(x, dtype=tdt, device="cuda")
    else:
        x = rng.integers(-lim, lim, size=(L.n, b)).astype(np.float64)
        ref = np.stack([oracle.spmv(L, x[:, c]) for c in range(b)], axis=1)
        X = torch.tensor(x, dtype=tdt, device="cuda")
    Y = torch.empty_like(X)
    lap.lap_spmv(plan, X, Y)
    torch.cuda.synchronize()
    got = Y.double().cpu().numpy()
    assert np.array_equal(got, ref), f"max diff {np.abs(got - ref).max()}"


@pytest.mark.parametrize("name", ["cl30k", "cl30k_w", "star9000"])
@pytest.mark.parametrize("lt,ht", [(1, 1), (1, 1 << 30), (1 << 30, 1 << 30), (8, 128), (64, 2048), (32, 512)])
def test_every_layout_keeps_the_product_exact(name, lt, ht):
    L = graph(name)
    plan = lap.Plan(L)
    assert plan.layout() == (32, 512)
    plan.set_layout(lt, ht)
    assert plan.layout() == (lt, ht)
    _spmv_exact(plan, L, "f32")
    _spmv_exact(plan, L, "f64")
    _spmv_exact(plan, L, "f32", b=5)


def test_set_layout_rejects_bad_thresholds():
    plan = lap.Plan(graph("cl30k"))
    for lt, ht in [(0, 10), (20, 10), (-1, -1)]:
        with pytest.raises(lap.LapError) as e:
            plan.set_layout(lt, ht)
        assert e.value.code == -1
    assert plan.layout() == (32, 512)


def test_autotune_chooses_a_timed_layout_and_caches_it(tmp_path):
    L = graph("cl30k")
    cache = tmp_path / "tune.json"
    plan = lap.Plan(L)
    info = plan.autotune("f32", 1, str(cache))
    assert not info["from_cache"] and info["candidates"] >= 2
    assert 0 < info["best_us"] <= info["default_us"] * (1 + 1e-12)
    assert plan.layout() == (info["long_threshold"], info["huge_threshold"])
    _spmv_exact(plan, L, "f32")
    doc = json.loads(cache.read_text())
    assert len(doc["entries"]) == 1
    e = doc["entries"][0]
    assert (e["long"], e["huge"]) == (info["long_threshold"], info["huge_threshold"])
    assert "|product|b1|f32|" in e["key"]
    # a second plan of the same graph takes the cached choice without timing
    plan2 = lap.Plan(L)
    info2 = plan2.autotune("f32", 1, str(cache))
    assert info2["from_cache"] and info2["candidates"] == 0
    assert plan2.layout() == plan.layout()
    # another block width is another entry
    info3 = plan2.autotune("f32", 4, str(cache))
    assert not info3["from_cache"]
    assert len(json.loads(cache.read_text())["entries"]) == 2
    _spmv_exact(plan2, L, "f32", b=4)


def test_eigs_after_retuning_match_the_dense_reference():
    L = graph("pa5k")
    plan = lap.Plan(L)
    k = 6
    ref = np.linalg.eigvalsh(L.dense())[:k]
    for lt, ht in [(8, 128), (1, 1), (1 << 30, 1 << 30)]:
        plan.set_layout(lt, ht)
        for prec in ("mixed", "fp64"):
            r = lap.lap_eigs(plan, k, 1e-8, precision=prec)
            assert r.nconv == k
            assert np.all(np.abs(r.evals - ref) <= 1e-8 * np.maximum(ref, 1e-3)), (lt, ht, prec, r.evals - ref)


@pytest.mark.parametrize("dtype,prec", [("f32", "mixed"), ("f64", "fp64")])
def test_pcg_target_tunes_for_the_inner_solve(dtype, prec, tmp_path):
    L = graph("pa5k")
    plan = lap.Plan(L)
    cache = tmp_path / "t.json"
    info = plan.autotune(dtype, 1, str(cache), target="pcg")
    assert not info["from_cache"] and info["candidates"] >= 2
    assert 0 < info["best_us"] <= info["default_us"] * (1 + 1e-12)
    assert plan.layout() == (info["long_threshold"], info["huge_threshold"])
    assert "|pcg|b1|" + dtype + "|" in json.loads(cache.read_text())["entries"][0]["key"]
    with pytest.raises(lap.LapError):
        plan.autotune(dtype, 4, None, target="pcg")
    k = 6
    ref = np.linalg.eigvalsh(L.dense())[:k]
    r = lap.lap_eigs(plan, k, 1e-8, precision=prec)
    assert r.nconv == k
    assert np.all(np.abs(r.evals - ref) <= 1e-8 * np.maximum(ref, 1e-3))
