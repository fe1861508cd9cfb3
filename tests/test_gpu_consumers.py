"""GPU consumers of the eigenpairs (lap_fiedler_bisect, lap_pinv_apply)
against the FP64 reference oracle/consumers.py, fed the same eigenpairs:
the partition bit for bit (ties by index included) and its cut size
exactly (integer weights, so every partial sum is exact), T^(k) X and
S^(k) X to relative 1e-12."""
import functools

import numpy as np
import pytest

from oracle import consumers as cs
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
def solved(name):
    L = gg.disjoint_union(gg.cycle_graph(40), gg.workload("pa5k", 4)) if name == "union" else gg.workload(name, 1001)
    plan = lap.Plan(L)
    r = lap.lap_eigs(plan, 10, 1e-10, precision="fp64")
    return L, plan, r


@pytest.mark.parametrize("name", ["cl30k", "cl30k_w", "pa5k"])
@pytest.mark.parametrize("frac", [0.0, 0.1, 0.5, 1.0])
def test_fiedler_bisection_matches_reference(name, frac):
    L, plan, r = solved(name)
    f = r.evecs[:, 1].copy()
    n1 = int(round(frac * L.n))
    part, cut = lap.lap_fiedler_bisect(plan, torch.tensor(f, device="cuda"), n1)
    ref_part, ref_cut = cs.bisect(L, f, n1)
    assert np.array_equal(part.cpu().numpy(), ref_part)
    assert cut == ref_cut
    if 0 < n1 < L.n:
        assert cut >= n1 * (L.n - n1) * r.evals[1] / L.n * (1 - 1e-9)


def test_fiedler_bisection_ties_go_by_index():
    L, plan, r = solved("cl30k")
    f = np.round(r.evecs[:, 1] * 50.0)  # a few dozen distinct values, many ties
    for n1 in (1, 777, L.n // 2, L.n - 1):
        part, cut = lap.lap_fiedler_bisect(plan, torch.tensor(f, device="cuda"), n1)
        ref_part, ref_cut = cs.bisect(L, f, n1)
        assert np.array_equal(part.cpu().numpy(), ref_part) and cut == ref_cut
    bad = f.copy()
    bad[5] = np.nan
    with pytest.raises(lap.LapError) as e:
        lap.lap_fiedler_bisect(plan, torch.tensor(bad, device="cuda"), 3)
    assert e.value.code == lap.LAP_EINVAL


@pytest.mark.parametrize("name", ["cl30k", "union"])
@pytest.mark.parametrize("sigma", [0.0, 2.5])
def test_pinv_approximations_match_reference(name, sigma):
    L, plan, r = solved(name)
    V = torch.tensor(np.ascontiguousarray(r.evecs.T), device="cuda")
    X = np.random.default_rng(4).standard_normal((3, L.n))
    Y = lap.lap_pinv_apply(r.evals, V, torch.tensor(X, device="cuda"), sigma=sigma).cpu().numpy()
    ref = (cs.pinv_S(r.evals, r.evecs, sigma, X.T) if sigma > 0 else cs.pinv_T(r.evals, r.evecs, X.T)).T
    assert np.allclose(Y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
