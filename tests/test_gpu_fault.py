"""The failure paths of lap_eigs forced from the host (LAPEIG_FAULT, read at
each solve): a start block whose first column turns non-finite on the
device is partly dropped and the seeded start fills in (warm_start_used
counts the columns kept), and correction equations whose projected operator
is negative definite stop at the PCG's first iteration with M(-r) (the
breakdown branch of Algorithm 2 step 8) while the outer iteration still
certifies every pair.  Values against dense eigh at relative 1e-8,
residuals recomputed on the host.  Every kernel runs normally: the hooks
only change the data (a NaN entry, the shift) that the host hands over."""
import numpy as np
import pytest

import paper_1311_1695_amd as lap
from paper_1311_1695_amd import graphgen as gg
from tests._lapcheck import residuals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lap.load_library()
    yield


def _graph():
    u, v = gg.pa_edges(1500, 3, 77)
    return gg.laplacian_from_edges(1500, u, v, name="pa1500")


def _certified(L, r, k, tol=1e-8):
    assert r.nconv == k
    rr = residuals(L.to_scipy(), r.evals, r.evecs)
    bound = tol * np.maximum(np.minimum(r.evals, 1.0), (r.evals <= 0) * 1.0)
    assert np.all(rr <= bound * (1 + 1e-6) + 1e-14)
    w = np.linalg.eigvalsh(L.dense())[:k]
    assert np.allclose(r.evals, w, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("block", [1, 4])
def test_fault_nan_init_drops_the_column(monkeypatch, block):
    L = _graph()
    k = 6
    init = np.random.default_rng(5).standard_normal((L.n, 4))
    kw = dict(precision="mixed", seed=1, init=init)
    if block > 1:
        kw.update(block=block, m_min=8, m_max=20)
    plan = lap.Plan(L)
    clean = lap.lap_eigs(plan, k, 1e-8, **kw)
    _certified(L, clean, k)
    assert clean.warm_start_used == 4
    monkeypatch.setenv("LAPEIG_FAULT", "nan_init")
    r = lap.lap_eigs(plan, k, 1e-8, **kw)
    _certified(L, r, k)
    assert r.warm_start_used == 3
    plan.close()


@pytest.mark.parametrize("block", [1, 4])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_fault_pcg_breakdown_still_certifies(monkeypatch, block, precision):
    L = _graph()
    k = 5
    kw = dict(precision=precision, seed=1)
    if block > 1:
        kw.update(block=block, m_min=8, m_max=20)
    plan = lap.Plan(L)
    clean = lap.lap_eigs(plan, k, 1e-8, **kw)
    _certified(L, clean, k)
    monkeypatch.setenv("LAPEIG_FAULT", "nan_init,pcg_breakdown")
    r = lap.lap_eigs(plan, k, 1e-8, **kw)
    _certified(L, r, k)
    # every correction equation stopped at its first iteration
    assert r.inner <= r.outer * block
    assert clean.inner > clean.outer
    print(f"block {block} {precision}: outer {clean.outer} -> {r.outer}, inner {clean.inner} -> {r.inner}")
    plan.close()
