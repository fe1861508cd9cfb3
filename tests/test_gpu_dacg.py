"""GPU DACG (lap_eigs_dacg, Algorithm 3) against the oracle's DACG
(oracle.dacg, the same nonlinear CG in plain FP64 C with the same seeded
start vectors and Jacobi preconditioner) and against dense or JD
references: eigenvalues within relative 1e-8, vectors by cluster-aware
subspace angle <= 1e-6, residuals recomputed on the host.  Iteration
counts track the oracle's at tol 1e-6; below that the Rayleigh quotient is
flat to FP64 rounding (its error is the square of the residual), the
conjugate directions are rounding-dominated, and the count of the final
phase depends on the order of floating-point additions (a numpy copy of
the same iteration differs from the C oracle by 17 % on the grid), so at
1e-8 only the certified result is compared."""
import numpy as np
import pytest

import oracle
import paper_1311_1695_amd as lap
from paper_1311_1695_amd import graphgen as gg
from tests._lapcheck import check_against_reference, residuals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lap.load_library()
    yield


CASES = {
    "grid20x30": (lambda: gg.grid_graph(20, 30), 6),
    "path200": (lambda: gg.path_graph(200), 5),
    "union": (lambda: gg.disjoint_union(gg.grid_graph(10, 12), gg.path_graph(30)), 5),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_dacg_matches_oracle_dacg(name):
    make, k = CASES[name]
    L = make()
    plan = lap.Plan(L)
    r = lap.lap_eigs_dacg(plan, k, 1e-8, kmax=40000)
    ref = oracle.dacg(L, k, 1e-8, precond=oracle.PREC_JACOBI, itmax=40000)
    assert r.nconv == k and ref.nconv == k
    assert np.allclose(r.evals, ref.evals, rtol=1e-8, atol=1e-13)
    rr = residuals(L.to_scipy(), r.evals, r.evecs)
    bound = 1e-8 * np.maximum(np.minimum(r.evals, 1.0), (r.evals <= 0) * 1.0)
    assert np.all(rr <= bound * (1 + 1e-6) + 1e-14)
    assert np.abs(r.evecs.T @ r.evecs - np.eye(k)).max() <= 1e-8
    w, V = np.linalg.eigh(L.dense())
    check_against_reference(r.evals, r.evecs, w, V, val_rtol=1e-8, angle_tol=1e-6)
    print(f"{name}: DACG iterations GPU {r.inner}, oracle {ref.inner}; products {r.mvp}")


def test_dacg_power_law_graph_at_1e6():
    """The Chung-Lu graph of 24k vertices, 3 pairs at the paper's tolerance
    1e-6 (DACG's final phase at 1e-8 is rounding-dominated there): values
    against the oracle's JD at 1e-10 (the quadratic bound (1e-6 lambda)^2 /
    gap keeps them within relative 1e-8), vectors within the Davis-Kahan
    bound of their residuals."""
    L = gg.workload("cl30k", 1001)
    plan = lap.Plan(L)
    r = lap.lap_eigs_dacg(plan, 3, 1e-6, kmax=40000)
    assert r.nconv == 3
    j = oracle.jd(L, 6, 1e-10)
    assert np.allclose(r.evals, j.evals[:3], rtol=1e-8, atol=1e-13)
    rr = residuals(L.to_scipy(), r.evals, r.evecs)
    assert np.all(rr[1:] <= 1e-6 * np.minimum(r.evals[1:], 1.0) * (1 + 1e-6))
    for i in (1, 2):
        gap = min(abs(j.evals[i] - j.evals[i - 1]), abs(j.evals[i + 1] - j.evals[i]))
        sin = np.sqrt(max(0.0, 1.0 - float(r.evecs[:, i] @ j.evecs[:, i]) ** 2))
        assert sin <= 2 * rr[i] / gap + 1e-8
    print(f"cl30k at 1e-6: DACG iterations {r.inner}, products {r.mvp}")


@pytest.mark.parametrize("name", ["grid20x30", "path200", "union"])
def test_dacg_iterations_track_oracle_at_1e6(name):
    make, k = CASES[name]
    L = make()
    plan = lap.Plan(L)
    r = lap.lap_eigs_dacg(plan, k, 1e-6, kmax=40000)
    ref = oracle.dacg(L, k, 1e-6, precond=oracle.PREC_JACOBI, itmax=40000)
    assert r.nconv == k and ref.nconv == k
    assert np.allclose(r.evals, ref.evals, rtol=1e-10, atol=1e-13)
    print(f"{name} at 1e-6: DACG iterations GPU {r.inner}, oracle {ref.inner}")
    # identical on the grid and the union; the path's spectrum (lambda_j ~ j^2)
    # is the most clustered, and its count varies by several percent
    assert abs(r.inner - ref.inner) <= (0.15 if name == "path200" else 0.02) * ref.inner + 5


def test_dacg_limits_and_errors():
    L = gg.grid_graph(20, 30)
    plan = lap.Plan(L)
    r = lap.lap_eigs_dacg(plan, 6, 1e-8, kmax=50, allow_noconv=True)
    assert r.status == lap.LAP_ENOCONV and r.nconv == 1  # the zero pair only
    with pytest.raises(lap.LapError) as e:
        lap.lap_eigs_dacg(plan, 3, 1e-8, precond="fsai")
    assert e.value.code == lap.LAP_EUNSUPPORTED
