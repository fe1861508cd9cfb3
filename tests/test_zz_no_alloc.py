"""lap_spmv_noalloc (the product without device allocation, its scratch in
a fixed device array) against lap_spmv through the C ABI: bit-identical
results on two calls in a row, the second with a smaller input, in both
vertex orders and precisions, with and without shifts; sizes beyond the
fixed scratch are rejected with LAP_EINVAL."""
import ctypes

import numpy as np
import pytest

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


def _noalloc(plan, X, Y, shift=None, plan_order=False):
    lib = lap.load_library()
    f = lib.lap_spmv_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_void_p]
    f.restype = ctypes.c_int
    b = 1 if X.dim() == 1 else int(X.shape[1])
    sh = None
    if shift is not None:
        sh = np.ascontiguousarray(np.broadcast_to(np.asarray(shift, dtype=np.float64), (b,)))
    code = f(plan._h, lap.LAP_F32 if X.dtype == torch.float32 else lap.LAP_F64, b, X.data_ptr(), Y.data_ptr(),
             None if sh is None else sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
             lap.LAP_ORDER_PLAN if plan_order else 0, torch.cuda.current_stream().cuda_stream)
    return code


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_product_matches_lap_spmv_twice(dtype):
    tdt = torch.float32 if dtype == "f32" else torch.float64
    big = lap.Plan(gg.workload("cl330k", 1001))    # hub rows cut into chunks
    small = lap.Plan(gg.workload("pa5k", 1001))
    cases = [(big, 8, [0.5, -1.0, 0.0, 2.0, 3.0, 0.25, 1.0, -0.5], False),
             (small, 3, None, True),
             (big, 1, None, False),
             (small, 1, [1.5], False)]
    for plan, b, shift, plan_order in cases:
        g = torch.Generator(device="cuda").manual_seed(b)
        shape = (plan.n, b) if b > 1 else (plan.n,)
        X = torch.randint(-8, 9, shape, generator=g, device="cuda").to(tdt)
        Y_ref = torch.full_like(X, float("nan"))
        Y = torch.full_like(X, float("nan"))
        lap.lap_spmv(plan, X, Y_ref, shift=shift, plan_order=plan_order)
        assert _noalloc(plan, X, Y, shift, plan_order) == lap.LAP_OK
        torch.cuda.synchronize()
        assert torch.equal(Y, Y_ref), (plan.n, b, shift, plan_order)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    plan = lap.Plan(gg.workload("cl330k", 1001))
    X = torch.zeros((plan.n, 64), dtype=torch.float64, device="cuda")  # 2 x 152 MB > 64 MiB
    Y = torch.zeros_like(X)
    assert _noalloc(plan, X, Y) == lap.LAP_EINVAL
    assert b"scratch" in lap.load_library().lap_last_error()
    # plan order needs no copies: the same block fits
    assert _noalloc(plan, X, Y, plan_order=True) == lap.LAP_OK
    torch.cuda.synchronize()
