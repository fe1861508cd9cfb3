"""Python binding of liblapeig.so, the gfx950 Jacobi-Davidson solver for the
smallest eigenpairs of a graph Laplacian (Bergamaschi, Bozzo & Franceschet,
"Computing the smallest eigenpairs of the graph Laplacian", Algorithm 2).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI of ``include/lapeig.h``.  PyTorch is used for device
memory and streams.  Importing this module never falls back to anything: if
the compiled library is missing, every entry point raises.

Entry points mirror the C ABI names:
  lap_plan_create(L, stream=None, order="hub") -> Plan
  lap_eigs(plan, k, tol, **opts)  -> EigResult
  lap_spmv(plan, X, Y, shift=None, plan_order=False, stream=None)
  lap_orth(Q, W, stream=None)     -> rank
  lap_sym_eig(H, stream=None)     -> (theta, Y, sweeps)
  lap_pcg(plan, theta, Q, R, T, itmax=20, rtol=1e-2, dtype="f32", plan_order=False) -> iters
Column blocks for lap_orth / lap_pcg are torch tensors of shape (b, n): row c
is column c of the n x b column-major block the C ABI expects.  lap_spmv
blocks are (n, b) row-major tensors, or (n,) vectors.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

__all__ = ["LapError", "Plan", "Batch", "EigResult", "lap_plan_create", "lap_eigs", "lap_eigs_csr", "lap_spmv",
           "lap_orth", "lap_sym_eig", "lap_pcg", "lap_batch_create", "lap_batch_eigs", "lap_eigs_batch", "library_path",
           "load_library", "LAP_PREC_FP64", "LAP_PREC_MIXED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblapeig.so")
_lib = None

LAP_OK, LAP_EINVAL, LAP_ENOTLAPLACIAN, LAP_ENOMEM, LAP_EDEVICE, LAP_ENOCONV, LAP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
LAP_F32, LAP_F64 = 0, 1
LAP_PREC_FP64, LAP_PREC_MIXED = 0, 1
LAP_ORDER_PLAN = 1
LAP_PCG_FSAI = 2
LAP_PRECOND_JACOBI, LAP_PRECOND_FSAI = 0, 1
LAP_PLAN_ORDER_HUB, LAP_PLAN_ORDER_CALLER = 0, 1

EXPORTED = ["lap_eigs_default_opts", "lap_plan_create", "lap_plan_create_ex", "lap_plan_destroy", "lap_plan_n", "lap_plan_perm",
            "lap_plan_set_layout", "lap_plan_layout", "lap_plan_autotune",
            "lap_mpnn_create", "lap_mpnn_destroy", "lap_mpnn_num_params", "lap_mpnn_get_params",
            "lap_mpnn_set_params", "lap_mpnn_infer", "lap_mpnn_loss_grad", "lap_mpnn_train_step",
            "lap_mpnn_save", "lap_mpnn_load", "lap_mpnn_get_config", "lap_fiedler_bisect", "lap_pinv_apply",
            "lap_eigs", "lap_eigs_csr", "lap_eigs_dacg", "lap_eigs_irlm", "lap_spmv", "lap_spmv_noalloc", "lap_orth", "lap_sym_eig", "lap_pcg", "lap_batch_create",
            "lap_batch_destroy", "lap_batch_total_n", "lap_batch_autotune", "lap_batch_layout", "lap_batch_eigs", "lap_batch_eigs_ex",
            "lap_eigs_batch", "lap_status_string", "lap_last_error"]


class LapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} [{code}]")
        self.code = code


class _TuneInfo(ctypes.Structure):
    _fields_ = [("long_threshold", ctypes.c_int32), ("huge_threshold", ctypes.c_int32),
                ("best_us", ctypes.c_double), ("default_us", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32)]


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("rowptr", ctypes.POINTER(ctypes.c_int32)),
                ("col", ctypes.POINTER(ctypes.c_int32)), ("val", ctypes.POINTER(ctypes.c_double))]


class _Opts(ctypes.Structure):
    _fields_ = [("m_min", ctypes.c_int), ("m_max", ctypes.c_int), ("itmax", ctypes.c_int),
                ("rtol_pcg", ctypes.c_double), ("kmax", ctypes.c_int), ("precision", ctypes.c_int),
                ("block", ctypes.c_int), ("seed", ctypes.c_uint64), ("init", ctypes.POINTER(ctypes.c_double)),
                ("init_cols", ctypes.c_int), ("init_on_device", ctypes.c_int), ("precond", ctypes.c_int)]


class _MpnnConfig(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int32), ("hidden", ctypes.c_int32), ("random_channels", ctypes.c_int32),
                ("out_cols", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class _Info(ctypes.Structure):
    _fields_ = [("nconv", ctypes.c_int), ("ncomp", ctypes.c_int), ("outer", ctypes.c_int),
                ("inner", ctypes.c_int), ("mvp", ctypes.c_longlong), ("seconds", ctypes.c_double),
                ("warm_start_used", ctypes.c_int)]


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load liblapeig.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise LapError(LAP_EUNSUPPORTED, f"{_LIB_PATH} is missing: build it with "
                                         f"`python -m paper_1311_1695_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    i32p, f64p, ip = P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_int)
    lib.lap_eigs_default_opts.argtypes = [P(_Opts)]
    lib.lap_eigs_default_opts.restype = None
    lib.lap_plan_create.argtypes = [P(_Csr), vp, P(vp)]
    lib.lap_plan_create_ex.argtypes = [P(_Csr), vp, ctypes.c_int, P(vp)]
    lib.lap_plan_destroy.argtypes = [vp]
    lib.lap_plan_destroy.restype = None
    lib.lap_plan_n.argtypes = [vp]
    lib.lap_plan_n.restype = ctypes.c_int32
    lib.lap_plan_perm.argtypes = [vp, i32p]
    lib.lap_plan_set_layout.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    lib.lap_plan_layout.argtypes = [vp, i32p, i32p]
    lib.lap_plan_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int32, ctypes.c_char_p, P(_TuneInfo)]
    lib.lap_eigs.argtypes = [vp, ctypes.c_int, ctypes.c_double, P(_Opts), f64p, vp, ctypes.c_int, f64p, P(_Info)]
    lib.lap_eigs_csr.argtypes = [P(_Csr), ctypes.c_int, ctypes.c_double, P(_Opts), f64p, f64p, f64p, P(_Info)]
    lib.lap_eigs_dacg.argtypes = [vp, ctypes.c_int, ctypes.c_double, P(_Opts), f64p, vp, ctypes.c_int, f64p,
                                  P(_Info)]
    lib.lap_eigs_irlm.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                  P(_Opts), f64p, vp, ctypes.c_int, f64p, P(_Info)]
    lib.lap_spmv.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, f64p, ctypes.c_int, vp]
    lib.lap_spmv_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, f64p, ctypes.c_int, vp]
    lib.lap_orth.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, vp, ip, vp]
    lib.lap_sym_eig.argtypes = [ctypes.c_int, vp, vp, vp, ip, vp]
    lib.lap_pcg.argtypes = [vp, ctypes.c_int, ctypes.c_int, f64p, vp, ctypes.c_int, vp, vp, ctypes.c_int,
                            ctypes.c_double, ip, ctypes.c_int, vp]
    lib.lap_batch_create.argtypes = [P(_Csr), ctypes.c_int, P(vp)]
    lib.lap_batch_destroy.argtypes = [vp]
    lib.lap_batch_destroy.restype = None
    lib.lap_batch_total_n.argtypes = [vp]
    lib.lap_batch_autotune.argtypes = [vp, ctypes.c_int, i32p, f64p]
    lib.lap_batch_layout.argtypes = [vp, ctypes.c_int, i32p, i32p]
    lib.lap_batch_total_n.restype = ctypes.c_int32
    lib.lap_batch_eigs.argtypes = [vp, ctypes.c_int, ctypes.c_double, P(_Opts), f64p, f64p, f64p, P(_Info), vp]
    lib.lap_batch_eigs_ex.argtypes = [vp, ctypes.c_int, ctypes.c_double, P(_Opts), f64p, vp, ctypes.c_int, f64p,
                                      P(_Info), vp]
    lib.lap_eigs_batch.argtypes = [P(_Csr), ctypes.c_int, ctypes.c_int, ctypes.c_double, P(_Opts), f64p, f64p,
                                   f64p, P(_Info), vp]
    lib.lap_mpnn_create.argtypes = [P(_MpnnConfig), P(vp)]
    lib.lap_mpnn_destroy.argtypes = [vp]
    lib.lap_mpnn_destroy.restype = None
    lib.lap_mpnn_num_params.argtypes = [vp]
    lib.lap_mpnn_num_params.restype = ctypes.c_int64
    f32p = P(ctypes.c_float)
    lib.lap_mpnn_get_params.argtypes = [vp, f32p]
    lib.lap_mpnn_set_params.argtypes = [vp, f32p]
    lib.lap_mpnn_infer.argtypes = [vp, vp, ctypes.c_uint64, vp, vp]
    lib.lap_mpnn_loss_grad.argtypes = [vp, vp, ctypes.c_uint64, vp, ctypes.c_int, f64p, f32p, vp]
    lib.lap_mpnn_train_step.argtypes = [vp, vp, ctypes.c_uint64, vp, ctypes.c_int, ctypes.c_float, f64p, vp]
    lib.lap_mpnn_save.argtypes = [vp, ctypes.c_char_p]
    lib.lap_mpnn_load.argtypes = [ctypes.c_char_p, P(vp)]
    lib.lap_mpnn_get_config.argtypes = [vp, P(_MpnnConfig)]
    lib.lap_fiedler_bisect.argtypes = [vp, vp, ctypes.c_int, vp, f64p, vp]
    lib.lap_pinv_apply.argtypes = [ctypes.c_int, ctypes.c_int, f64p, vp, ctypes.c_double, ctypes.c_int, vp, vp, vp]
    lib.lap_status_string.argtypes = [ctypes.c_int]
    lib.lap_status_string.restype = ctypes.c_char_p
    lib.lap_last_error.argtypes = []
    lib.lap_last_error.restype = ctypes.c_char_p
    for name in ["lap_plan_create", "lap_plan_create_ex", "lap_plan_perm", "lap_eigs", "lap_eigs_csr", "lap_spmv", "lap_orth", "lap_sym_eig",
                 "lap_pcg", "lap_batch_create", "lap_batch_eigs", "lap_batch_eigs_ex", "lap_eigs_batch", "lap_spmv_noalloc", "lap_mpnn_save", "lap_mpnn_load", "lap_mpnn_get_config",
                 "lap_fiedler_bisect", "lap_pinv_apply", "lap_eigs_dacg", "lap_eigs_irlm", "lap_batch_autotune",
                 "lap_batch_layout"]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code):
    if code != LAP_OK:
        lib = load_library()
        raise LapError(code, lib.lap_last_error().decode() or lib.lap_status_string(code).decode())


def _stream_handle(stream):
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _csr_struct(L):
    rp = np.ascontiguousarray(L.rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(L.col, dtype=np.int32)
    vl = np.ascontiguousarray(L.val, dtype=np.float64)
    s = _Csr(int(L.n), int(rp[-1]) if len(rp) else 0, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
             cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), vl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return s, (rp, cl, vl)


class Plan:
    """A validated Laplacian resident on the current HIP device."""

    def __init__(self, L, stream=None, order="hub"):
        """order: "hub" (lap_plan_create) or "caller" (lap_plan_create_ex with
        LAP_PLAN_ORDER_CALLER: inside a degree, the caller's vertex order)."""
        lib = load_library()
        if order not in ("hub", "caller"):
            raise LapError(LAP_EINVAL, "order must be 'hub' or 'caller'")
        self._csr, self._keep = _csr_struct(L)
        h = ctypes.c_void_p()
        if order == "hub":
            _check(lib.lap_plan_create(ctypes.byref(self._csr), _stream_handle(stream), ctypes.byref(h)))
        else:
            _check(lib.lap_plan_create_ex(ctypes.byref(self._csr), _stream_handle(stream), LAP_PLAN_ORDER_CALLER,
                                          ctypes.byref(h)))
        self._h = h
        self.n = int(lib.lap_plan_n(h))

    def perm(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        _check(load_library().lap_plan_perm(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def layout(self):
        """(long_threshold, huge_threshold) of the product's row classes."""
        lt, ht = ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().lap_plan_layout(self._h, ctypes.byref(lt), ctypes.byref(ht)))
        return int(lt.value), int(ht.value)

    def set_layout(self, long_threshold, huge_threshold):
        _check(load_library().lap_plan_set_layout(self._h, int(long_threshold), int(huge_threshold)))

    def autotune(self, dtype="f32", b=1, cache_path=None, target="product") -> dict:
        """Time a kernel ("product": the Laplacian product; "pcg": one
        projected-PCG iteration of lap_eigs) for a grid of row-class
        thresholds, keep the fastest; see lap_plan_autotune."""
        info = _TuneInfo()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(load_library().lap_plan_autotune(self._h, {"product": 0, "pcg": 1}[target],
                                                {"f32": LAP_F32, "f64": LAP_F64}[dtype], int(b), path,
                                                ctypes.byref(info)))
        return {"long_threshold": info.long_threshold, "huge_threshold": info.huge_threshold,
                "best_us": info.best_us, "default_us": info.default_us, "candidates": info.candidates,
                "from_cache": bool(info.from_cache)}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().lap_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lap_plan_create(L, stream=None, order="hub") -> Plan:
    return Plan(L, stream, order=order)


def lap_plan_set_layout(plan: Plan, long_threshold, huge_threshold):
    plan.set_layout(long_threshold, huge_threshold)


def lap_plan_layout(plan: Plan):
    return plan.layout()


def lap_plan_autotune(plan: Plan, dtype="f32", b=1, cache_path=None, target="product") -> dict:
    return plan.autotune(dtype, b, cache_path, target)


@dataclasses.dataclass
class EigResult:
    evals: np.ndarray
    evecs: object          # numpy (n, k) or torch tensor (k, n) when on the device
    res: np.ndarray
    nconv: int
    ncomp: int
    outer: int
    inner: int
    mvp: int
    seconds: float
    status: int
    warm_start_used: int = 0


def _precision_code(precision):
    if isinstance(precision, str):
        if precision not in ("mixed", "fp64"):
            raise LapError(LAP_EINVAL, "precision must be 'mixed' or 'fp64'")
        return LAP_PREC_MIXED if precision == "mixed" else LAP_PREC_FP64
    return int(precision)


def _opts(precision="mixed", m_min=5, m_max=10, itmax=20, rtol_pcg=1e-2, kmax=0, block=1, seed=1, init=None,
          precond="jacobi"):
    lib = load_library()
    o = _Opts()
    lib.lap_eigs_default_opts(ctypes.byref(o))
    o.m_min, o.m_max, o.itmax, o.rtol_pcg, o.kmax = m_min, m_max, itmax, rtol_pcg, kmax
    o.precision = {"mixed": LAP_PREC_MIXED, "fp64": LAP_PREC_FP64}[precision] if isinstance(precision, str) else int(precision)
    o.block, o.seed = block, seed
    o.precond = {"jacobi": LAP_PRECOND_JACOBI, "fsai": LAP_PRECOND_FSAI}[precond] if isinstance(precond, str) \
        else int(precond)
    keep = None
    if init is not None and hasattr(init, "data_ptr"):
        # a torch tensor on the device, (p, n) row-major = n x p column-major
        keep = init
        o.init = ctypes.cast(ctypes.c_void_p(init.data_ptr()), ctypes.POINTER(ctypes.c_double))
        o.init_cols = int(init.shape[0]) if init.dim() == 2 else 1
        o.init_on_device = 1
    elif init is not None:
        keep = np.asfortranarray(np.asarray(init, dtype=np.float64))
        if keep.ndim == 1:
            keep = keep[:, None]
        o.init = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.init_cols = keep.shape[1]
    return o, keep


def lap_eigs(plan: Plan, k: int, tol: float, *, evecs_on_device=False, allow_noconv=False, _fn="lap_eigs",
             _pre=(), **kw) -> EigResult:
    """The k smallest eigenpairs (k counts the zero eigenvalues).  Keyword
    options: precision ('mixed' | 'fp64'), m_min, m_max, itmax, rtol_pcg,
    kmax, block, seed, init (n x p numpy start block, or a (p, n) float64
    device tensor such as Mpnn.infer returns), precond ('jacobi' | 'fsai')."""
    lib = load_library()
    o, keep = _opts(**kw)
    n = plan.n
    ev = np.zeros(k)
    res = np.zeros(k)
    info = _Info()
    if evecs_on_device:
        import torch
        X = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        xp = ctypes.c_void_p(X.data_ptr())
    else:
        X = np.zeros((k, n))
        xp = ctypes.c_void_p(X.ctypes.data)
    code = getattr(lib, _fn)(plan._h, int(k), float(tol), *_pre, ctypes.byref(o),
                        ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), xp, int(bool(evecs_on_device)),
                        res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(info))
    if code != LAP_OK and not (allow_noconv and code == LAP_ENOCONV):
        _check(code)
    nc = info.nconv
    vec = X[:nc] if evecs_on_device else X[:nc].T.copy()
    return EigResult(ev[:nc].copy(), vec, res[:nc].copy(), nc, info.ncomp, info.outer, info.inner,
                     int(info.mvp), info.seconds, code, info.warm_start_used)


def lap_eigs_dacg(plan: Plan, k: int, tol: float, **kw) -> EigResult:
    """The k smallest eigenpairs by DACG (Algorithm 3); options as lap_eigs
    (kmax: iterations per pair; seed; precond 'jacobi').  outer = pairs
    computed by DACG, inner = its iterations."""
    return lap_eigs(plan, k, tol, _fn="lap_eigs_dacg", **kw)


def lap_eigs_irlm(plan: Plan, k: int, tol: float, *, m=0, rtol_inner=0.0, itmax_inner=0, **kw) -> EigResult:
    """The k smallest eigenpairs by IRLM on G^+ with PCG inner solves
    (Algorithm 1 right); m Krylov size, rtol_inner / itmax_inner of the inner
    PCG (0: defaults), options as lap_eigs (seed, precond, kmax = restart
    limit).  outer = Lanczos steps, inner = PCG iterations."""
    return lap_eigs(plan, k, tol, _fn="lap_eigs_irlm",
                    _pre=(ctypes.c_int(int(m)), ctypes.c_double(float(rtol_inner)), ctypes.c_int(int(itmax_inner))),
                    **kw)


def lap_eigs_csr(L, k, tol, **kw) -> EigResult:
    plan = Plan(L)
    try:
        return lap_eigs(plan, k, tol, **kw)
    finally:
        plan.close()


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return LAP_F32
    if t.dtype == torch.float64:
        return LAP_F64
    raise LapError(LAP_EINVAL, f"unsupported dtype {t.dtype}")


def lap_spmv(plan: Plan, X, Y, shift=None, plan_order=False, stream=None):
    """Y = G X - X diag(shift) on the device; X, Y: (n,) or (n, b) row-major."""
    lib = load_library()
    if X.dtype != Y.dtype or X.shape != Y.shape or not X.is_contiguous() or not Y.is_contiguous():
        raise LapError(LAP_EINVAL, "X and Y must be contiguous tensors of one shape and dtype")
    b = 1 if X.dim() == 1 else int(X.shape[1])
    sh = None
    if shift is not None:
        sh = np.ascontiguousarray(np.broadcast_to(np.asarray(shift, dtype=np.float64), (b,)))
    _check(lib.lap_spmv(plan._h, _dtype_code(X), b, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                        None if sh is None else sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        LAP_ORDER_PLAN if plan_order else 0, _stream_handle(stream)))


def lap_spmv_noalloc(plan: Plan, X, Y, shift=None, plan_order=False, stream=None):
    """lap_spmv without device allocation (its scratch is a fixed device
    array of the library); same arguments and results."""
    lib = load_library()
    if X.dtype != Y.dtype or X.shape != Y.shape or not X.is_contiguous() or not Y.is_contiguous():
        raise LapError(LAP_EINVAL, "X and Y must be contiguous tensors of one shape and dtype")
    b = 1 if X.dim() == 1 else int(X.shape[1])
    sh = None
    if shift is not None:
        sh = np.ascontiguousarray(np.broadcast_to(np.asarray(shift, dtype=np.float64), (b,)))
    _check(lib.lap_spmv_noalloc(plan._h, _dtype_code(X), b, ctypes.c_void_p(X.data_ptr()),
                                ctypes.c_void_p(Y.data_ptr()),
                                None if sh is None else sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                LAP_ORDER_PLAN if plan_order else 0, _stream_handle(stream)))


def lap_orth(Q, W, stream=None) -> int:
    """W <- orthonormal basis of (I - QQ')W (double precision).  Q: (q, n)
    rows are orthonormal columns; W: (b, n), in place.  Returns the rank."""
    lib = load_library()
    import torch
    if W.dtype != torch.float64 or not W.is_contiguous():
        raise LapError(LAP_EINVAL, "W must be a contiguous float64 tensor of shape (b, n)")
    b, n = int(W.shape[0]), int(W.shape[1])
    q = 0 if Q is None else int(Q.shape[0])
    qp = ctypes.c_void_p(Q.data_ptr()) if q else ctypes.c_void_p(0)
    rank = ctypes.c_int(0)
    _check(lib.lap_orth(LAP_F64, n, q, qp, b, ctypes.c_void_p(W.data_ptr()), ctypes.byref(rank),
                        _stream_handle(stream)))
    return rank.value


def lap_sym_eig(H, stream=None):
    """All eigenpairs of a small symmetric matrix (the Rayleigh-Ritz step).
    H: (m, m) float64 device tensor, symmetric.  Returns (theta, Y, sweeps):
    theta (m,) ascending and Y (m, m) with column j the eigenvector of
    theta[j], both float64 device tensors, and -1 when the secular-equation
    path solved H, else the number of Jacobi sweeps."""
    lib = load_library()
    import torch
    if H.dtype != torch.float64 or H.dim() != 2 or H.shape[0] != H.shape[1] or not H.is_cuda:
        raise LapError(LAP_EINVAL, "H must be a square float64 device tensor")
    m = int(H.shape[0])
    Hc = H.t().contiguous()  # column-major
    theta = torch.empty(m, dtype=torch.float64, device=H.device)
    Yc = torch.empty((m, m), dtype=torch.float64, device=H.device)  # row j = column j of Y
    sw = ctypes.c_int(0)
    _check(lib.lap_sym_eig(m, ctypes.c_void_p(Hc.data_ptr()), ctypes.c_void_p(theta.data_ptr()),
                           ctypes.c_void_p(Yc.data_ptr()), ctypes.byref(sw), _stream_handle(stream)))
    return theta, Yc.t(), sw.value


def lap_pcg(plan: Plan, theta, Q, R, T, itmax=20, rtol=1e-2, dtype="f32", plan_order=False, stream=None,
            precond="jacobi"):
    """PCG on the projected correction equations; Q: (q, n), R and T: (b, n)
    float64 device tensors; precond 'jacobi' (D^-1) or 'fsai'.  Returns the
    iterations per column."""
    lib = load_library()
    b = int(R.shape[0])
    th = np.ascontiguousarray(np.broadcast_to(np.asarray(theta, dtype=np.float64), (b,)))
    q = 0 if Q is None else int(Q.shape[0])
    its = np.zeros(b, dtype=np.int32)
    _check(lib.lap_pcg(plan._h, {"f32": LAP_F32, "f64": LAP_F64}[dtype], b,
                       th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       ctypes.c_void_p(Q.data_ptr()) if q else ctypes.c_void_p(0), q,
                       ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(T.data_ptr()), int(itmax), float(rtol),
                       its.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                       (LAP_ORDER_PLAN if plan_order else 0) | (LAP_PCG_FSAI if precond == "fsai" else 0),
                       _stream_handle(stream)))
    return its


def lap_fiedler_bisect(plan: Plan, fiedler, n1: int, stream=None):
    """Spectral bisection: (part, cut) with part an int32 device tensor (0 for
    the n1 vertices of smallest Fiedler entry, ties by index) and cut the
    weight of the edges between the sides.  fiedler: float64 device tensor
    of n entries, caller order."""
    import torch
    if fiedler.dtype != torch.float64 or fiedler.numel() != plan.n or not fiedler.is_contiguous():
        raise LapError(LAP_EINVAL, "fiedler must be a contiguous float64 device tensor of n entries")
    part = torch.empty(plan.n, dtype=torch.int32, device=fiedler.device)
    cut = ctypes.c_double(0.0)
    _check(load_library().lap_fiedler_bisect(plan._h, ctypes.c_void_p(fiedler.data_ptr()), int(n1),
                                             ctypes.c_void_p(part.data_ptr()), ctypes.byref(cut),
                                             _stream_handle(stream)))
    return part, cut.value


def lap_pinv_apply(evals, evecs, X, sigma=0.0, stream=None):
    """Y = T^(k) X (sigma = 0) or S^(k) X (sigma > 0).  evals: k host values;
    evecs: (k, n) float64 device tensor (row j = eigenvector j); X: (b, n)
    float64 device tensor.  Returns Y like X."""
    import torch
    ev = np.ascontiguousarray(np.asarray(evals, dtype=np.float64))
    k, n = int(evecs.shape[0]), int(evecs.shape[1])
    if X.dim() == 1:
        X = X[None, :]
    if not (evecs.is_contiguous() and X.is_contiguous()) or X.shape[1] != n or ev.size != k:
        raise LapError(LAP_EINVAL, "evecs (k, n), X (b, n) contiguous float64, k eigenvalues")
    Y = torch.empty_like(X)
    _check(load_library().lap_pinv_apply(n, k, ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         ctypes.c_void_p(evecs.data_ptr()), float(sigma), int(X.shape[0]),
                                         ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                         _stream_handle(stream)))
    return Y


class Batch:
    """Many connected graphs resident on the device for lap_batch_eigs."""

    def __init__(self, graphs):
        lib = load_library()
        self._keep = []
        arr = (_Csr * len(graphs))()
        for g, L in enumerate(graphs):
            st, keep = _csr_struct(L)
            arr[g] = st
            self._keep.append(keep)
        self._arr = arr
        self.ns = [int(L.n) for L in graphs]
        h = ctypes.c_void_p()
        _check(lib.lap_batch_create(arr, len(graphs), ctypes.byref(h)))
        self._h = h

    def autotune(self, precision="mixed"):
        """Time the row-class thresholds of the batched product in that
        precision and keep the fastest; returns (threshold, seconds per pass)."""
        thr, secs = ctypes.c_int32(0), ctypes.c_double(0.0)
        _check(load_library().lap_batch_autotune(self._h, _precision_code(precision), ctypes.byref(thr),
                                                  ctypes.byref(secs)))
        return int(thr.value), float(secs.value)

    def layout(self, precision="mixed"):
        """(threshold in use, tuned) for that precision."""
        thr, tuned = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(load_library().lap_batch_layout(self._h, _precision_code(precision), ctypes.byref(thr),
                                                ctypes.byref(tuned)))
        return int(thr.value), bool(tuned.value)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().lap_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lap_batch_create(graphs) -> Batch:
    return Batch(graphs)


def lap_batch_eigs(batch: Batch, k: int, tol: float, *, evecs_on_device=False, allow_noconv=False, stream=None,
                   **kw):
    """The k smallest pairs of every graph of the batch; returns a list of
    EigResult (evecs as numpy n x k arrays in each graph's vertex order, or,
    with evecs_on_device, (k, n) float64 views of one device tensor)."""
    lib = load_library()
    o, keep = _opts(**kw)
    nb = len(batch.ns)
    ev = np.zeros(nb * k)
    res = np.zeros(nb * k)
    total = k * sum(batch.ns)
    if evecs_on_device:
        import torch
        X = torch.zeros(total, dtype=torch.float64, device="cuda")
        xp = ctypes.c_void_p(X.data_ptr())
    else:
        X = np.zeros(total)
        xp = ctypes.c_void_p(X.ctypes.data)
    infos = (_Info * nb)()
    code = lib.lap_batch_eigs_ex(batch._h, int(k), float(tol), ctypes.byref(o),
                                 ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), xp, int(bool(evecs_on_device)),
                                 res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), infos, _stream_handle(stream))
    if code != LAP_OK and not (allow_noconv and code == LAP_ENOCONV):
        _check(code)
    out, off = [], 0
    for g, n in enumerate(batch.ns):
        inf = infos[g]
        nc = inf.nconv
        if evecs_on_device:
            vec = X[off:off + n * k].view(k, n)[:nc]
        else:
            vec = X[off:off + n * k].reshape(k, n).T[:, :nc].copy()
        out.append(EigResult(ev[g * k:g * k + nc].copy(), vec, res[g * k:g * k + nc].copy(), nc,
                             inf.ncomp, inf.outer, inf.inner, int(inf.mvp), inf.seconds, code))
        off += n * k
    return out


def lap_eigs_batch(graphs, k, tol, **kw):
    b = Batch(graphs)
    try:
        return lap_batch_eigs(b, k, tol, **kw)
    finally:
        b.close()


class Mpnn:
    """The warm-start network of lap_mpnn_* on the current device (all of its
    arithmetic in the library's kernels).  X and the inferred start block
    are float64 device tensors of shape (columns, n), i.e. n x columns
    column-major, in the caller's vertex order."""

    def __init__(self, layers=2, hidden=32, random_channels=4, out_cols=9, seed=1):
        lib = load_library()
        self.cfg = _MpnnConfig(int(layers), int(hidden), int(random_channels), int(out_cols), int(seed))
        h = ctypes.c_void_p()
        _check(lib.lap_mpnn_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h
        self.num_params = int(lib.lap_mpnn_num_params(h))

    @property
    def out_cols(self) -> int:
        return int(self.cfg.out_cols)

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        _check(load_library().lap_mpnn_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_params(self, params):
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        assert a.size == self.num_params
        _check(load_library().lap_mpnn_set_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def infer(self, plan: Plan, feature_seed=1, stream=None):
        import torch
        V = torch.empty((self.out_cols, plan.n), dtype=torch.float64, device="cuda")
        _check(load_library().lap_mpnn_infer(self._h, plan._h, int(feature_seed), ctypes.c_void_p(V.data_ptr()),
                                             _stream_handle(stream)))
        return V

    def loss_grad(self, plan: Plan, X, feature_seed=1, stream=None, want_grad=True):
        loss = ctypes.c_double()
        g = np.empty(self.num_params, dtype=np.float32) if want_grad else None
        _check(load_library().lap_mpnn_loss_grad(
            self._h, plan._h, int(feature_seed), ctypes.c_void_p(X.data_ptr()), int(X.shape[0]),
            ctypes.byref(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if want_grad else None,
            _stream_handle(stream)))
        return loss.value, g

    def train_step(self, plan: Plan, X, lr=1e-2, feature_seed=1, stream=None) -> float:
        loss = ctypes.c_double()
        _check(load_library().lap_mpnn_train_step(self._h, plan._h, int(feature_seed), ctypes.c_void_p(X.data_ptr()),
                                                  int(X.shape[0]), float(lr), ctypes.byref(loss),
                                                  _stream_handle(stream)))
        return loss.value

    def save(self, path):
        """Write the parameters and the Adam state to `path` (lap_mpnn_save)."""
        _check(load_library().lap_mpnn_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        """A network created from a file written by save (lap_mpnn_load)."""
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.lap_mpnn_load(os.fsencode(path), ctypes.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self.num_params = int(lib.lap_mpnn_num_params(h))
        self.cfg = _MpnnConfig()
        _check(lib.lap_mpnn_get_config(h, ctypes.byref(self.cfg)))
        return self

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().lap_mpnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lap_mpnn_create(**cfg) -> Mpnn:
    return Mpnn(**cfg)
