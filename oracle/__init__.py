"""Plain FP64 CPU oracle for the Jacobi-Davidson Laplacian eigensolver.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are its only users.  The product library never
imports, links or executes anything here, and the two share no code.

The arithmetic lives in ``lapeig_oracle.c`` (serial C, double precision,
each function citing the passage of the paper it follows); this module only
compiles it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lapeig_oracle.c")
_DEFAULT_LIB = os.path.join(_HERE, "liblapeig_oracle.so")
# an alternative build (used by the tests that plant mistakes in a copy of the source)
_LIB_PATH = os.environ.get("LAPEIG_ORACLE_LIB") or _DEFAULT_LIB
_lib = None

PREC_NONE, PREC_JACOBI, PREC_IC0, PREC_FSAI = 0, 1, 2, 3
FSAI_TAU = 1e-8  # the shift of S = G + tau D in the solvers' FSAI (see lapeig_oracle.c)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no target-specific tuning)."""
    return build_from(_SRC, _DEFAULT_LIB, force)


def build_from(src: str, out: str, force: bool = True) -> str:
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


class _JDOpts(ctypes.Structure):
    _fields_ = [("m_min", ctypes.c_int), ("m_max", ctypes.c_int), ("itmax", ctypes.c_int),
                ("rtol_pcg", ctypes.c_double), ("kmax", ctypes.c_int),
                ("precond", ctypes.c_int), ("criterion", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("fsai_pos", ctypes.POINTER(ctypes.c_int))]


class _DacgOpts(ctypes.Structure):
    _fields_ = [("itmax", ctypes.c_int), ("precond", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("fsai_pos", ctypes.POINTER(ctypes.c_int))]


class _JDInfo(ctypes.Structure):
    _fields_ = [("nconv", ctypes.c_int), ("ncomp", ctypes.c_int), ("outer", ctypes.c_int),
                ("inner", ctypes.c_int), ("nfloor", ctypes.c_int), ("status", ctypes.c_int),
                ("mvp", ctypes.c_longlong)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.environ.get("LAPEIG_ORACLE_LIB") and (
            not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    i32p, f64p = P(ctypes.c_int), P(ctypes.c_double)
    lib.orc_spmv.argtypes = [ctypes.c_int, i32p, i32p, f64p, f64p, f64p]
    lib.orc_quadform.argtypes = [ctypes.c_int, i32p, i32p, f64p, f64p]
    lib.orc_quadform.restype = ctypes.c_double
    lib.orc_components.argtypes = [ctypes.c_int, i32p, i32p, i32p]
    lib.orc_components.restype = ctypes.c_int
    lib.orc_dense_eig.argtypes = [ctypes.c_int, f64p, f64p, f64p]
    lib.orc_dense_eig.restype = ctypes.c_int
    lib.orc_mgs.argtypes = [ctypes.c_int, ctypes.c_int, f64p, f64p]
    lib.orc_mgs.restype = ctypes.c_double
    lib.orc_ic0_create.argtypes = [ctypes.c_int, i32p, i32p, f64p, i32p]
    lib.orc_ic0_create.restype = ctypes.c_void_p
    lib.orc_ic0_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_ic0_apply.argtypes = [ctypes.c_void_p, f64p, f64p]
    lib.orc_pcg_correction.argtypes = [ctypes.c_int, i32p, i32p, f64p, ctypes.c_double,
                                       ctypes.c_int, f64p, f64p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, f64p, i32p]
    lib.orc_pcg_correction.restype = ctypes.c_int
    lib.orc_pcg_correction_ex.argtypes = [ctypes.c_int, i32p, i32p, f64p, ctypes.c_double,
                                          ctypes.c_int, f64p, f64p, ctypes.c_int, i32p, ctypes.c_int,
                                          ctypes.c_double, f64p, i32p]
    lib.orc_pcg_correction_ex.restype = ctypes.c_int
    lib.orc_fsai_create.argtypes = [ctypes.c_int, i32p, i32p, f64p, i32p, ctypes.c_double]
    lib.orc_fsai_create.restype = ctypes.c_void_p
    lib.orc_fsai_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_fsai_nnz.argtypes = [ctypes.c_void_p]
    lib.orc_fsai_nnz.restype = ctypes.c_int
    lib.orc_fsai_export.argtypes = [ctypes.c_void_p, i32p, i32p, f64p]
    lib.orc_fsai_apply.argtypes = [ctypes.c_void_p, f64p, f64p]
    lib.orc_dacg.argtypes = [ctypes.c_int, i32p, i32p, f64p, ctypes.c_int, ctypes.c_double,
                             P(_DacgOpts), f64p, f64p, f64p, P(_JDInfo)]
    lib.orc_dacg.restype = ctypes.c_int
    lib.orc_start_value.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.orc_start_value.restype = ctypes.c_double
    lib.orc_jd.argtypes = [ctypes.c_int, i32p, i32p, f64p, ctypes.c_int, ctypes.c_double,
                           P(_JDOpts), f64p, f64p, f64p, P(_JDInfo)]
    lib.orc_jd.restype = ctypes.c_int
    _lib = lib
    return lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _csr(L):
    rp, rpp = _i32(L.rowptr)
    cl, clp = _i32(L.col)
    vl, vlp = _f64(L.val)
    return (rp, cl, vl), (rpp, clp, vlp)


def spmv(L, x):
    """y = G x (Section 2).  x: (n,) float64."""
    lib = _load()
    keep, (rp, cl, vl) = _csr(L)
    x, xp = _f64(x)
    y = np.empty(L.n, dtype=np.float64)
    lib.orc_spmv(L.n, rp, cl, vl, xp, y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return y


def quadform(L, x):
    """x'Gx by eq. (1)."""
    lib = _load()
    keep, (rp, cl, vl) = _csr(L)
    x, xp = _f64(x)
    return float(lib.orc_quadform(L.n, rp, cl, vl, xp))


def components(L):
    """(ncomp, labels) by breadth-first search."""
    lib = _load()
    keep, (rp, cl, vl) = _csr(L)
    lab = np.empty(L.n, dtype=np.int32)
    nc = lib.orc_components(L.n, rp, cl, lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return int(nc), lab


def dense_eig(A):
    """Cyclic Jacobi on a small dense symmetric matrix: (evals asc, evecs cols)."""
    lib = _load()
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty(n * n)
    sweeps = lib.orc_dense_eig(n, A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if sweeps < 0:
        raise RuntimeError("cyclic Jacobi did not converge")
    return w, V.reshape(n, n).T.copy()


def mgs(Q, v):
    """Modified Gram-Schmidt of v against the orthonormal columns of Q."""
    lib = _load()
    Q = np.asfortranarray(np.asarray(Q, dtype=np.float64).reshape(len(v), -1))
    v = np.array(v, dtype=np.float64, copy=True)
    nrm = lib.orc_mgs(len(v), Q.shape[1], Q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return v, float(nrm)


class IC0:
    """Incomplete Cholesky with no fill-in of G (Section 4)."""

    def __init__(self, L):
        lib = _load()
        self._keep, (rp, cl, vl) = _csr(L)
        nf = ctypes.c_int(0)
        self.n = L.n
        self._h = lib.orc_ic0_create(L.n, rp, cl, vl, ctypes.byref(nf))
        self.nfloor = nf.value

    def apply(self, r):
        lib = _load()
        r, rp = _f64(r)
        z = np.empty(self.n)
        lib.orc_ic0_apply(self._h, rp, z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return z

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_ic0_destroy(self._h)
            self._h = None


class FSAI:
    """Factorized sparse approximate inverse Z of S = G + tau D in a vertex
    order (pos[v] = position of vertex v; None = natural order): P = Z'Z
    (the approximate-inverse preconditioner of the Conclusion)."""

    def __init__(self, L, pos=None, tau=FSAI_TAU):
        lib = _load()
        self._keep, (rp, cl, vl) = _csr(L)
        self.n = L.n
        self._pos = None if pos is None else np.ascontiguousarray(pos, dtype=np.int32)
        pp = None if self._pos is None else self._pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        self._h = lib.orc_fsai_create(L.n, rp, cl, vl, pp, float(tau))

    def matrix(self):
        """Z as a scipy CSR matrix (rows and columns are vertex indices)."""
        import scipy.sparse as sp
        lib = _load()
        nnz = lib.orc_fsai_nnz(self._h)
        rp = np.empty(self.n + 1, dtype=np.int32)
        cl = np.empty(nnz, dtype=np.int32)
        vl = np.empty(nnz)
        lib.orc_fsai_export(self._h, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                            cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                            vl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return sp.csr_matrix((vl, cl, rp), shape=(self.n, self.n))

    def apply(self, r):
        lib = _load()
        r, rp = _f64(r)
        z = np.empty(self.n)
        lib.orc_fsai_apply(self._h, rp, z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return z

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_fsai_destroy(self._h)
            self._h = None


def pcg_correction(L, theta, Q, r, precond=PREC_JACOBI, itmax=20, rtol=1e-2, pos=None):
    """PCG on (I-QQ')(G-theta I)(I-QQ') t = -r (Algorithm 2 step 8).
    pos: the vertex order of FSAI (precond=PREC_FSAI), None = natural.
    Returns (t, mvp, breakdown)."""
    lib = _load()
    keep, (rp, cl, vl) = _csr(L)
    n = L.n
    Q = np.asfortranarray(np.asarray(Q, dtype=np.float64).reshape(n, -1))
    r, rpp = _f64(r)
    t = np.empty(n)
    br = ctypes.c_int(0)
    posa = None if pos is None else np.ascontiguousarray(pos, dtype=np.int32)
    pp = None if posa is None else posa.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    mvp = lib.orc_pcg_correction_ex(n, rp, cl, vl, float(theta), Q.shape[1],
                                    Q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rpp,
                                    int(precond), pp, int(itmax), float(rtol),
                                    t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(br))
    return t, int(mvp), bool(br.value)


def start_value(seed: int, i: int) -> float:
    return float(_load().orc_start_value(ctypes.c_uint64(seed), ctypes.c_uint64(i)))


@dataclass
class JDResult:
    evals: np.ndarray
    evecs: np.ndarray
    res: np.ndarray
    nconv: int
    ncomp: int
    outer: int
    inner: int
    mvp: int
    nfloor: int
    status: int


def jd(L, k, tol, *, m_min=5, m_max=10, itmax=20, rtol_pcg=1e-2, kmax=0,
       precond=PREC_IC0, criterion=0, seed=1, fsai_pos=None) -> JDResult:
    """Algorithm 2 for the k smallest eigenpairs of G (k counts the zero
    pairs).  Paper defaults: m_min 5, m_max 10, ITMAX 20, delta_PCG 1e-2,
    IC(0) preconditioning (Section 4)."""
    lib = _load()
    keep, (rp, cl, vl) = _csr(L)
    n = L.n
    posa = None if fsai_pos is None else np.ascontiguousarray(fsai_pos, dtype=np.int32)
    opts = _JDOpts(m_min, m_max, itmax, rtol_pcg, kmax, precond, criterion, seed,
                   None if posa is None else posa.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    info = _JDInfo()
    ev = np.zeros(k)
    X = np.zeros(n * k)
    res = np.zeros(k)
    st = lib.orc_jd(n, rp, cl, vl, int(k), float(tol), ctypes.byref(opts),
                    ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(info))
    nc = info.nconv
    return JDResult(evals=ev[:nc].copy(), evecs=X.reshape(k, n).T[:, :nc].copy(),
                    res=res[:nc].copy(), nconv=nc, ncomp=info.ncomp, outer=info.outer,
                    inner=info.inner, mvp=int(info.mvp), nfloor=info.nfloor, status=int(st))


def dacg(L, k, tol, *, itmax=0, precond=PREC_IC0, seed=1, fsai_pos=None) -> JDResult:
    """Algorithm 3 (DACG) for the k smallest eigenpairs of G (k counts the
    zero pairs).  outer = pairs computed, inner = nonlinear CG iterations,
    mvp = Laplacian products."""
    lib = _load()
    keep, (rp, cl, vl) = _csr(L)
    n = L.n
    posa = None if fsai_pos is None else np.ascontiguousarray(fsai_pos, dtype=np.int32)
    opts = _DacgOpts(itmax, precond, seed, None if posa is None else posa.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    info = _JDInfo()
    ev = np.zeros(k)
    X = np.zeros(n * k)
    res = np.zeros(k)
    st = lib.orc_dacg(n, rp, cl, vl, int(k), float(tol), ctypes.byref(opts),
                      ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(info))
    nc = info.nconv
    return JDResult(evals=ev[:nc].copy(), evecs=X.reshape(k, n).T[:, :nc].copy(),
                    res=res[:nc].copy(), nconv=nc, ncomp=info.ncomp, outer=info.outer,
                    inner=info.inner, mvp=int(info.mvp), nfloor=info.nfloor, status=int(st))
