"""The C ABI on the CPU: the library loads, exports every function that
include/lapeig.h declares, and rejects bad input before any HIP call (so
these run without a GPU: a valid matrix gets past validation and only then
meets the missing device)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1311_1695_amd as lap
from paper_1311_1695_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lapeig.h")

pytestmark = pytest.mark.skipif(not os.path.exists(lap.library_path()), reason="liblapeig.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lap_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = lap.load_library()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), f"{name} declared in lapeig.h but not exported"
    assert sorted(lap.EXPORTED) == names


def test_status_strings_and_default_opts():
    lib = lap.load_library()
    for code in range(-6, 1):
        assert lib.lap_status_string(code)
    o = lap._Opts()
    lib.lap_eigs_default_opts(ctypes.byref(o))
    # the paper's parameters (Section 4)
    assert (o.m_min, o.m_max, o.itmax, o.rtol_pcg, o.block) == (5, 10, 20, 1e-2, 1)


def _create(rowptr, col, val, n=None):
    class L:
        pass
    L.n = len(rowptr) - 1 if n is None else n
    L.rowptr, L.col, L.val = np.asarray(rowptr), np.asarray(col), np.asarray(val, dtype=float)
    with pytest.raises(lap.LapError) as e:
        lap.Plan(L)
    return e.value


def _good():
    L = gg.path_graph(4)
    return L.rowptr.copy(), L.col.copy(), L.val.copy()


def test_valid_matrix_passes_validation_then_needs_a_device():
    rp, cl, vl = _good()
    err = _create(rp, cl, vl)
    assert err.code in (lap.LAP_EDEVICE, lap.LAP_ENOMEM)


def test_batch_autotune_and_layout_argument_checks():
    lib = lap.load_library()
    thr, tuned, secs = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
    assert lib.lap_batch_autotune(None, lap.LAP_PREC_MIXED, ctypes.byref(thr), ctypes.byref(secs)) == lap.LAP_EINVAL
    assert lib.lap_batch_layout(None, lap.LAP_PREC_MIXED, ctypes.byref(thr), ctypes.byref(tuned)) == lap.LAP_EINVAL
    with pytest.raises(lap.LapError):
        lap._precision_code("bf16")
    # the solve entry points reject a NULL batch before touching the device,
    # with the eigenvectors asked for on the host or on the device
    ev = (ctypes.c_double * 10)()
    for on_device in (0, 1):
        assert lib.lap_batch_eigs_ex(None, 5, 1e-8, None, ev, None, on_device, None, None, None) == lap.LAP_EINVAL
    assert lib.lap_batch_eigs(None, 5, 1e-8, None, ev, None, None, None, None) == lap.LAP_EINVAL


def test_plan_order_argument_checked_before_hip():
    rp, cl, vl = _good()

    class L:
        pass
    L.n, L.rowptr, L.col, L.val = 4, rp, cl, vl
    lib = lap.load_library()
    csr, keep = lap._csr_struct(L)
    h = ctypes.c_void_p()
    for bad in (-1, 2, 7):
        assert lib.lap_plan_create_ex(ctypes.byref(csr), None, bad, ctypes.byref(h)) == lap.LAP_EINVAL
        assert not h.value
    with pytest.raises(lap.LapError) as e:
        lap.Plan(L, order="rcm")
    assert e.value.code == lap.LAP_EINVAL
    # a valid order gets past the checks and then needs the device
    for order in ("hub", "caller"):
        with pytest.raises(lap.LapError) as e:
            lap.Plan(L, order=order)
        assert e.value.code in (lap.LAP_EDEVICE, lap.LAP_ENOMEM)


@pytest.mark.parametrize("case", [
    "rowptr0", "rowptr_decreasing", "rowptr_end", "col_range", "col_unsorted", "col_duplicate",
    "nonfinite", "positive_offdiag", "asym_pattern", "asym_values", "bad_diagonal", "bad_diagonal_float",
])
def test_invalid_laplacian_rejected_before_hip(case):
    rp, cl, vl = _good()  # path 0-1-2-3: rows [0,1] [0,1,2] [1,2,3] [2,3]
    if case == "rowptr0":
        rp = rp + 1; rp[0] = 1
    elif case == "rowptr_decreasing":
        rp[2], rp[3] = rp[3], rp[2]
    elif case == "rowptr_end":
        rp[-1] -= 1
    elif case == "col_range":
        cl[-1] = 9
    elif case == "col_unsorted":
        cl[2], cl[3] = cl[3], cl[2]; vl[2], vl[3] = vl[3], vl[2]
    elif case == "col_duplicate":
        cl[3] = cl[2]
    elif case == "nonfinite":
        vl[0] = np.nan
    elif case == "positive_offdiag":
        vl[1] = 1.0; vl[2] = 1.0
    elif case == "asym_pattern":
        # drop edge 2->3 from row 2 only (keep the row's diagonal consistent)
        keep = np.ones(len(cl), bool); keep[7] = False
        cl, vl = cl[keep], vl[keep]
        vl[6] = 1.0
        rp = rp.copy(); rp[3:] -= 1
    elif case == "asym_values":
        vl = vl.copy(); vl[1] = -2.0; vl[0] = 2.0
    elif case == "bad_diagonal":
        vl[0] = 2.0
    elif case == "bad_diagonal_float":
        vl = vl * 0.3; vl[0] *= (1 + 1e-9)
    err = _create(rp, cl, vl)
    assert err.code in (lap.LAP_ENOTLAPLACIAN,), (case, err)
    assert "row" in str(err) or "rowptr" in str(err)


def test_bad_sizes_rejected():
    err = _create(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), n=0)
    assert err.code == lap.LAP_EINVAL


def test_entry_points_reject_null_arguments():
    lib = lap.load_library()
    ev = np.zeros(3)
    assert lib.lap_eigs(None, 3, 1e-8, None, ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0,
                        None, None) == lap.LAP_EINVAL
    assert lib.lap_spmv(None, lap.LAP_F32, 1, None, None, None, 0, None) == lap.LAP_EINVAL
    assert lib.lap_orth(lap.LAP_F32, 10, 0, None, 1, None, None, None) == lap.LAP_EINVAL
    assert lib.lap_orth(lap.LAP_F64, 10, 0, None, 1, None, None, None) == lap.LAP_EINVAL
    assert lib.lap_sym_eig(4, None, None, None, None, None) == lap.LAP_EINVAL
    assert lib.lap_sym_eig(0, None, None, None, None, None) == lap.LAP_EINVAL
    assert lib.lap_sym_eig(97, None, None, None, None, None) == lap.LAP_EINVAL
    th = np.zeros(1)
    assert lib.lap_pcg(None, lap.LAP_F32, 1, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0,
                       None, None, 20, 1e-2, None, 0, None) == lap.LAP_EINVAL
    assert lib.lap_last_error()


def test_layout_and_tuning_entry_points_reject_null_plans():
    lib = lap.load_library()
    lt, ht = ctypes.c_int32(), ctypes.c_int32()
    assert lib.lap_plan_set_layout(None, 32, 512) == -1
    assert lib.lap_plan_layout(None, ctypes.byref(lt), ctypes.byref(ht)) == -1
    info = lap._TuneInfo()
    assert lib.lap_plan_autotune(None, 0, 0, 1, None, ctypes.byref(info)) == -1


@pytest.mark.parametrize("cfg", [dict(hidden=0), dict(hidden=33), dict(layers=-1), dict(layers=9),
                                 dict(random_channels=17), dict(out_cols=0), dict(out_cols=32)])
def test_network_config_is_validated_before_the_device(cfg):
    base = dict(layers=2, hidden=32, random_channels=4, out_cols=9, seed=1)
    base.update(cfg)
    lib = lap.load_library()
    c = lap._MpnnConfig(base["layers"], base["hidden"], base["random_channels"], base["out_cols"], base["seed"])
    h = ctypes.c_void_p()
    assert lib.lap_mpnn_create(ctypes.byref(c), ctypes.byref(h)) == -1
    assert not h.value


def test_network_entry_points_reject_null_handles():
    lib = lap.load_library()
    loss = ctypes.c_double()
    assert lib.lap_mpnn_create(None, None) == -1
    assert lib.lap_mpnn_num_params(None) == 0
    assert lib.lap_mpnn_get_params(None, None) == -1
    assert lib.lap_mpnn_set_params(None, None) == -1
    assert lib.lap_mpnn_infer(None, None, 1, None, None) == -1
    assert lib.lap_mpnn_loss_grad(None, None, 1, None, 4, ctypes.byref(loss), None, None) == -1
    assert lib.lap_mpnn_train_step(None, None, 1, None, 4, 1e-3, ctypes.byref(loss), None) == -1
    lib.lap_mpnn_destroy(None)


def test_eigs_options_default_to_a_host_start_block():
    lib = lap.load_library()
    o = lap._Opts()
    lib.lap_eigs_default_opts(ctypes.byref(o))
    assert o.init_on_device == 0 and o.init_cols == 0 and not o.init


def _net_file(path, *, magic=b"LAPEIG-MPNN\n", fmt=1, layers=1, hidden=4, rc=0, oc=2, num_params=None,
              step=3, payload=None, checksum=None, payload_bytes=None, drop=None):
    """A network file in the documented format (lapeig.h, lap_mpnn_save),
    written here field by field so each check of the loader can be hit."""
    # per layer a 2 F_in x F_out matrix and F_out biases (F_0 = 3 + rc)
    dims = [3 + rc] + [hidden] * layers + [oc]
    np_ = sum(2 * dims[i] * dims[i + 1] + dims[i + 1] for i in range(layers + 1))
    if num_params is None:
        num_params = np_
    if payload is None:
        rng = np.random.default_rng(0)
        payload = np.concatenate([rng.standard_normal(2 * np_), rng.random(np_)]).astype("<f4").tobytes()
    h = 0xcbf29ce484222325
    for byte in payload:  # FNV-1a 64
        h = ((h ^ byte) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    fields = {"format": fmt, "layers": layers, "hidden": hidden, "random_channels": rc, "out_cols": oc,
              "seed": 5, "num_params": num_params, "adam_step": step,
              "payload_bytes": len(payload) if payload_bytes is None else payload_bytes,
              "dtype": "float32-le", "fnv1a64": "%016x" % (h if checksum is None else checksum)}
    if drop:
        del fields[drop]
    import json
    with open(path, "wb") as fh:
        fh.write(magic)
        fh.write((json.dumps(fields) + "\n").encode())
        fh.write(payload)
    return np_


def _load_code(path):
    lib = lap.load_library()
    h = ctypes.c_void_p()
    code = lib.lap_mpnn_load(os.fsencode(path) if path is not None else None, ctypes.byref(h))
    assert not h.value
    return code


def test_network_file_is_checked_before_the_device(tmp_path):
    """lap_mpnn_load reads and checks the whole file on the host: every
    malformed file is rejected with LAP_EINVAL (LAP_EUNSUPPORTED for a newer
    format) before any HIP call; a valid one gets past the checks and only
    then meets the missing device."""
    p = str(tmp_path / "net.bin")
    assert _load_code(None) == lap.LAP_EINVAL
    assert _load_code(str(tmp_path / "missing.bin")) == lap.LAP_EINVAL
    cases = [dict(magic=b"NOT-A-NET\n"), dict(fmt=2), dict(layers=9), dict(hidden=0), dict(hidden=33),
             dict(rc=17), dict(oc=0), dict(oc=32), dict(step=-1), dict(num_params=7), dict(payload_bytes=12),
             dict(checksum=1), dict(drop="fnv1a64"), dict(drop="num_params")]
    for kw in cases:
        _net_file(p, **kw)
        want = lap.LAP_EUNSUPPORTED if kw.get("fmt") == 2 else lap.LAP_EINVAL
        assert _load_code(p) == want, kw
    n = _net_file(p)
    good = open(p, "rb").read()
    with open(p, "wb") as fh:  # truncated payload
        fh.write(good[:-4])
    assert _load_code(p) == lap.LAP_EINVAL
    with open(p, "wb") as fh:  # trailing bytes
        fh.write(good + b"\0")
    assert _load_code(p) == lap.LAP_EINVAL
    bad = np.concatenate([np.full(2 * n, np.nan), np.ones(n)]).astype("<f4").tobytes()
    _net_file(p, payload=bad)  # non-finite values (checksum valid)
    assert _load_code(p) == lap.LAP_EINVAL
    neg = np.concatenate([np.zeros(2 * n), -np.ones(n)]).astype("<f4").tobytes()
    _net_file(p, payload=neg)  # negative second moments
    assert _load_code(p) == lap.LAP_EINVAL
    _net_file(p)
    if not _has_gpu():
        assert _load_code(p) == lap.LAP_EDEVICE
    lib = lap.load_library()
    assert lib.lap_mpnn_save(None, os.fsencode(p)) == lap.LAP_EINVAL
    cfg = lap._MpnnConfig()
    assert lib.lap_mpnn_get_config(None, ctypes.byref(cfg)) == lap.LAP_EINVAL


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
