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
