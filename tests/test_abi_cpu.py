"""The C-ABI library on the CPU: it loads, exports every declared entry point,
and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mffv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mffv_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def mf():
    from paper_2408_03452_amd import mffv
    if not os.path.exists(mffv.LIB_PATH):
        pytest.fail("libmffv.so is not built (run __graft_entry__.build())")
    mffv.lib()
    return mffv


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mffv_create_grid", "mffv_destroy_grid", "mffv_set_transmissibility",
                 "mffv_apply", "mffv_cg_solve", "mffv_cg_solve_batched"):
        assert must in names


def test_library_exports_every_declared_symbol(mf):
    raw = ctypes.CDLL(mf.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_version_and_defaults(mf):
    assert "gfx950" in mf.version()
    o = mf.default_opts()
    assert o.tol == 1e-6 and o.max_iter == 100000 and o.precision == mf.FP32
    assert o.precond == mf.PRECOND_NONE and o.check_every == 16 and o.max_outer == 10


def test_argument_errors_before_any_gpu_work(mf):
    L = mf.lib()
    h = ctypes.c_void_p()
    assert L.mffv_create_grid(2, 4, 4, None, ctypes.byref(h)) == mf.EINVAL
    assert "nx >= 3" in mf.last_error()
    assert L.mffv_create_grid(8, 0, 4, None, ctypes.byref(h)) == mf.EINVAL
    assert L.mffv_create_grid(4096, 4096, 4096, None, ctypes.byref(h)) == mf.EINVAL
    assert "2^31" in mf.last_error()
    assert L.mffv_create_grid(8, 8, 8, None, None) == mf.EINVAL
    assert h.value is None
    assert L.mffv_apply(None, 1, 2) == mf.EINVAL
    assert "NULL" in mf.last_error()
    assert L.mffv_cg_solve(None, 1, 2, None, None) == mf.EINVAL
    assert L.mffv_cg_solve_f64(None, 1, 2, None, None) == mf.EINVAL
    assert L.mffv_set_transmissibility(None, 1, 2, 3, None, 0.0, None, None, None) == mf.EINVAL
    assert L.mffv_perm_to_trans(4, 4, 4, None, 1.0, 1, 2, 3, None) == mf.EINVAL
    assert L.mffv_perm_to_trans(4, 4, 4, 16, -1.0, 32, 48, 64, None) == mf.EINVAL
    assert L.mffv_copy_probe(16, 32, 17, None) == mf.EINVAL
    assert L.mffv_cg_solve_batched(None, 0, None, None, None, None) == mf.EINVAL
    assert L.mffv_set_batched_launch(-1, 4) == mf.EINVAL
    assert L.mffv_set_batched_watchdog(-1.0) == mf.EINVAL
    assert L.mffv_set_batched_watchdog(float("nan")) == mf.EINVAL
    assert L.mffv_set_batched_watchdog(2.0) == mf.OK       # the default again
    assert L.mffv_step_rhs(None, 1, None, 0.0, 2, None, None, None, 3) == mf.EINVAL
    assert L.mffv_time_steps(None, 1, 1, None, 0.0, None, None, None, 2, None, None) == mf.EINVAL
    # face-list grids: faces are checked on the host before any device work
    fk = (ctypes.c_int * 2)(0, 1)
    bad_l = (ctypes.c_int * 2)(1, 1)                      # a face joining a cell to itself
    far_l = (ctypes.c_int * 2)(1, 4)                      # a cell out of range
    for fl_ in (bad_l, far_l):
        assert L.mffv_create_grid_faces(4, 2, fk, fl_, None, ctypes.byref(h)) == mf.EINVAL
    assert "face 1" in mf.last_error()
    assert L.mffv_create_grid_faces(0, 0, None, None, None, ctypes.byref(h)) == mf.EINVAL
    assert L.mffv_create_grid_faces(4, 2, None, None, None, ctypes.byref(h)) == mf.EINVAL
    assert L.mffv_create_grid_faces(4, 0, None, None, None, None) == mf.EINVAL
    assert L.mffv_set_face_transmissibility(None, 1, None, 0.0, None, None, None) == mf.EINVAL
    L.mffv_destroy_grid(None)  # no-op


def test_binding_refuses_host_tensors(mf):
    import torch
    with pytest.raises(ValueError):
        mf._ptr(torch.zeros(4), torch.float32, 4, "x")
