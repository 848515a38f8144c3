"""The C ABI: the built library loads, exports every function include/psoam.h
declares, and rejects bad arguments with status codes before touching a
device (so these run on a machine without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psoam.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psoam_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2510_23739_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpsoam.so is not built (python -m paper_2510_23739_amd.build)")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["psoam_plan_create", "psoam_plan_destroy", "psoam_apply_A", "psoam_apply_AT",
              "psoam_prox_l1", "psoam_prox_tv", "psoam_prox_tv_ws_bytes", "psoam_solve",
              "psoam_solve_batch", "psoam_last_error"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_python_binding_covers_every_export():
    from paper_2510_23739_amd import _lib
    assert set(_declared()) == set(_lib.EXPORTS)


def test_validation_before_device_work(lib):
    from paper_2510_23739_amd import _lib
    out = C.c_void_p(1)
    g = _lib.Geom(4, 4, 4, 2, 3, 8, 3, 0)
    sp = _lib.Species()
    assert lib.psoam_plan_create(None, C.byref(sp), None, None, None, 4, 0, None,
                                 C.byref(out)) == _lib.EINVAL
    assert out.value is None
    assert b"NULL" in lib.psoam_last_error()
    import numpy as np
    phi = np.ones(4, np.float32)
    t0 = np.zeros((4, 3, 3), np.int32)
    taps = np.zeros((4, 3, 3, 4), np.float32)
    args = lambda gg, w=4, prec=0: (C.byref(gg), C.byref(sp), phi.ctypes.data_as(C.c_void_p),
                                    t0.ctypes.data_as(C.c_void_p), taps.ctypes.data_as(C.c_void_p),
                                    w, prec, None, C.byref(out))
    bad_f = _lib.Geom(4, 4, 4, 2, 3, 8, 2, 0)
    assert lib.psoam_plan_create(*args(bad_f)) == _lib.EINVAL
    assert b"odd" in lib.psoam_last_error()
    bad_s = _lib.Geom(4, 4, 4, 9, 3, 8, 3, 0)
    assert lib.psoam_plan_create(*args(bad_s)) == _lib.EINVAL
    assert lib.psoam_plan_create(*args(g, w=0)) == _lib.EINVAL
    assert lib.psoam_plan_create(*args(g, prec=7)) == _lib.EUNSUPPORTED
    # tau must be positive
    assert lib.psoam_plan_create(*args(g)) == _lib.EINVAL
    assert b"tau" in lib.psoam_last_error()
    many = _lib.Geom(4, 4, 4, 2, 65, 8, 3, 0)
    for s in range(2):
        sp.tau[s] = 2.0
    assert lib.psoam_plan_create(*args(many)) == _lib.EUNSUPPORTED
    phi_bad = np.array([1, 0, 1, 1], np.float32)
    assert lib.psoam_plan_create(C.byref(g), C.byref(sp), phi_bad.ctypes.data_as(C.c_void_p),
                                 t0.ctypes.data_as(C.c_void_p), taps.ctypes.data_as(C.c_void_p),
                                 4, 0, None, C.byref(out)) == _lib.EINVAL
    taps_bad = taps.copy()
    taps_bad[1, 1, 1, 1] = np.nan
    assert lib.psoam_plan_create(C.byref(g), C.byref(sp), phi.ctypes.data_as(C.c_void_p),
                                 t0.ctypes.data_as(C.c_void_p),
                                 taps_bad.ctypes.data_as(C.c_void_p), 4, 0, None,
                                 C.byref(out)) == _lib.EINVAL
    # the separable form needs gamma = 0 and a 0/1 flag
    sep = _lib.Geom(4, 4, 4, 2, 3, 8, 3, 0, 1)
    sp.gamma = 1.0
    assert lib.psoam_plan_create(*args(sep)) == _lib.EINVAL
    assert b"gamma" in lib.psoam_last_error()
    sp.gamma = 0.0
    assert lib.psoam_plan_create(*args(_lib.Geom(4, 4, 4, 2, 3, 8, 3, 0, 2))) == _lib.EINVAL
    assert lib.psoam_prox_r3(None, None, None, 0.1, 0.1, 0.1, 3, None, None) == _lib.EINVAL
    assert lib.psoam_prox_r3_ws_bytes(None) == 0
    # entry points on a NULL plan / bad sizes
    assert lib.psoam_apply_A(None, None, None, None) == _lib.EINVAL
    assert lib.psoam_apply_AT(None, None, None, None) == _lib.EINVAL
    assert lib.psoam_prox_l1(None, None, -1, 0.1, 1, None) == _lib.EINVAL
    assert lib.psoam_prox_l1(None, None, 4, -0.1, 1, None) == _lib.EINVAL
    assert lib.psoam_prox_l1(None, None, 4, float("nan"), 1, None) == _lib.EINVAL
    assert lib.psoam_prox_l1(None, None, 4, 0.1, 1, None) == _lib.EINVAL
    assert lib.psoam_prox_l1(None, None, 0, 0.1, 1, None) == _lib.OK
    assert lib.psoam_prox_tv(None, None, None, 0.1, 3, 0, None, None) == _lib.EINVAL
    assert lib.psoam_prox_tv_ws_bytes(None) == 0
    assert lib.psoam_solve(None, None, None, None, None, None) == _lib.EINVAL
    assert lib.psoam_solve_batch(-1, None, None, None, None, None, None) == _lib.EINVAL
    assert lib.psoam_solve_batch(0, None, None, None, None, None, None) == _lib.OK
    assert lib.psoam_plan_destroy(None) == _lib.OK
    assert lib.psoam_plan_geom(None, None) == _lib.EINVAL
