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
    assert lib.psoam_plan_create(*args(g, prec=6)) == _lib.EUNSUPPORTED
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


def test_factorised_validation_before_device_work(lib):
    import numpy as np
    from paper_2510_23739_amd import _lib
    out = C.c_void_p(1)
    sp = _lib.Species()
    for s in range(2):
        sp.tau[s] = 2.0
    phi = np.ones(6, np.float32)
    spr = np.ones((6, 3, 3), np.float32)
    eir = np.array([0.5, 1.0, -0.5], np.float32)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)

    def call(g, sh, spr_=spr, eir_=eir):
        return lib.psoam_plan_create_factorised(C.byref(g), C.byref(sp), ptr(phi), ptr(spr_),
                                                ptr(eir_), C.byref(sh), 0, None, C.byref(out))

    g = _lib.Geom(4, 4, 6, 2, 3, 32, 3, 0, 0)
    good = dict(dr=0.6, z_focus=2.5, t_focus=16, n_eir=3, eir_origin=1)
    sh = lambda **kw: _lib.Shell(**{**good, **kw})
    assert lib.psoam_plan_create_factorised(None, C.byref(sp), ptr(phi), ptr(spr), ptr(eir),
                                            C.byref(sh()), 0, None, C.byref(out)) == _lib.EINVAL
    assert out.value is None
    assert call(g, sh(dr=0.0)) == _lib.EINVAL
    assert call(g, sh(dr=float("inf"))) == _lib.EINVAL
    assert call(g, sh(z_focus=float("nan"))) == _lib.EINVAL
    assert call(g, sh(n_eir=0)) == _lib.EINVAL
    assert call(g, sh(n_eir=33)) == _lib.EINVAL
    assert call(g, sh(eir_origin=3)) == _lib.EINVAL
    assert call(g, sh(eir_origin=-1)) == _lib.EINVAL
    bad_eir = eir.copy()
    bad_eir[2] = np.nan
    assert call(g, sh(), eir_=bad_eir) == _lib.EINVAL
    bad_spr = spr.copy()
    bad_spr[3, 1, 2] = np.inf
    assert call(g, sh(), spr_=bad_spr) == _lib.EINVAL
    assert call(_lib.Geom(4, 4, 6, 2, 3, 32, 3, 0, 1), sh()) == _lib.EUNSUPPORTED
    assert call(_lib.Geom(4, 4, 6, 2, 3, 4097, 3, 0, 0), sh()) == _lib.EUNSUPPORTED
    assert call(_lib.Geom(4, 4, 6, 2, 3, 32, 4, 0, 0), sh()) == _lib.EINVAL
    # a radius step so small that one voxel spans more than 64 samples
    assert call(_lib.Geom(4, 4, 6, 2, 3, 400, 3, 0, 0), sh(dr=0.01, t_focus=200)) == _lib.EUNSUPPORTED
    assert b"wider" in lib.psoam_last_error()


def test_calibration_library_is_separate():
    """The matrix-core calibration loop lives in its own library: built
    beside libpsoam.so, exporting its one entry point (which rejects bad
    arguments before any launch), and absent from the reconstruction ABI."""
    from paper_2510_23739_amd import build
    assert os.path.exists(build.CALIB_LIB), "libpsoam_calib.so is not built"
    cal = C.CDLL(build.CALIB_LIB)
    fn = cal.psoam_calib_mfma_bf16
    fn.restype = C.c_int
    fn.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    assert fn(None, 8, 8, None) == 1
    assert "psoam_calib_mfma_bf16" not in _declared()


def test_tuned_creation_validates_before_device_work(lib):
    from paper_2510_23739_amd import _lib
    import numpy as np
    out = C.c_void_p(1)
    rep = _lib.TuneReport()
    sp = _lib.Species()
    for s in range(2):
        sp.tau[s] = 2.0
    assert lib.psoam_plan_create_tuned(None, C.byref(sp), None, None, None, 4, 1, None,
                                       C.byref(out), C.byref(rep)) == _lib.EINVAL
    assert out.value is None
    phi = np.ones(4, np.float32)
    t0 = np.zeros((4, 3, 3), np.int32)
    taps = np.zeros((4, 3, 3, 4), np.float32)
    args = lambda gg, prec=1, o=C.byref(out): (
        C.byref(gg), C.byref(sp), phi.ctypes.data_as(C.c_void_p),
        t0.ctypes.data_as(C.c_void_p), taps.ctypes.data_as(C.c_void_p), 4, prec, None, o,
        C.byref(rep))
    g = _lib.Geom(4, 4, 4, 2, 3, 8, 3, 0)
    assert lib.psoam_plan_create_tuned(*args(g, o=None)) == _lib.EINVAL
    assert b"out is NULL" in lib.psoam_last_error()
    assert lib.psoam_plan_create_tuned(*args(_lib.Geom(4, 4, 4, 2, 3, 8, 2, 0))) == _lib.EINVAL
    assert b"odd" in lib.psoam_last_error()
    assert lib.psoam_plan_create_tuned(*args(g, prec=7)) == _lib.EUNSUPPORTED


def test_binding_checks_batch_and_l1_arguments():
    """solve_batch and prox_l1 check every tensor's shape, dtype, device and
    layout (and the batch's list lengths) before anything reaches the library."""
    import types

    import torch

    import paper_2510_23739_amd as pk
    plan = types.SimpleNamespace(y_shape=(2, 3, 3, 8), c_shape=(1, 3, 3, 4))
    p = torch.zeros(plan.y_shape)
    c = torch.zeros(plan.c_shape)
    with pytest.raises(ValueError, match="plans but"):
        pk.solve_batch([plan, plan], [p], [c, c], [{}, {}])
    with pytest.raises(ValueError, match="plans but"):
        pk.solve_batch([plan], [p], [c], [{}, {}])
    with pytest.raises(ValueError, match="CUDA"):     # host tensors
        pk.solve_batch([plan], [p], [c], [{}])
    with pytest.raises(ValueError, match="CUDA"):
        pk.prox_l1(torch.zeros(8), 0.1)
    with pytest.raises(ValueError, match="CUDA"):     # float64
        pk.prox_l1(torch.zeros(8, dtype=torch.float64), 0.1)
