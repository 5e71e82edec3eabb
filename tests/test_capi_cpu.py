"""The C-ABI library loads and exports every function include/taylens.h
declares; argument validation happens on the host before any HIP call, so the
error paths are testable without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "taylens.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(tl_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def tl():
    from paper_1307_0719_amd import taylens

    return taylens


def test_every_declared_symbol_is_exported(tl):
    names = _declared()
    assert len(names) >= 15
    lib = tl.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tl.EXPORTS)
    assert tl.version() == 10000


def _create(tl, lmax, ntheta, nphi, order=3, prec=1, pol=1, rotate=1, naive=0, batch=0, cap=0, maps16=0, lmax_phi=0,
            theta_fft=0):
    h = ctypes.c_void_p(123)
    o = tl.Options(order, prec, pol, rotate, naive, batch, cap, maps16, lmax_phi, theta_fft)
    rc = tl.lib().tl_plan_create(ctypes.byref(h), lmax, tl.Grid(ntheta, nphi), ctypes.byref(o), None)
    return rc, h, tl.lib().tl_last_error().decode()


@pytest.mark.parametrize("args,code", [
    ((-1, 3, 4), -1), ((10, 1, 20), -1), ((10, 11, 19), -1), ((10, 11, 18), -1), ((10, 11, 22), -2),
    ((10, 11, 20, 9), -1), ((10, 11, 20, -1), -1), ((10, 11, 20, 3, 7), -1), ((10, 11, 20, 7, 4), -2), ((10, 11, 20, 4, 4, 1, 1, 0, 7), -1),
    ((10, 11, 20, 3, 1, 2), -1), ((10, 11, 20, 3, 1, 1, 5), -1), ((10, 11, 20, 3, 1, 1, 1, 3), -1),
    ((10, 11, 20, 3, 1, 1, 0, 0, 2), -1), ((10, 11, 20, 3, 1, 1, 0, 0, 0, -5), -1),
    ((64, 65, 128, 3, 1, 1, 1, 0, 0, 1000), -4), ((10, 11, 20, 3, 1, 1, 1, 0, 0, 0, 2), -1),
    ((10, 11, 20, 3, 1, 1, 1, 0, 0, 0, 0, 9), -1), ((10, 11, 20, 3, 1, 1, 1, 0, 0, 0, 0, 11), -1),
    ((10, 11, 40000, 3, 1, 1, 1, 0, 0, 0, 0, 20000), -2),
    # theta_fft: 0 or 1; the FP64 form only; ntheta - 1 a power of two; lmax <= ntheta - 2
    ((10, 17, 20, 3, 0, 1, 1, 0, 0, 0, 0, 0, 2), -1), ((10, 17, 20, 3, 1, 1, 1, 0, 0, 0, 0, 0, 1), -2),
    ((10, 11, 20, 3, 0, 1, 1, 0, 0, 0, 0, 0, 1), -2), ((16, 17, 40, 3, 0, 1, 1, 0, 0, 0, 0, 0, 1), -2),
    ((10, 8194, 20, 3, 0, 1, 1, 0, 0, 0, 0, 0, 1), -2)])
def test_invalid_plan_arguments(tl, args, code):
    rc, h, msg = _create(tl, *args)
    assert rc == code, msg
    assert h.value is None
    assert msg


def test_null_arguments(tl):
    L = tl.lib()
    assert L.tl_plan_create(None, 8, tl.Grid(9, 16), None, None) == -1
    h = ctypes.c_void_p()
    assert L.tl_plan_create(ctypes.byref(h), 8, tl.Grid(9, 16), None, None) == -1
    for fn, n in (("tl_lens_map", 8), ("tl_deflection", 4), ("tl_legendre", 5), ("tl_synth_derivs", 5),
                  ("tl_remap", 7), ("tl_lens_map_pos", 9)):
        assert getattr(L, fn)(*([None] * n)) == -1, fn
    assert L.tl_plan_destroy(None) == 0
    assert L.tl_lens_map_batch(0, None, None, None) == 0
    assert L.tl_lens_map_batch(-1, None, None, None) == -1
    assert L.tl_lens_map_batch(2, None, None, None) == -1
    assert L.tl_plan_profile(None, 1) == -1
    assert L.tl_plan_stage_times(None, None, None) == -1
    v = ctypes.c_int64()
    assert L.tl_plan_query(None, 0, ctypes.byref(v)) == -1


def test_cnn_null_arguments(tl):
    L = tl.lib()
    h = ctypes.c_void_p()
    assert L.tl_cnn_create(None, None) == -1
    assert L.tl_cnn_create(ctypes.byref(h), None) == -1 and h.value is None
    assert L.tl_cnn_destroy(None) == 0
    assert L.tl_cnn_get_params(None, None) == -1
    assert L.tl_cnn_set_params(None, None) == -1
    assert L.tl_cnn_forward(None, None, None, None, None, None, 0, None) == -1
    assert L.tl_cnn_grad(None, None, None, None, None, None, 0, None, None) == -1
    assert L.tl_cnn_train_step(None, None, None, None, None, None, 0, None, ctypes.c_float(1e-3), None) == -1
    assert L.tl_lens_map_cnn(*([None] * 9)) == -1
    assert tl.CNN_NPARAM == 15142 and tl.CNN_NTRAIN == 15139


def test_batch_null_arguments(tl):
    L = tl.lib()
    h = ctypes.c_void_p()
    o = tl.BatchOptions(1, 1, 0, 0)
    assert L.tl_batch_create(None, 1, None, ctypes.byref(o)) == -1
    assert L.tl_batch_create(ctypes.byref(h), 0, None, ctypes.byref(o)) == -1
    assert L.tl_batch_create(ctypes.byref(h), 2, None, ctypes.byref(o)) == -1
    bad = tl.BatchOptions(1, 1, 9, 0)
    arr = (ctypes.c_void_p * 1)(None)
    assert L.tl_batch_create(ctypes.byref(h), 1, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(bad)) == -1
    assert L.tl_batch_create(ctypes.byref(h), 1, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(o)) == -1
    assert h.value is None
    assert L.tl_batch_destroy(None) == 0
    assert L.tl_batch_run(None, None, None) == -1
    assert L.tl_batch_info(None, None, None, None, None) == -1


def test_healpix_plan_arguments(tl):
    """HEALPix plans validate nside before any device call."""
    L = tl.lib()
    h = ctypes.c_void_p()
    o = tl.Options(3, 1, 1, 1, 0, 0, 0)
    assert L.tl_plan_create_healpix(None, 16, 4, ctypes.byref(o), None) == tl.TL_ERR_INVALID
    assert L.tl_plan_create_healpix(ctypes.byref(h), 16, 0, ctypes.byref(o), None) == tl.TL_ERR_INVALID
    assert L.tl_plan_create_healpix(ctypes.byref(h), 16, 4096, ctypes.byref(o), None) == tl.TL_ERR_UNSUPPORTED
    bad = tl.Options(9, 1, 1, 1, 0, 0, 0)
    assert L.tl_plan_create_healpix(ctypes.byref(h), 16, 4, ctypes.byref(bad), None) == tl.TL_ERR_INVALID
    # the potential's own band limit is an equal-theta feature
    sep = tl.Options(3, 1, 1, 1, 0, 0, 0, 0, 24)
    assert L.tl_plan_create_healpix(ctypes.byref(h), 16, 4, ctypes.byref(sep), None) == tl.TL_ERR_UNSUPPORTED
    # so are the theta-derivative FFTs along the great circles
    tf = tl.Options(3, 0, 1, 1, 0, 0, 0, 0, 0, 1)
    assert L.tl_plan_create_healpix(ctypes.byref(h), 16, 4, ctypes.byref(tf), None) == tl.TL_ERR_UNSUPPORTED
    assert not h.value
