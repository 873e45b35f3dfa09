"""The C ABI without a GPU: the library loads, exports every function that
include/kktfwi.h declares, and rejects bad arguments before any HIP call.

No call here launches GPU work: argument validation happens first, so each call
below returns its status code on a machine without a GPU as on one with it."""

import ctypes as C
import os

import numpy as np
import pytest

from paper_2204_06489_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libkktfwi.so not built")


def _desc(**over):
    nx, nz, K, nrec = 21, 15, 2, 5
    keep = {}

    def arr(vals, ct):
        a = (ct * len(vals))(*vals)
        keep[id(a)] = a
        return a

    d = _lib.KfDesc()
    d.nx, d.nz, d.h, d.npml = nx, nz, 10.0, 4
    d.pml_r0, d.pml_cref, d.omega = 1e-3, 2000.0, 2 * np.pi * 5.0
    d.K = K
    d.src_ix, d.src_iz = arr([5, 15], C.c_int32), arr([4, 4], C.c_int32)
    d.nrec = nrec
    d.rec_ix, d.rec_iz = arr([4, 7, 10, 13, 16], C.c_int32), arr([4] * nrec, C.c_int32)
    d.w = None
    d.eps, d.reg_on_update = 1.0, 1
    for k, v in over.items():
        if k in ("src_ix", "src_iz", "rec_ix", "rec_iz"):
            v = arr(v, C.c_int32)
        setattr(d, k, v)
    return d, keep


def _create(d, gamma=None):
    g = np.full((d.nz, d.nx), 1 / 2000.0**2) if gamma is None else gamma
    out = C.c_void_p(123)
    st = _lib.lib().kf_create(C.byref(d), g.ctypes.data_as(C.c_void_p) if g is not None else None, 0, None,
                              C.byref(out))
    return st, out


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = _lib.header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(names) >= set(_lib._SIGNATURES) - {"kf_version", "kf_last_error"}
    assert {"kkt_apply", "precond_apply", "newton_step", "helmholtz_solve"} <= set(names)
    assert L.kf_version().decode()


@pytest.mark.parametrize("field,value,code,text", [
    ("nx", 2, _lib.KF_ESHAPE, "nx and nz"),
    ("nz", 513, _lib.KF_ESHAPE, "nz must be <= 512"),
    ("h", 0.0, _lib.KF_EINVAL, "h must be > 0"),
    ("npml", 8, _lib.KF_EINVAL, "npml"),
    ("pml_r0", 1.5, _lib.KF_EINVAL, "pml_r0"),
    ("omega", -1.0, _lib.KF_EINVAL, "omega"),
    ("K", 0, _lib.KF_EINVAL, "K must be"),
    ("eps", 0.0, _lib.KF_EINVAL, "eps must be > 0"),
    ("src_ix", [5, 21], _lib.KF_EINVAL, "source 1 is off the grid"),
    ("rec_iz", [4, 4, -1, 4, 4], _lib.KF_EINVAL, "receiver 2 is off the grid"),
])
def test_create_rejects_bad_descriptions(field, value, code, text):
    d, keep = _desc(**{field: value})
    st, out = _create(d)
    assert st == code
    assert out.value is None
    assert text in _lib.lib().kf_last_error().decode()


def test_create_rejects_nonfinite_gamma_and_weights():
    d, keep = _desc()
    g = np.full((d.nz, d.nx), 1 / 2000.0**2)
    g[3, 4] = np.nan
    st, out = _create(d, g)
    assert st == _lib.KF_EINVAL and "gamma must be finite" in _lib.lib().kf_last_error().decode()
    w = np.ones(d.K * d.nrec)
    w[1] = np.inf
    d.w = w.ctypes.data_as(C.POINTER(C.c_double))
    st, out = _create(d)
    assert st == _lib.KF_EINVAL and "weights must be finite" in _lib.lib().kf_last_error().decode()


def test_null_handles_and_batches_are_rejected():
    L = _lib.lib()
    assert L.kf_destroy(None) == _lib.KF_OK
    assert L.kf_batch_destroy(None) == _lib.KF_OK
    assert L.kkt_apply(None, None, None) == _lib.KF_EINVAL
    assert "problem is NULL" in L.kf_last_error().decode()
    assert L.kf_factor(None, 1, None) == _lib.KF_EINVAL
    out = C.c_void_p(7)
    assert L.kf_batch_create(None, 0, None, C.byref(out)) == _lib.KF_EINVAL
    assert out.value is None
    nine = (C.c_void_p * 9)(*([1] * 9))
    assert L.kf_batch_create(nine, 9, None, C.byref(out)) == _lib.KF_EINVAL
    assert "1..8" in L.kf_last_error().decode()
    # concurrent Newton steps: validated before any HIP call (the handles are not read)
    opts = _lib.KfNewtonOpts()
    two = (C.c_void_p * 2)(1, 1)
    data = (C.c_void_p * 2)(8, 8)
    assert L.newton_step_concurrent(None, 1, data, C.byref(opts), None, None, 1, None) == _lib.KF_EINVAL
    assert L.newton_step_concurrent(two, 0, data, C.byref(opts), None, None, 1, None) == _lib.KF_EINVAL
    assert "1..16" in L.kf_last_error().decode()
    assert L.newton_step_concurrent(two, 2, data, C.byref(opts), None, None, 1, None) == _lib.KF_EINVAL
    assert "appears twice" in L.kf_last_error().decode()
