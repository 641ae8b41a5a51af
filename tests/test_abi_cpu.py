"""Host-side checks of the C-ABI library: it loads, exports every function
include/fmm.h declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2508_02626_amd import fmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = fmm.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(fmm.SYMBOLS) == names


def test_invalid_arguments_rejected_on_host():
    lib = fmm.lib()
    h = ctypes.c_void_p()
    o = fmm.Options()
    lib.fmm_default_options(ctypes.byref(o))
    assert (o.uniform_depth, o.max_depth, o.precision, o.want_field) == (-1, 21, 0, 1)
    assert (o.m2l_method, o.kernel, o.softening) == (0, 0, 0.0)
    # null positions
    assert lib.fmm_plan(None, 10, 4, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    assert b"null" in lib.fmm_last_error()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.fmm_plan(fake, 0, 4, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    assert lib.fmm_plan(fake, 10, 17, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    assert lib.fmm_plan(fake, 10, -1, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    assert lib.fmm_plan(fake, 10, 4, 0, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    o.precision = 7
    assert lib.fmm_plan(fake, 10, 4, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    o.precision = 0
    o.uniform_depth = 9
    assert lib.fmm_plan(fake, 10, 4, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    o.uniform_depth = -1
    o.max_depth = 22
    assert lib.fmm_plan(fake, 10, 4, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    o.max_depth = 21
    # softened kernel: FP64, sign-class M2L, order <= 10, eps finite >= 0
    o.kernel, o.softening = 1, 0.01
    for field, val in (("precision", 3), ("m2l_method", 1), ("softening", -1.0), ("softening", float("inf"))):
        keep = getattr(o, field)
        setattr(o, field, val)
        assert lib.fmm_plan(fake, 10, 4, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL, field
        setattr(o, field, keep)
    assert lib.fmm_plan(fake, 10, 11, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    o.kernel = 2
    assert lib.fmm_plan(fake, 10, 4, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    assert b"kernel" in lib.fmm_last_error()
    o.kernel, o.softening = 0, 0.0
    bad_root = (ctypes.c_double * 4)(0, 0, 0, -1)
    o.root = ctypes.cast(bad_root, ctypes.POINTER(ctypes.c_double))
    assert lib.fmm_plan(fake, 10, 4, 8, ctypes.byref(o), None, None, ctypes.byref(h)) == fmm.FMM_EINVAL
    assert h.value is None
    # plan-level calls with a null plan
    assert lib.fmm_evaluate(None, fake, fake, None, None) == fmm.FMM_EINVAL
    assert lib.fmm_plan_destroy(None) == fmm.FMM_EINVAL
    assert lib.fmm_evaluate_batch(None, None, None, None, -1, None) == fmm.FMM_EINVAL
    assert lib.fmm_evaluate_batch(None, None, None, None, 0, None) == fmm.FMM_OK
    alloc = fmm.Allocator()
    assert lib.fmm_plan(fake, 10, 4, 8, None, ctypes.byref(alloc), None, ctypes.byref(h)) == fmm.FMM_EINVAL
    # batched plan construction validates every entry before any device call
    hv = (ctypes.c_void_p * 2)()
    xv = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    nv = (ctypes.c_int64 * 2)(10, 10)
    ov = (ctypes.c_int32 * 2)(4, 17)
    lv = (ctypes.c_int32 * 2)(8, 8)
    assert lib.fmm_plan_batch(-1, None, None, None, None, None, None, None, 4, hv) == fmm.FMM_EINVAL
    assert lib.fmm_plan_batch(0, None, None, None, None, None, None, None, 4, hv) == fmm.FMM_OK
    assert lib.fmm_plan_batch(2, xv, nv, ov, lv, None, None, None, 4, hv) == fmm.FMM_EINVAL
    assert b"plan 1" in lib.fmm_last_error()
    assert hv[0] is None and hv[1] is None


def test_estimate_grows_with_n_and_order():
    a = fmm.estimate(10_000, 4)
    b = fmm.estimate(100_000, 4)
    c = fmm.estimate(100_000, 10)
    assert 0 < a < b < c
    with pytest.raises(fmm.FmmError):
        fmm.estimate(0, 4)
