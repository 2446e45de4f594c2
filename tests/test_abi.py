"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/mpdata.h declares, and validates descriptors before
touching any device."""
import ctypes
import os
import re

import pytest

from paper_1407_1309_amd import mpdata

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpdata.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpdata_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(mpdata.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = mpdata.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _desc(shape, dtype=mpdata.F64, n_iters=2, opts=0, bc=0, has_g=0):
    d = mpdata.Desc()
    d.n_dims = len(shape)
    for k in range(3):
        d.shape[k] = shape[k] if k < len(shape) else 1
        d.bc[k] = bc
    d.dtype, d.n_iters, d.opts, d.has_g = dtype, n_iters, opts, has_g
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(shape=(0,)), mpdata.EINVAL),
    (dict(shape=(2,)), mpdata.EINVAL),                    # periodic needs >= 3
    (dict(shape=(4, 4, 4, 4)[:3], n_iters=0), mpdata.EINVAL),
    (dict(shape=(8,), n_iters=9), mpdata.EINVAL),
    (dict(shape=(8,), opts=64), mpdata.EINVAL),           # unknown option bit
    (dict(shape=(8,), opts=mpdata.OPT_ABS | mpdata.OPT_IGA), mpdata.EINVAL),
    (dict(shape=(8,), bc=5), mpdata.EINVAL),
    (dict(shape=(8,), dtype=7), mpdata.EINVAL),
    (dict(shape=(8,), opts=mpdata.OPT_IGA, n_iters=3), mpdata.EUNSUPPORTED),
    (dict(shape=(1 << 31,)), mpdata.EINVAL),              # 32-bit per-dimension indices
    (dict(shape=(1 << 30,)), mpdata.EINVAL),
    (dict(shape=(4, 1 << 30), bc=1), mpdata.EINVAL),
])
def test_init_rejects_bad_descriptors(kw, code):
    L = mpdata.lib()
    d = _desc(**kw)
    assert L.mpdata_workspace_bytes(ctypes.byref(d)) == 0
    h = ctypes.c_void_p()
    rc = L.mpdata_init(ctypes.byref(d), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h))
    assert rc == code
    assert not h.value
    assert L.mpdata_last_error().decode()


def test_open_boundary_allows_one_cell():
    L = mpdata.lib()
    d = _desc((1,), bc=mpdata.BC_OPEN)
    assert L.mpdata_workspace_bytes(ctypes.byref(d)) > 0


def test_init_rejects_missing_or_small_workspace():
    L = mpdata.lib()
    d = _desc((64, 64))
    need = L.mpdata_workspace_bytes(ctypes.byref(d))
    assert need >= 2 * 64 * 64 * 8
    h = ctypes.c_void_p()
    assert L.mpdata_init(ctypes.byref(d), None, need, None, ctypes.byref(h)) == mpdata.EWORKSPACE
    assert L.mpdata_init(ctypes.byref(d), ctypes.c_void_p(256), need - 1, None,
                         ctypes.byref(h)) == mpdata.EWORKSPACE
    assert L.mpdata_init(ctypes.byref(d), ctypes.c_void_p(257), need, None,
                         ctypes.byref(h)) == mpdata.EWORKSPACE


def test_workspace_scales_with_dtype():
    L = mpdata.lib()
    a = L.mpdata_workspace_bytes(ctypes.byref(_desc((128, 96), dtype=mpdata.F64)))
    b = L.mpdata_workspace_bytes(ctypes.byref(_desc((128, 96), dtype=mpdata.F32)))
    assert a > b > 0


def test_null_plan_calls_fail_cleanly():
    L = mpdata.lib()
    assert L.mpdata_step(None, None, None, None, None, None, 1) == mpdata.EINVAL
    assert L.mpdata_set_kernel(None, 0) == mpdata.EINVAL
    P3, D3 = ctypes.c_void_p * 3, ctypes.c_double * 3
    assert L.mpdata_vip_advector(None, P3(), None, P3(), None, 0.1, D3(1, 1, 1), 0.0,
                                 P3()) == mpdata.EINVAL
    assert L.mpdata_sw_step(None, None, P3(), None, P3(), P3(), 0.1, D3(1, 1, 1), 1.0, 0.0,
                            1) == mpdata.EINVAL
    assert L.mpdata_set_cancel_flag(None, None) == mpdata.EINVAL
    out = ctypes.c_int64(7)
    assert L.mpdata_steps_done(None, ctypes.byref(out)) == mpdata.EINVAL
    assert L.mpdata_osc_step(None, None, None, None, None, None, None, 0.1, 1) == mpdata.EINVAL
    assert L.mpdata_step_rhs(None, None, None, None, None, None, None, 0.0, None,
                             0.0) == mpdata.EINVAL
    assert L.mpdata_last_error()  # the message of the last failure
    L.mpdata_destroy(None)


def test_batched_sizing_validates_shapes():
    L = mpdata.lib()
    shapes = (ctypes.c_int64 * 4)(64, 80, 2, 100)
    assert L.mpdata_batched_workspace_bytes(2, shapes, mpdata.F32, 2, 1, 0) == 0
    shapes = (ctypes.c_int64 * 4)(64, 80, 70, 100)
    assert L.mpdata_batched_workspace_bytes(2, shapes, mpdata.F32, 2, 1, 0) >= 4 * (64 * 80 + 70 * 100)
