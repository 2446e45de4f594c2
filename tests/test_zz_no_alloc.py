"""mpdata_diag_noalloc (the allocation-free diagnostics, called through the
C ABI) against mpdata_diag of a plan on the same fields: two calls in a row,
the second with a smaller field, so the shared scratch array is reused with
fewer block partials; both FP64 and FP32, with and without G, and a field
with non-finite values."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1407_1309_amd import mpdata, synth

pytestmark = pytest.mark.gpu


def _abi_noalloc(psi, g):
    out = (ctypes.c_double * 3)()
    bad = ctypes.c_int64(0)
    rc = mpdata.lib().mpdata_diag_noalloc(
        mpdata.F64 if psi.dtype == torch.float64 else mpdata.F32, psi.numel(),
        ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(g.data_ptr()) if g is not None else None,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), out, ctypes.byref(bad))
    return rc, (out[0], out[1], out[2], int(bad.value))


def _abi_plan(psi, g):
    plan = mpdata.Plan(tuple(psi.shape), dtype=psi.dtype, has_g=g is not None)
    out = (ctypes.c_double * 3)()
    bad = ctypes.c_int64(0)
    torch.cuda.synchronize()
    rc = mpdata.lib().mpdata_diag(plan._handle, ctypes.c_void_p(psi.data_ptr()),
                                  ctypes.c_void_p(g.data_ptr()) if g is not None else None,
                                  out, ctypes.byref(bad))
    return rc, (out[0], out[1], out[2], int(bad.value))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("with_g", [False, True], ids=["g1", "g"])
def test_noalloc_diag_matches_plan_diag(dtype, with_g):
    gen = synth.rng(77)
    # large field first (1024 block partials), then a small one (few blocks)
    for shape in [(1500, 1300), (37, 29)]:
        psi = torch.from_numpy(gen.normal(size=shape)).to("cuda", dtype)
        g = torch.from_numpy(gen.uniform(0.5, 2.0, size=shape)).to("cuda", dtype) if with_g \
            else None
        rc_a, a = _abi_noalloc(psi, g)
        rc_b, b = _abi_plan(psi, g)
        assert rc_a == rc_b == mpdata.OK, (shape, rc_a, rc_b)
        assert a == b, (shape, a, b)          # same kernels, same partials: same bits
        assert a[3] == 0


def test_noalloc_diag_nonfinite_and_errors():
    x = torch.ones(5000, dtype=torch.float64, device="cuda")
    x[17] = float("nan")
    x[4000] = float("inf")
    rc_a, a = _abi_noalloc(x, None)
    rc_b, b = _abi_plan(x, None)
    assert rc_a == rc_b == mpdata.ENONFINITE
    assert a == b and a[3] == 2
    y = torch.ones(10, dtype=torch.float64, device="cuda")
    rc, _ = _abi_noalloc(y, None)
    assert rc == mpdata.OK
    out = (ctypes.c_double * 3)()
    bad = ctypes.c_int64(0)
    L = mpdata.lib()
    assert L.mpdata_diag_noalloc(mpdata.F64, 0, ctypes.c_void_p(y.data_ptr()), None, None, out,
                                 ctypes.byref(bad)) == mpdata.EINVAL
    assert L.mpdata_diag_noalloc(mpdata.F64, (1 << 40) + 1, ctypes.c_void_p(y.data_ptr()), None,
                                 None, out, ctypes.byref(bad)) == mpdata.EINVAL
    assert L.mpdata_diag_noalloc(7, 10, ctypes.c_void_p(y.data_ptr()), None, None, out,
                                 ctypes.byref(bad)) == mpdata.EINVAL
    # the Python wrapper gives the same numbers
    s, mn, mx, nb = mpdata.diag_noalloc(y)
    assert (s, mn, mx, nb) == (10.0, 1.0, 1.0, 0)
