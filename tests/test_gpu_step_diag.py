"""Diagnostics formed by the step itself (mpdata_set_step_diag /
mpdata_step_diag): the sum of G psi, min, max and non-finite count of each
step call's result, against the oracle's diagnostics of that same field
(sum within 1e-14 of sum |G psi|, the extrema and the count exact), through
the fused 2-D kernel (which accumulates them while it stores each cell: every
chunk length, the safe-mode redo of a chunk, odd and even step counts) and
through the kernels that are followed by a separate pass."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
FCT, IGA, TOT = 1, 2, 4


def _check(plan, p, g=None):
    s, mn, mx, bad = plan.step_diag()
    field = p.double().cpu().numpy()
    gg = g.double().cpu().numpy() if g is not None else None
    rs, rmn, rmx, rbad = oracle.diag(field, gg)
    scale = np.sum(np.abs(field * (gg if gg is not None else 1.0)))
    assert abs(s - rs) <= 1e-14 * scale, (s, rs)
    assert (mn, mx, bad) == (rmn, rmx, rbad)
    return s


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("rows", [0, 16, 40, 7, 1000])
@pytest.mark.parametrize("n_steps", [1, 4])
def test_step_diag_fused2d(rows, n_steps, dtype):
    case = synth.case_2d(shape=(300, 211), seed=4, sigma=(8.0, 30.0))
    plan = mpdata.Plan(case.psi.shape, dtype=dtype, n_iters=3, opts=FCT)
    plan.set_tile_rows(rows)
    plan.set_step_diag(True)
    c = [dev(x, dtype) for x in case.c]
    p = dev(case.psi, dtype)
    plan.step(p, c, n_steps=n_steps)
    _check(plan, p)
    # the same bits as without the diagnostics
    q = dev(case.psi, dtype)
    plan.set_step_diag(False)
    plan.step(q, c, n_steps=n_steps)
    torch.cuda.synchronize()
    assert torch.equal(p, q)


def test_step_diag_safe_mode_redo():
    """A subnormal band makes the fused kernel redo chunks in safe mode; the
    partials of a redone chunk are those of the redo."""
    shape = (130, 150)
    gen = synth.rng(12)
    c = synth.small_advector(shape, 0.45, gen)
    psi = synth.blob_field(shape, 6, (10.0, 30.0), "uniform", gen, periodic=True)
    psi[40:60, :] = gen.uniform(0.0, 1.0, size=(20, shape[1])) * 2.0 ** -1060
    plan = mpdata.Plan(shape, n_iters=3, opts=FCT)
    plan.set_step_diag(True)
    p = dev(psi, torch.float64)
    plan.step(p, [dev(x, torch.float64) for x in c], n_steps=3)
    _check(plan, p)


PATHS = [((64, 70), 1, 2, FCT, False, mpdata.KERNEL_AUTO),        # 2-D single pass
         ((64, 70), 0, 3, FCT | TOT, True, mpdata.KERNEL_AUTO),    # single pass (G, tot)
         ((64, 70), 0, 3, FCT | TOT, True, mpdata.KERNEL_STAGED),  # stage by stage
         ((64, 70), 0, 3, FCT, False, mpdata.KERNEL_STAGED),
         ((12, 14, 70), 1, 2, TOT | IGA, True, mpdata.KERNEL_AUTO),  # 3-D one launch
         ((300,), 0, 2, FCT, False, mpdata.KERNEL_AUTO)]             # 1-D resident


@pytest.mark.parametrize("shape,bc,n_iters,opts,with_g,kernel", PATHS)
def test_step_diag_other_paths(shape, bc, n_iters, opts, with_g, kernel):
    gen = synth.rng(21)
    g = gen.uniform(0.7, 1.3, size=shape) if with_g else None
    if len(shape) == 1:
        c = [np.full(shape[0] + 1, 0.41)]
    elif bc == 0:
        c = synth.small_advector(shape, 0.45, gen, g=g)
    else:
        c = synth.random_advector(shape, 0.4, gen)
    psi = synth.blob_field(shape, 5, (3.0, 9.0), "normal" if opts & IGA else "uniform", gen,
                           periodic=(bc == 0))
    plan = mpdata.Plan(shape, n_iters=n_iters, opts=opts, bc=bc, has_g=with_g, kernel=kernel)
    plan.set_step_diag(True)
    p = dev(psi, torch.float64)
    gd = dev(g, torch.float64)
    plan.step(p, [dev(x, torch.float64) for x in c], g=gd, n_steps=3)
    _check(plan, p, gd)
    plan.step(p, [dev(x, torch.float64) for x in c], g=gd, n_steps=0)   # the field as it is
    _check(plan, p, gd)


def test_step_diag_nonfinite_and_errors():
    case = synth.case_2d(shape=(128, 96), seed=6, sigma=(4.0, 12.0))
    plan = mpdata.Plan(case.psi.shape, n_iters=3, opts=FCT)
    out = (ctypes.c_double * 3)()
    bad = ctypes.c_int64(0)
    L = mpdata.lib()
    assert L.mpdata_step_diag(plan._handle, out, ctypes.byref(bad)) == mpdata.EINVAL
    plan.set_step_diag(True)
    assert L.mpdata_step_diag(plan._handle, out, ctypes.byref(bad)) == mpdata.EINVAL
    p = dev(case.psi, torch.float64)
    p[60, 50] = float("nan")
    c = [dev(x, torch.float64) for x in case.c]
    plan.step(p, c, n_steps=2)
    torch.cuda.synchronize()
    assert L.mpdata_step_diag(plan._handle, out, ctypes.byref(bad)) == mpdata.ENONFINITE
    assert bad.value == int(torch.sum(~torch.isfinite(p)).item()) >= 1
    plan.set_step_diag(False)
    assert L.mpdata_step_diag(plan._handle, out, ctypes.byref(bad)) == mpdata.EINVAL
