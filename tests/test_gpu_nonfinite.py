"""Failure detection through every step kernel: a NaN or an infinity
written into psi or into one advector wall reaches psi of the following
steps, and mpdata_diag (called through the C ABI) then returns
MPDATA_ENONFINITE; mpdata_courant_max reports a non-finite advector before
a run.  The paper's counterpart is the NaN check of its debug builds
(Sect. 2.4).  The clean run of the same inputs is finite and returns
MPDATA_OK, so the status comes from the injected value."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
FCT, IGA, TOT = 1, 2, 4


def _diag_status(plan, psi, g=None):
    out = (ctypes.c_double * 3)()
    bad = ctypes.c_int64(0)
    torch.cuda.synchronize()
    rc = mpdata.lib().mpdata_diag(plan._handle, ctypes.c_void_p(psi.data_ptr()),
                                  ctypes.c_void_p(g.data_ptr()) if g is not None else None,
                                  out, ctypes.byref(bad))
    return rc, int(bad.value)


# (name, shape, bc, n_iters, opts, with_g, kernel): one configuration per
# kernel family the automatic choice can take, plus the staged path
FAMILIES = [
    ("fused2d", (70, 150), 0, 3, FCT, False, mpdata.KERNEL_AUTO),
    ("pass2d", (70, 150), 1, 2, FCT, False, mpdata.KERNEL_AUTO),
    ("staged2d", (70, 150), 0, 3, FCT | TOT, True, mpdata.KERNEL_STAGED),
    ("staged3d", (12, 14, 30), 1, 2, FCT, True, mpdata.KERNEL_STAGED),
    ("fused3d", (12, 14, 70), 1, 2, TOT | IGA, True, mpdata.KERNEL_AUTO),
    ("resident1d", (300,), 0, 3, FCT, False, mpdata.KERNEL_AUTO),
    ("kahan_fused2d", (70, 150), 0, 2, FCT | mpdata.OPT_KAHAN, False, mpdata.KERNEL_AUTO),
]


def _family_inputs(shape, bc, opts, with_g, seed=5):
    gen = synth.rng(seed)
    nd = len(shape)
    g = gen.uniform(0.7, 1.3, size=shape) if with_g else None
    if nd == 1:
        c = [np.full(shape[0] + 1, 0.41)]
    elif bc == 0:
        c = synth.small_advector(shape, 0.5, gen, g=g)
    else:
        c = synth.random_advector(shape, 0.4, gen)
    m = min(shape)
    psi = synth.blob_field(shape, 5, (m / 8, m / 3), "normal" if opts & IGA else "uniform", gen,
                           periodic=(bc == 0)) + (0.0 if opts & IGA else 0.1)
    return psi, c, g


@pytest.mark.parametrize("where", ["psi", "wall"])
@pytest.mark.parametrize("value", [np.nan, np.inf, -np.inf], ids=["nan", "inf", "-inf"])
@pytest.mark.parametrize("name,shape,bc,n_iters,opts,with_g,kernel", FAMILIES,
                         ids=[f[0] for f in FAMILIES])
def test_nonfinite_reaches_diag(name, shape, bc, n_iters, opts, with_g, kernel, value, where):
    psi, c, g = _family_inputs(shape, bc, opts, with_g)
    plan = mpdata.Plan(shape, n_iters=n_iters, opts=opts, bc=bc, has_g=with_g, kernel=kernel)
    gd = dev(g, torch.float64)
    cd = [dev(x, torch.float64) for x in c]
    # the clean run is finite
    p = dev(psi, torch.float64)
    plan.step(p, cd, g=gd, n_steps=3)
    assert _diag_status(plan, p, gd) == (mpdata.OK, 0), name
    # one interior cell / one interior wall of the last dimension
    mid = tuple(s // 2 for s in shape)
    p = dev(psi, torch.float64)
    if where == "psi":
        p[mid] = value
    else:
        cd[-1][mid] = value
    plan.step(p, cd, g=gd, n_steps=3)
    rc, bad = _diag_status(plan, p, gd)
    assert rc == mpdata.ENONFINITE and bad >= 1, (name, rc, bad)
    if where == "wall":
        with pytest.raises(mpdata.MPDATAError) as ei:
            plan.courant_max(cd, g=gd)
        assert ei.value.code == mpdata.ENONFINITE


@pytest.mark.parametrize("where", ["psi", "wall"])
@pytest.mark.parametrize("value", [np.nan, np.inf], ids=["nan", "inf"])
def test_nonfinite_batched(value, where):
    """The batched launch: a non-finite value in one grid shows in that grid's
    cells after the steps (diag of the packed buffer as one 1-D field), and
    the other grids stay finite and equal to a clean run."""
    cases = synth.case_batch(grids=range(3), n_grids=3, lo=33, hi=90)
    shapes = [c.psi.shape for c in cases]
    bp = mpdata.BatchedPlan(shapes, dtype=torch.float32, n_iters=2, opts=FCT)
    psi = bp.pack([c.psi for c in cases], "psi")
    c0 = bp.pack([c.c[0] for c in cases], "c0")
    c1 = bp.pack([c.c[1] for c in cases], "c1")
    clean = psi.clone()
    bp.step(clean, c0, c1, n_steps=4)
    flat = mpdata.Plan((bp.n_psi,), dtype=torch.float32)
    assert _diag_status(flat, clean) == (mpdata.OK, 0)
    # grid 1, an interior cell / an interior wall
    psis = [x.psi.copy() for x in cases]
    walls = [x.c[0].copy() for x in cases]
    mid = (shapes[1][0] // 2, shapes[1][1] // 2)
    if where == "psi":
        psis[1][mid] = value
    else:
        walls[1][mid] = value
    p = bp.pack(psis, "psi")
    cc0 = bp.pack(walls, "c0")
    bp.step(p, cc0, c1, n_steps=4)
    rc, bad = _diag_status(flat, p)
    assert rc == mpdata.ENONFINITE and bad >= 1
    got = bp.unpack(p, "psi")
    ref = bp.unpack(clean, "psi")
    for k in (0, 2):
        assert torch.equal(got[k], ref[k]), k
