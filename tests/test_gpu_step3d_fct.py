"""3-D steps with the limiter or more than two passes: the one-launch 3-D
kernel forms each pass's raw pseudo-velocities (pass 2 from the donor pass
it forms itself, later passes from the previous result) and writes them,
then the limiter coefficients and the limited corrective pass run as two
cell kernels (without the limiter, the corrective pass alone).  Against the oracle
(every element within the element-wise bar): every option mix with and
without G, both boundary types and mixed ones, tiles and plane chunks with
ragged tails, FP64 and FP32, and a larger grid; the abs option (|psi| in
the psi-fractions, on variable-sign fields) and the divergent-flow term
included."""
import numpy as np
import pytest
import torch

import oracle
from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import as_dtype, assert_parity, dev, rel_l2

pytestmark = pytest.mark.gpu
FCT, IGA, TOT, KAHAN = mpdata.OPT_FCT, mpdata.OPT_IGA, mpdata.OPT_TOT, mpdata.OPT_KAHAN
ABS, DFL = mpdata.OPT_ABS, mpdata.OPT_DFL


def _case(shape, bcs, opts, with_g, seed):
    gen = synth.rng(seed)
    g = gen.uniform(0.7, 1.3, size=shape) if with_g else None
    c = synth.random_advector(shape, 0.3, gen)
    for d, b in enumerate(bcs):                     # periodic: shared edge wall
        if b == 0:
            hi = [slice(None)] * 3
            lo = [slice(None)] * 3
            hi[d], lo[d] = -1, 0
            c[d][tuple(hi)] = c[d][tuple(lo)]
    m = min(shape)
    signed = opts & (IGA | ABS)
    psi = synth.blob_field(shape, 4, (m / 6, m / 3), "normal" if signed else "uniform", gen,
                           periodic=False) + (0.0 if signed else 0.05)
    return psi, c, g


def _run(psi, c, g, bcs, opts, dtype, n_steps, kernel=mpdata.KERNEL_AUTO, n_iters=2):
    plan = mpdata.Plan(psi.shape, dtype=dtype, n_iters=n_iters, opts=opts, bc=list(bcs),
                       has_g=g is not None, kernel=kernel)
    p = dev(psi, dtype)
    plan.timing(1)
    plan.step(p, [dev(x, dtype) for x in c], g=dev(g, dtype), n_steps=n_steps)
    name = plan.timing_read()[2]
    plan.timing(0)
    torch.cuda.synchronize()
    return p.double().cpu().numpy(), name


OPTS = [FCT, FCT | IGA, FCT | TOT, FCT | TOT | IGA, FCT | KAHAN, FCT | TOT | IGA | KAHAN,
        FCT | ABS, FCT | ABS | TOT, FCT | DFL, FCT | DFL | TOT | IGA]
CASES = [((12, 11, 10), (1, 1, 1)), ((37, 45, 70), (1, 1, 1)), ((20, 33, 65), (0, 0, 0)),
         ((23, 17, 40), (1, 0, 1)), ((200, 20, 33), (0, 1, 0))]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("with_g", [False, True], ids=["g1", "g"])
@pytest.mark.parametrize("opts", OPTS)
@pytest.mark.parametrize("shape,bcs", CASES, ids=lambda v: "x".join(map(str, v)))
def test_step3d_fct_vs_oracle(shape, bcs, opts, with_g, dtype):
    psi, c, g = _case(shape, bcs, opts, with_g, seed=sum(shape) + opts)
    psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
    ref = oracle.step(psi, c, g=g, n_iters=2, opts=opts, bc=list(bcs), n_steps=3)
    out, name = _run(psi, c, g, bcs, opts, dtype, 3)
    assert name == "k_step3d", name
    assert_parity(out, ref, dtype, f"{shape} {bcs} opts={opts}")


def test_step3d_fct_larger_grid():
    """96 x 128 x 80 open, the 3-D recipe's G(z) and advector with the
    limiter added, 4 steps against the oracle (its OpenMP build)."""
    case = synth.case_3d(shape=(96, 128, 80), sigma=(2.0, 8.0), seed=9)
    opts = case.opts | FCT
    ref = oracle.step(case.psi, case.c, g=case.g, n_iters=2, opts=opts, bc=1, n_steps=4,
                      parallel=True)
    out, name = _run(case.psi, case.c, case.g, (1, 1, 1), opts, torch.float64, 4)
    assert name == "k_step3d", name
    assert_parity(out, ref, torch.float64, "96x128x80 tot+iga+fct")


def test_step3d_fct_close_to_staged():
    """The stage-by-stage path computes the same quantities (its
    pseudo-velocities' 1 / mean G is an IEEE quotient, the one-launch
    kernel's a refined reciprocal): the two agree to rounding (relative L2:
    a limiter decision taken on the other side of a tie would show as one
    cell's deviation, which the norm bounds without failing on)."""
    psi, c, g = _case((30, 40, 50), (1, 1, 1), FCT | TOT | IGA, True, seed=3)
    a, _ = _run(psi, c, g, (1, 1, 1), FCT | TOT | IGA, torch.float64, 3)
    b, name = _run(psi, c, g, (1, 1, 1), FCT | TOT | IGA, torch.float64, 3,
                   kernel=mpdata.KERNEL_STAGED)
    assert name == "staged step"
    assert rel_l2(a, b) <= 1e-13


@pytest.mark.parametrize("n_iters", [3, 4])
@pytest.mark.parametrize("with_g", [False, True], ids=["g1", "g"])
@pytest.mark.parametrize("opts", [0, FCT, TOT, FCT | TOT, FCT | KAHAN, ABS | FCT, DFL | FCT,
                                  DFL | TOT])
@pytest.mark.parametrize("shape,bcs", [((23, 17, 40), (1, 0, 1)), ((130, 21, 34), (0, 0, 0)),
                                       ((15, 36, 33), (1, 1, 1))],
                         ids=lambda v: "x".join(map(str, v)))
def test_step3d_more_passes_vs_oracle(shape, bcs, opts, with_g, n_iters):
    """Three and four passes: each later pass reads the previous result and
    takes the previous pass's limited (or raw) velocities as its advector."""
    psi, c, g = _case(shape, bcs, opts, with_g, seed=sum(shape) + 3 * opts + n_iters)
    ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=list(bcs), n_steps=3)
    out, name = _run(psi, c, g, bcs, opts, torch.float64, 3, n_iters=n_iters)
    assert name == "k_step3d", name
    assert_parity(out, ref, torch.float64, f"{shape} {bcs} opts={opts} n_iters={n_iters}")


@pytest.mark.parametrize("n_iters,opts", [(2, TOT | IGA), (2, FCT | TOT), (3, FCT), (3, DFL | FCT)])
@pytest.mark.parametrize("shape,bcs", [((3, 17, 40), (0, 0, 0)), ((3, 9, 70), (0, 1, 1)),
                                       ((4, 20, 33), (0, 1, 0)), ((1, 20, 33), (1, 1, 1)),
                                       ((2, 35, 36), (1, 0, 1))],
                         ids=lambda v: "x".join(map(str, v)))
def test_step3d_thin_first_dimension_vs_oracle(shape, bcs, n_iters, opts):
    """The fewest planes each boundary type allows along the marching
    dimension (3 periodic, 1 and 2 open): every plane of a chunk is near
    both ends, so the plane map's wrap or clamp and the ring slots of the
    warm-up and drain planes all come into play."""
    psi, c, g = _case(shape, bcs, opts, True, seed=sum(shape) + opts + n_iters)
    ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=list(bcs), n_steps=3)
    out, name = _run(psi, c, g, bcs, opts, torch.float64, 3, n_iters=n_iters)
    assert name == "k_step3d", name
    assert_parity(out, ref, torch.float64, f"{shape} {bcs} opts={opts} n_iters={n_iters}")
