"""The 2-D single-pass kernel (donor pass + one launch per corrective pass)
against the oracle: strip and chunk tails, the smallest grids, every
boundary combination and the options it takes (fct, iga, abs, dfl, Kahan;
n_iters 2 and 3)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import TOL, as_dtype, dev, rel_l2

pytestmark = pytest.mark.gpu
FCT, IGA, ABS, DFL, KAHAN = (mpdata.OPT_FCT, mpdata.OPT_IGA, mpdata.OPT_ABS, mpdata.OPT_DFL,
                             mpdata.OPT_KAHAN)
OPEN, PER = mpdata.BC_OPEN, mpdata.BC_PERIODIC


def _inputs(shape, bcs, opts, seed):
    gen = synth.rng(seed)
    c = synth.random_advector(shape, 0.45, gen)        # divergent
    for d, b in enumerate(bcs):                        # periodic: shared edge wall
        if b == PER:
            idx = [slice(None)] * 2
            idx[d] = -1
            src = [slice(None)] * 2
            src[d] = 0
            c[d][tuple(idx)] = c[d][tuple(src)]
    psi = gen.uniform(-0.5, 1.0, size=shape) if opts & (IGA | ABS) else \
        gen.uniform(0.1, 1.0, size=shape)
    return psi, c


def _run(psi, c, bcs, opts, n_iters, n_steps, dtype):
    plan = mpdata.Plan(psi.shape, dtype=dtype, n_iters=n_iters, opts=opts, bc=list(bcs))
    p = dev(psi, dtype)
    cd = [dev(x, dtype) for x in c]
    plan.timing(1)
    plan.step(p, cd, n_steps=n_steps)
    _, n, name = plan.timing_read()
    plan.timing(0)
    torch.cuda.synchronize()
    return p.double().cpu().numpy(), name


SHAPES = [(1, 1), (1, 5), (3, 1), (2, 64), (33, 59), (40, 60), (37, 61), (31, 62), (29, 63),
          (70, 118), (65, 119), (130, 177)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("opts", [IGA | FCT | DFL, FCT | DFL], ids=["iga_fct_dfl", "fct_dfl"])
def test_pass2d_shapes_open(shape, opts):
    psi, c = _inputs(shape, (OPEN, OPEN), opts, seed=shape[0] * 1000 + shape[1] + opts)
    ref = oracle.step(psi, c, n_iters=2, opts=opts, bc=OPEN, n_steps=4)
    out, name = _run(psi, c, (OPEN, OPEN), opts, 2, 4, torch.float64)
    assert name == "k_pass2d"
    assert rel_l2(out, ref) <= TOL[torch.float64]
    assert np.abs(out - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)


OPTS = [0, FCT, IGA, IGA | FCT, DFL, IGA | DFL, ABS | FCT, ABS | FCT | DFL, KAHAN | FCT | DFL,
        KAHAN | IGA | FCT]
BCS = [(OPEN, OPEN), (OPEN, PER), (PER, OPEN), (PER, PER)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("bcs", BCS, ids=["oo", "op", "po", "pp"])
@pytest.mark.parametrize("opts", OPTS)
@pytest.mark.parametrize("shape", [(67, 131), (128, 59)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_pass2d_options_and_boundaries(shape, opts, bcs, dtype):
    psi, c = _inputs(shape, bcs, opts, seed=7 * opts + 3 * bcs[0] + bcs[1])
    psi, c = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c]
    iters = [2] if opts & IGA else [2, 3]
    for n_iters in iters:
        ref = oracle.step(psi, c, n_iters=n_iters, opts=opts, bc=list(bcs), n_steps=3)
        out, name = _run(psi, c, bcs, opts, n_iters, 3, dtype)
        fused = bcs == (PER, PER) and not (opts & (IGA | DFL))
        assert name == ("k_fused2d" if fused else "k_pass2d"), name
        assert rel_l2(out, ref) <= TOL[dtype], (n_iters, name)


def test_pass2d_matches_staged_bitwise_zero_and_identity():
    """psi == 0 stays 0 and a zero advector is the identity, exactly."""
    shape = (45, 70)
    for opts in (FCT | DFL, IGA | FCT | DFL, ABS | FCT):
        z = np.zeros(shape)
        gen = synth.rng(3)
        c = synth.random_advector(shape, 0.4, gen)
        out, name = _run(z, c, (OPEN, OPEN), opts, 2, 3, torch.float64)
        assert name == "k_pass2d" and not out.any()
        psi = gen.uniform(0.1, 1.0, size=shape)
        c0 = [np.zeros_like(x) for x in c]
        out, _ = _run(psi, c0, (OPEN, OPEN), opts, 2, 3, torch.float64)
        assert np.array_equal(out, psi)
