"""The 2-D single-pass kernel (donor pass + one launch per corrective pass)
against the oracle: strip and chunk tails, the smallest grids, every
boundary combination and the options it takes (fct, iga, abs, dfl, Kahan,
third-order terms; n_iters 2 and 3), with G = 1 and with a variable G (also
at 2048^2)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import TOL, as_dtype, assert_parity, dev, rel_l2

pytestmark = pytest.mark.gpu
FCT, IGA, ABS, DFL, KAHAN, TOT = (mpdata.OPT_FCT, mpdata.OPT_IGA, mpdata.OPT_ABS, mpdata.OPT_DFL,
                                  mpdata.OPT_KAHAN, mpdata.OPT_TOT)
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


def _run(psi, c, bcs, opts, n_iters, n_steps, dtype, g=None):
    plan = mpdata.Plan(psi.shape, dtype=dtype, n_iters=n_iters, opts=opts, bc=list(bcs),
                       has_g=g is not None)
    p = dev(psi, dtype)
    cd = [dev(x, dtype) for x in c]
    plan.timing(1)
    plan.step(p, cd, g=dev(g, dtype), n_steps=n_steps)
    _, n, name = plan.timing_read()
    plan.timing(0)
    torch.cuda.synchronize()
    return p.double().cpu().numpy(), name


SHAPES = [(1, 1), (1, 5), (3, 1), (2, 64), (33, 59), (40, 60), (37, 61), (31, 62), (29, 63),
          (70, 118), (65, 119), (130, 177)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("opts", [IGA | FCT | DFL, FCT | DFL, TOT | FCT, TOT | IGA | FCT | DFL],
                         ids=["iga_fct_dfl", "fct_dfl", "tot_fct", "tot_iga_fct_dfl"])
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


def _g_field(shape, seed):
    """A smooth positive G (0.8..1.2) with a little noise."""
    gen = synth.rng(seed)
    i = np.arange(shape[0])[:, None] / shape[0]
    j = np.arange(shape[1])[None, :] / shape[1]
    return 1.0 + 0.15 * np.sin(2 * np.pi * i) * np.cos(2 * np.pi * j) + \
        0.05 * gen.uniform(-1.0, 1.0, size=shape)


G_OPTS = [0, FCT, IGA | FCT, FCT | DFL, ABS | FCT, KAHAN | FCT, IGA | DFL, KAHAN | IGA | FCT]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("bcs", BCS, ids=["oo", "op", "po", "pp"])
@pytest.mark.parametrize("opts", G_OPTS)
def test_pass2d_variable_g(opts, bcs, dtype):
    """G in the donor and corrective updates (divided by the cell's G), in
    the pseudo-velocities (the walls' mean G) and in the limiter's
    coefficients: every boundary combination, against the oracle with the
    same G; every element within the element-wise bar."""
    shape = (67, 131)
    psi, c = _inputs(shape, bcs, opts, seed=11 * opts + 5 * bcs[0] + bcs[1])
    g = _g_field(shape, seed=opts + 2 * bcs[0] + bcs[1])
    psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
    for n_iters in ([2] if opts & IGA else [2, 3]):
        ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=list(bcs), n_steps=3)
        out, name = _run(psi, c, bcs, opts, n_iters, 3, dtype, g=g)
        assert name == "k_pass2d", name
        assert_parity(out, ref, dtype, f"n_iters={n_iters}")


@pytest.mark.parametrize("bcs,opts,n_iters", [((PER, PER), FCT, 3), ((OPEN, OPEN), IGA | FCT | DFL, 2)],
                         ids=["periodic_fct_iters3", "open_iga_fct_dfl"])
def test_pass2d_variable_g_full_size(bcs, opts, n_iters):
    """2048^2 FP64 with a variable G: the whole field after 2 steps against
    the oracle."""
    shape = (2048, 2048)
    case = synth.case_2d()
    c = [x.copy() for x in case.c]
    g = _g_field(shape, seed=9)
    psi = case.psi if not opts & IGA else case.psi - 0.5 * case.psi.mean()
    ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=list(bcs), n_steps=2,
                      parallel=True)
    out, name = _run(psi, c, bcs, opts, n_iters, 2, torch.float64, g=g)
    assert name == "k_pass2d", name
    assert_parity(out, ref, torch.float64, "2048^2 with G")


T_OPTS = [TOT, TOT | FCT, TOT | IGA | FCT, TOT | FCT | DFL, TOT | ABS | FCT, TOT | KAHAN | FCT,
          TOT | IGA, TOT | IGA | DFL]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("with_g", [False, True], ids=["g1", "g"])
@pytest.mark.parametrize("bcs", BCS, ids=["oo", "op", "po", "pp"])
@pytest.mark.parametrize("opts", T_OPTS)
@pytest.mark.parametrize("shape", [(67, 131), (45, 58)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_pass2d_third_order(shape, opts, bcs, with_g, dtype):
    """The third-order terms (Sect. 3.1.2: the D and E terms of both
    pseudo-velocities), with and without G, every boundary combination,
    strip and chunk tails; against the oracle, every element within the
    element-wise bar."""
    psi, c = _inputs(shape, bcs, opts, seed=13 * opts + 3 * bcs[0] + bcs[1] + with_g)
    g = _g_field(shape, seed=opts + bcs[0]) if with_g else None
    psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
    for n_iters in ([2] if opts & IGA else [2, 3]):
        ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=list(bcs), n_steps=3)
        out, name = _run(psi, c, bcs, opts, n_iters, 3, dtype, g=g)
        assert name == "k_pass2d", name
        assert_parity(out, ref, dtype, f"n_iters={n_iters}")


@pytest.mark.parametrize("bcs,opts,n_iters", [((PER, PER), TOT | FCT, 3),
                                              ((OPEN, OPEN), TOT | IGA | FCT, 2)],
                         ids=["periodic_tot_fct_iters3", "open_tot_iga_fct"])
def test_pass2d_third_order_full_size(bcs, opts, n_iters):
    """2048^2 FP64 with the third-order terms and a variable G: the whole
    field after 2 steps against the oracle."""
    case = synth.case_2d()
    g = _g_field(case.psi.shape, seed=4)
    psi = case.psi if not opts & IGA else case.psi - 0.5 * case.psi.mean()
    ref = oracle.step(psi, case.c, g=g, n_iters=n_iters, opts=opts, bc=list(bcs), n_steps=2,
                      parallel=True)
    out, name = _run(psi, case.c, bcs, opts, n_iters, 2, torch.float64, g=g)
    assert name == "k_pass2d", name
    assert_parity(out, ref, torch.float64, "2048^2 tot with G")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n_iters,opts", [(2, FCT), (3, FCT), (3, FCT | KAHAN), (2, 0),
                                          (3, ABS | FCT)])
def test_pass_kernel_same_bits_as_fused(n_iters, opts, dtype):
    """Where both apply (2-D periodic, G = 1, no tot / iga / dfl) one launch
    per corrective pass gives the bits of the whole-step fused kernel: the
    adjoint recomputes its segments with the former (recording each pass)
    and takes its checkpoints -- like the caller's own forward run -- with
    the latter.  The 2048^2 step recipe and the adjoint's 1024^2 recipe, and
    a ragged grid."""
    cases = [synth.case_2d(), synth.case_adjoint(n=1024, n_steps=20)["case"],
             synth.case_2d(shape=(150, 131), seed=8, sigma=(6.0, 20.0))]
    for case in cases:
        psi = as_dtype(case.psi, dtype)
        c = [as_dtype(x, dtype) for x in case.c]
        outs = []
        for kernel, want in ((mpdata.KERNEL_FUSED, "k_fused2d"), (mpdata.KERNEL_PASS, "k_pass2d")):
            plan = mpdata.Plan(psi.shape, dtype=dtype, n_iters=n_iters, opts=opts,
                               kernel=kernel)
            p = dev(psi, dtype)
            cd = [dev(x, dtype) for x in c]
            plan.timing(1)
            plan.step(p, cd, n_steps=5)
            assert plan.timing_read()[2] == want
            plan.timing(0)
            outs.append(p)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1]), (psi.shape, float((outs[0] - outs[1]).abs().max()))


def test_pass_kernel_rejected_where_absent():
    with pytest.raises(mpdata.MPDATAError):
        mpdata.Plan((300,), n_iters=2, kernel=mpdata.KERNEL_PASS)
    with pytest.raises(mpdata.MPDATAError):
        mpdata.Plan((64, 64), n_iters=1, kernel=mpdata.KERNEL_PASS)


@pytest.mark.parametrize("with_g", [False, True], ids=["g1", "g"])
@pytest.mark.parametrize("bcs", [(PER, PER), (PER, OPEN)], ids=["pp", "po"])
@pytest.mark.parametrize("opts", [IGA | FCT | DFL, TOT | FCT, FCT | DFL, TOT | IGA | FCT])
@pytest.mark.parametrize("shape", [(3, 70), (4, 61), (5, 130)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_pass2d_few_periodic_rows(shape, opts, bcs, with_g):
    """Fewer periodic rows than a chunk's march: the rows a chunk loads wrap
    around the domain several times (the row map is carried from row to
    row), against the oracle with a non-constant field."""
    psi, c = _inputs(shape, bcs, opts, seed=shape[0] * 97 + opts + bcs[1] + with_g)
    g = _g_field(shape, seed=opts + shape[0]) if with_g else None
    for n_iters in ([2] if opts & IGA else [2, 3]):
        ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=list(bcs), n_steps=3)
        out, name = _run(psi, c, bcs, opts, n_iters, 3, torch.float64, g=g)
        assert name == "k_pass2d", name
        assert_parity(out, ref, torch.float64, f"{shape} n_iters={n_iters}")
