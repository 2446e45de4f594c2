"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar: relative L2 <= 1e-12 for the FP64 path and <= 1e-5 for the FP32 path
(the oracle consumes the FP32-rounded inputs widened to FP64).  Sizes span
several tiles with ragged tails; full workload sizes are checked on whole
fields where the oracle is fast enough and on sampled sub-blocks otherwise.
"""
import types

import numpy as np
import pytest
import torch

import oracle
from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import TOL, as_dtype, assert_parity, dev, gpu_run, rel_l2

pytestmark = pytest.mark.gpu

FCT, IGA, TOT = 1, 2, 4
OPTS = [0, FCT, TOT, FCT | TOT, IGA, IGA | FCT, IGA | TOT, IGA | TOT | FCT]
KERNELS = [mpdata.KERNEL_STAGED, mpdata.KERNEL_AUTO]
DTYPES = [torch.float64, torch.float32]


def _inputs(shape, bc, opts, seed, with_g):
    gen = synth.rng(seed)
    nd = len(shape)
    g = gen.uniform(0.6, 1.4, size=shape) if with_g else None
    if bc == 0:
        c = synth.small_advector(shape, 0.5, gen, g=g) if nd > 1 else [np.full(shape[0] + 1, 0.43)]
    else:
        c = synth.random_advector(shape, 0.45, gen)
    m = min(shape)
    psi = synth.blob_field(shape, 6, (m / 10, m / 4), "normal" if opts & (IGA | 8) else "uniform",
                           gen, periodic=(bc == 0))
    return psi, c, g


CASES = []
for shape in [(1000,), (150, 197), (37, 29, 41)]:
    for bc in (0, 1):
        for opts in OPTS:
            CASES.append((shape, bc, opts))


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("shape,bc,opts", CASES)
def test_parity_small(shape, bc, opts, dtype):
    n_iters = 2 if opts & IGA else 3
    with_g = (opts % 2 == 0)
    psi, c, g = _inputs(shape, bc, opts, seed=len(shape) * 100 + bc * 10 + opts, with_g=with_g)
    psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
    n_steps = 5
    ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=n_steps)
    for kernel in KERNELS:
        out = gpu_run(psi, c, g, dtype, n_iters, opts, bc, n_steps, kernel=kernel)
        assert_parity(out, ref, dtype, kernel)


KAHAN = mpdata.OPT_KAHAN
KAHAN_CASES = []
for shape in [(300,), (150, 197), (37, 29, 41)]:
    for bc in (0, 1):
        for opts in (KAHAN, FCT | KAHAN, TOT | KAHAN, IGA | TOT | KAHAN):
            KAHAN_CASES.append((shape, bc, opts))


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("shape,bc,opts", KAHAN_CASES)
def test_parity_kahan(shape, bc, opts, dtype):
    """Kahan-compensated donor updates through every kernel family (staged,
    fused 2-D, resident 1-D), with and without G."""
    n_iters = 2 if opts & IGA else 3
    for with_g in (False, True):
        psi, c, g = _inputs(shape, bc, opts, seed=len(shape) * 100 + bc * 10 + opts + with_g,
                            with_g=with_g)
        psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
        ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=5)
        for kernel in KERNELS:
            out = gpu_run(psi, c, g, dtype, n_iters, opts, bc, 5, kernel=kernel)
            assert_parity(out, ref, dtype, (kernel, with_g))


ABS = mpdata.OPT_ABS
ABS_CASES = []
for shape in [(300,), (150, 197), (37, 29, 41)]:
    for bc in (0, 1):
        for opts in (ABS, ABS | FCT, ABS | TOT, ABS | TOT | FCT | KAHAN):
            ABS_CASES.append((shape, bc, opts))


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("shape,bc,opts", ABS_CASES)
def test_parity_abs(shape, bc, opts, dtype):
    """abs option (|psi| in the psi-fractions) on variable-sign fields through
    the staged, fused 2-D, one-pass 2-D, 3-D and resident 1-D kernels, with
    and without G."""
    for with_g in (False, True):
        psi, c, g = _inputs(shape, bc, opts, seed=len(shape) * 100 + bc * 10 + opts + with_g,
                            with_g=with_g)
        psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
        ref = oracle.step(psi, c, g=g, n_iters=3, opts=opts, bc=bc, n_steps=5)
        for kernel in KERNELS:
            out = gpu_run(psi, c, g, dtype, 3, opts, bc, 5, kernel=kernel)
            assert_parity(out, ref, dtype, (kernel, with_g))


DFL = mpdata.OPT_DFL
DFL_CASES = []
for shape in [(300,), (150, 197), (37, 29, 41)]:
    for bc in (0, 1):
        for opts in (DFL, DFL | FCT, DFL | TOT | IGA, DFL | TOT | FCT | KAHAN):
            DFL_CASES.append((shape, bc, opts))


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("shape,bc,opts", DFL_CASES)
def test_parity_dfl(shape, bc, opts, dtype):
    """Divergent-flow term through the staged, one-pass 2-D, 3-D and
    resident 1-D kernels, on divergent (open) and non-divergent (periodic)
    advectors, with and without G."""
    n_iters = 2 if opts & IGA else 3
    for with_g in (False, True):
        psi, c, g = _inputs(shape, bc, opts, seed=len(shape) * 100 + bc * 10 + opts + with_g,
                            with_g=with_g)
        psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
        ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=5)
        for kernel in KERNELS:
            out = gpu_run(psi, c, g, dtype, n_iters, opts, bc, 5, kernel=kernel)
            assert_parity(out, ref, dtype, (kernel, with_g))


def test_abs_option_errors():
    with pytest.raises(mpdata.MPDATAError) as ei:
        mpdata.Plan((32, 32), n_iters=2, opts=ABS | IGA)
    assert ei.value.code == mpdata.EINVAL
    x = torch.zeros((32, 32), dtype=torch.float64, device="cuda")
    c = [torch.zeros((33, 32), dtype=torch.float64, device="cuda"),
         torch.zeros((32, 33), dtype=torch.float64, device="cuda")]
    for opts in (ABS, mpdata.OPT_DFL):
        plan = mpdata.Plan((32, 32), n_iters=2, opts=opts, adj_steps=2, ckpt_every=1)
        with pytest.raises(mpdata.MPDATAError) as ei:
            plan.adv_adj(x, c, x, n_steps=2, ckpt_every=1)
        assert ei.value.code == mpdata.EUNSUPPORTED


@pytest.mark.parametrize("n_iters", [1, 2, 3, 4])
def test_parity_pass_counts(n_iters):
    shape = (130, 70)
    psi, c, g = _inputs(shape, 0, FCT, seed=7, with_g=True)
    ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=FCT, n_steps=3)
    for kernel in KERNELS:
        out = gpu_run(psi, c, g, torch.float64, n_iters, FCT, 0, 3, kernel=kernel)
        assert_parity(out, ref, torch.float64)


def test_parity_1d_workload_full():
    """1-D periodic, nx=500, C=0.5, n_iters=2, 1000 steps: whole field."""
    case = synth.case_1d()
    ref = oracle.step(case.psi, case.c, n_iters=2, n_steps=case.n_steps)
    out = gpu_run(case.psi, case.c, None, torch.float64, 2, 0, 0, case.n_steps)
    assert_parity(out, ref, torch.float64)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_parity_2d_workload_full(dtype):
    """2-D periodic 2048^2, n_iters=3 with the limiter: whole field after 2
    steps at full size, in the launch configuration the benchmark times."""
    case = synth.case_2d()
    psi = as_dtype(case.psi, dtype)
    c = [as_dtype(x, dtype) for x in case.c]
    ref = oracle.step(psi, c, n_iters=3, opts=FCT, n_steps=2)
    out = gpu_run(psi, c, None, dtype, 3, FCT, 0, 2)
    assert_parity(out, ref, dtype)


def _subblock_check(case, out, dtype, n_steps, centres, half=6, step_radius=3):
    """Compare `out` with the oracle run on sub-blocks around `centres`; the
    block margin exceeds the domain of dependence (step_radius cells per
    step), so its own boundaries do not reach the compared core (real
    boundaries are kept)."""
    shape = case.psi.shape
    nd = len(shape)
    radius = step_radius * n_steps + 2
    errs = []
    for ctr in centres:
        lo = [max(0, ctr[d] - half - radius) if case.bc else ctr[d] - half - radius for d in range(nd)]
        hi = [min(shape[d], ctr[d] + half + radius + 1) if case.bc else ctr[d] + half + radius + 1
              for d in range(nd)]
        idx = [np.arange(lo[d], hi[d]) % shape[d] for d in range(nd)]
        ix = np.ix_(*idx)
        sub_psi = as_dtype(case.psi[ix], dtype)
        sub_g = as_dtype(case.g[ix], dtype) if case.g is not None else None
        sub_c = []
        for d in range(nd):
            wi = list(idx)
            wi[d] = np.arange(lo[d], hi[d] + 1) % (shape[d] + (1 if case.bc else 0))
            sub_c.append(as_dtype(case.c[d][np.ix_(*wi)], dtype))
        ref = oracle.step(sub_psi, sub_c, g=sub_g, n_iters=case.n_iters, opts=case.opts,
                          bc=case.bc, n_steps=n_steps)
        core = []
        for d in range(nd):
            a = max(lo[d], ctr[d] - half) - lo[d]
            b = min(hi[d], ctr[d] + half + 1) - lo[d]
            core.append(slice(a, b))
        got = out[ix][tuple(core)]
        errs.append(assert_parity(got, ref[tuple(core)], dtype, ctr)[0])
    return max(errs)


def test_parity_3d_workload_sampled():
    """3-D open 384x384x256 (G(z), tot + iga, n_iters=2): full-size GPU run,
    oracle on sub-blocks at corners, edges, faces and the interior."""
    case = synth.case_3d()
    n_steps = 2
    out = gpu_run(case.psi, case.c, case.g, torch.float64, 2, case.opts, 1, n_steps)
    s = case.psi.shape
    centres = [(0, 0, 0), (s[0] - 1, s[1] - 1, s[2] - 1), (0, s[1] // 2, s[2] - 1),
               (s[0] // 2, s[1] // 2, s[2] // 2), (s[0] - 3, 5, s[2] // 3), (100, 0, 128)]
    assert _subblock_check(case, out, torch.float64, n_steps, centres) <= 1e-12


@pytest.mark.parametrize("kernel", KERNELS)
def test_parity_2d_large_sampled(kernel):
    """Maximum-size check: a 16384 x 16390 periodic FP64 grid (2.1 GB per
    field, byte offsets far past 2^31, ragged last strip), n_iters=3 with the
    limiter, 2 steps; oracle on sub-blocks at the corners, edges and
    interior (dependence radius 5 cells per step)."""
    shape = (16384, 16390)
    gen = synth.rng(71)
    c = list(synth.stream_advector_2d(shape, 0.5, gen, n_modes=4, kmax=3))
    x0 = np.sin(2 * np.pi * 3 * (np.arange(shape[0]) + 0.5) / shape[0])
    x1 = np.cos(2 * np.pi * 5 * (np.arange(shape[1]) + 0.5) / shape[1])
    psi = 1.0 + 0.5 * np.outer(x0, x1)
    psi[1000:3000, 5000:9000] += 1.0          # sharp edges for the limiter
    case = types.SimpleNamespace(psi=psi, c=c, g=None, n_iters=3, opts=FCT, bc=0)
    n_steps = 2
    out = gpu_run(psi, c, None, torch.float64, 3, FCT, 0, n_steps, kernel=kernel)
    s = shape
    centres = [(0, 0), (s[0] - 1, s[1] - 1), (0, s[1] - 1), (s[0] - 1, 0), (1000, 5000),
               (2999, 8999), (s[0] // 2, s[1] // 2), (12345, 16389)]
    assert _subblock_check(case, out, torch.float64, n_steps, centres, step_radius=5) <= 1e-12


@pytest.mark.parametrize("shape,bc", [((3,), 0), ((1,), 1), ((3, 3), 0), ((1, 1), 1), ((2, 7), 1),
                                      ((3, 3, 3), 0), ((1, 2, 1), 1), ((6, 16, 64), 0)])
def test_degenerate_cases(shape, bc):
    """Degenerate inputs through every kernel family: the smallest grids each
    boundary type allows, psi == 0 (every psi-fraction is 0/0), a zero
    advector (identity), and a constant field in a non-divergent flow."""
    nd = len(shape)
    gen = synth.rng(81)
    walls = [tuple(n + (1 if e == d else 0) for e, n in enumerate(shape)) for d in range(nd)]
    for opts in (0, FCT, TOT | FCT, IGA | TOT, mpdata.OPT_KAHAN | FCT, mpdata.OPT_ABS | FCT,
                 mpdata.OPT_DFL | FCT):
        n_iters = 2 if opts & IGA else 3
        # psi == 0 stays 0 exactly
        c = [gen.uniform(-0.2 / nd, 0.2 / nd, size=w) for w in walls]
        if bc == 0:
            c = synth.periodic_fix(c)
        z = np.zeros(shape)
        for kernel in KERNELS:
            out = gpu_run(z, c, None, torch.float64, n_iters, opts, bc, 3, kernel=kernel)
            assert np.all(out == 0.0), (opts, kernel)
        # zero advector: identity
        psi = gen.uniform(0.1, 1.0, size=shape)
        c0 = [np.zeros(w) for w in walls]
        for kernel in KERNELS:
            out = gpu_run(psi, c0, None, torch.float64, n_iters, opts, bc, 3, kernel=kernel)
            assert np.array_equal(out, psi), (opts, kernel)
        # constant field, non-divergent advector, against the oracle
        if bc == 0 and min(shape) >= 3:
            cn = synth.small_advector(shape, 0.4, gen)
            k = np.full(shape, 0.75)
            ref = oracle.step(k, cn, n_iters=n_iters, opts=opts, bc=0, n_steps=3)
            for kernel in KERNELS:
                out = gpu_run(k, cn, None, torch.float64, n_iters, opts, 0, 3, kernel=kernel)
                assert_parity(out, ref, torch.float64, (opts, kernel))
                assert np.max(np.abs(out - 0.75)) <= 1e-13, (opts, kernel)


def test_resume_is_bitwise():
    """Resumability (the paper's advance()): 3 + 4 steps == 7 steps, bit for bit."""
    case = synth.case_2d(n=192, n_steps=7)
    for kernel in KERNELS:
        plan = mpdata.Plan(case.psi.shape, n_iters=3, opts=FCT, kernel=kernel)
        c = [dev(x, torch.float64) for x in case.c]
        a = dev(case.psi, torch.float64)
        b = a.clone()
        plan.step(a, c, n_steps=7)
        plan.step(b, c, n_steps=3)
        plan.step(b, c, n_steps=4)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_gpu_invariants_conservation_and_bounds():
    """On the GPU path itself: sum(G psi) conserved (periodic) and, with the
    limiter, no new global extrema."""
    case = synth.case_2d(n=512, seed=9)
    plan = mpdata.Plan(case.psi.shape, n_iters=3, opts=FCT)
    c = [dev(x, torch.float64) for x in case.c]
    p = dev(case.psi, torch.float64)
    s0, mn0, mx0, bad0 = plan.diag(p)
    plan.step(p, c, n_steps=50)
    s1, mn1, mx1, bad1 = plan.diag(p)
    assert bad0 == bad1 == 0
    assert abs(s1 - s0) <= 1e-13 * abs(s0)
    assert mx1 <= mx0 and mn1 >= mn0 - 1e-15


def test_diag_matches_oracle():
    gen = synth.rng(5)
    shape = (333, 257)
    psi = gen.normal(size=shape)
    g = gen.uniform(0.5, 2.0, size=shape)
    plan = mpdata.Plan(shape, has_g=True)
    s, mn, mx, bad = plan.diag(dev(psi, torch.float64), dev(g, torch.float64))
    rs, rmn, rmx, rbad = oracle.diag(psi, g)
    assert abs(s - rs) <= 1e-14 * np.sum(np.abs(g * psi)) and (mn, mx, bad) == (rmn, rmx, rbad)
    psi[3, 5] = np.nan
    psi[100, 7] = np.inf
    s, mn, mx, bad = plan.diag(dev(psi, torch.float64), dev(g, torch.float64))
    assert bad == 2


def test_courant_max_matches_oracle():
    case = synth.case_3d(shape=(40, 36, 28))
    plan = mpdata.Plan(case.psi.shape, n_iters=2, opts=case.opts, bc=1, has_g=True)
    got = plan.courant_max([dev(x, torch.float64) for x in case.c], g=dev(case.g, torch.float64))
    ref = oracle.courant_max(case.psi.shape, case.c, g=case.g, bc=1)
    assert abs(got - ref) <= 1e-15 * ref


def test_step_argument_errors():
    plan = mpdata.Plan((64, 64))
    p = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
    c0 = torch.zeros(65, 64, dtype=torch.float64, device="cuda")
    c1 = torch.zeros(64, 65, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        plan.step(p, [c0])
    with pytest.raises(ValueError):
        plan.step(p, [c0, c1.float()])
    L = mpdata.lib()
    import ctypes
    rc = L.mpdata_step(plan._handle, ctypes.c_void_p(p.data_ptr()), None,
                       ctypes.c_void_p(c0.data_ptr()), None, None, 1)
    assert rc == mpdata.EINVAL
    rc = L.mpdata_step(plan._handle, ctypes.c_void_p(p.data_ptr()),
                       ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(c0.data_ptr()),
                       ctypes.c_void_p(c1.data_ptr()), None, 1)
    assert rc == mpdata.EINVAL          # g given to a plan without has_g


def test_zero_steps_is_identity():
    case = synth.case_2d(n=64)
    p = dev(case.psi, torch.float64)
    q = p.clone()
    mpdata.Plan(case.psi.shape, n_iters=3, opts=FCT).step(p, [dev(x, torch.float64) for x in case.c],
                                                          n_steps=0)
    torch.cuda.synchronize()
    assert torch.equal(p, q)


@pytest.mark.parametrize("shape", [(96, 80), (24, 20, 70), (300,)], ids=["2d", "3d", "1d"])
def test_timing_window(shape):
    """mpdata_timing brackets the next m step launches without changing the
    result; launches beyond m are not counted."""
    nd = len(shape)
    rng = np.random.default_rng(11)
    psi = rng.uniform(0.0, 1.0, size=shape)
    c = synth.periodic_fix(synth.random_advector(shape, 0.3, rng))
    opts = 0 if nd == 3 else FCT
    plan = mpdata.Plan(shape, n_iters=2, opts=opts, bc=mpdata.BC_PERIODIC)
    cd = [dev(x, torch.float64) for x in c]
    a = dev(psi, torch.float64)
    plan.step(a, cd, n_steps=4)
    b = dev(psi, torch.float64)
    plan.timing(3)
    plan.step(b, cd, n_steps=4)
    ms, n, name = plan.timing_read()
    plan.timing(0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert n == (1 if nd == 1 else 3)
    assert ms > 0.0 and name
    plan.timing(0)
    assert plan.timing_read()[1] == 0


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_fused_tile_rows_bitwise_independent(dtype):
    """The fused kernel's chunk length changes only the speed: every setting
    gives the same bits (and the staged path agrees to round-off)."""
    case = synth.case_2d(shape=(300, 211), seed=4, sigma=(8.0, 30.0))
    c = [dev(x, dtype) for x in case.c]
    plan = mpdata.Plan(case.psi.shape, dtype=dtype, n_iters=3, opts=FCT)
    ref = None
    for rows in (0, 1, 7, 16, 33, 64, 299, 300, 1000):
        plan.set_tile_rows(rows)
        p = dev(case.psi, dtype)
        plan.step(p, c, n_steps=3)
        torch.cuda.synchronize()
        if ref is None:
            ref = p
        assert torch.equal(p, ref), rows
    tuned = plan.autotune(dev(case.psi, dtype), c)
    assert tuned > 0
    p = dev(case.psi, dtype)
    plan.step(p, c, n_steps=3)
    torch.cuda.synchronize()
    assert torch.equal(p, ref)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("opts", OPTS)
def test_parity_1d_resident(opts, bc, dtype):
    """1-D grids small enough for the LDS-resident kernel (all steps of a
    call in one launch), every option, with and without G."""
    n_iters = 2 if opts & IGA else 3
    for with_g in (False, True):
        psi, c, g = _inputs((300,), bc, opts, seed=40 + opts + bc, with_g=with_g)
        if bc == 0:
            c = [np.full(301, -0.37)]
        psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
        ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=25)
        out = gpu_run(psi, c, g, dtype, n_iters, opts, bc, 25, kernel=mpdata.KERNEL_FUSED)
        assert_parity(out, ref, dtype, with_g)


F3_CASES = []
for shape, bc in [((9, 37, 130), 1), ((10, 16, 64), 0), ((7, 45, 70), 0), ((12, 20, 67), 1)]:
    for n_iters, opts in [(1, 0), (2, 0), (2, TOT), (2, IGA), (2, IGA | TOT), (2, IGA | TOT | 32),
                          (2, 8), (2, 8 | TOT), (2, 16), (2, 16 | IGA | TOT), (1, 8 | 16)]:
        F3_CASES.append((shape, bc, n_iters, opts))


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("shape,bc,n_iters,opts", F3_CASES)
def test_parity_3d_fused(shape, bc, n_iters, opts, dtype):
    """3-D two-pass steps through the donor + corrective kernel pair (several
    (j, k) tiles with ragged edges, marching chunks along i), with and
    without G, against the oracle and against the staged path."""
    for with_g in (True, False):
        psi, c, g = _inputs(shape, bc, opts, seed=300 + opts + 10 * bc, with_g=with_g)
        psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
        ref = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=3)
        fused = gpu_run(psi, c, g, dtype, n_iters, opts, bc, 3, kernel=mpdata.KERNEL_FUSED)
        staged = gpu_run(psi, c, g, dtype, n_iters, opts, bc, 3, kernel=mpdata.KERNEL_STAGED)
        assert_parity(fused, ref, dtype, with_g)
        assert_parity(fused, staged, dtype, with_g)


def test_3d_fused_chunk_independent():
    """Planes per chunk change only the speed (bit for bit)."""
    case = synth.case_3d(shape=(40, 36, 70))
    c = [dev(x, torch.float64) for x in case.c]
    g = dev(case.g, torch.float64)
    plan = mpdata.Plan(case.psi.shape, n_iters=2, opts=case.opts, bc=1, has_g=True)
    ref = None
    for planes in (0, 1, 5, 17, 40):
        plan.set_tile_rows(planes)
        p = dev(case.psi, torch.float64)
        plan.step(p, c, g=g, n_steps=2)
        torch.cuda.synchronize()
        if ref is None:
            ref = p
        assert torch.equal(p, ref), planes
