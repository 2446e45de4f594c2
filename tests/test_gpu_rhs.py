"""Source terms (euler_a / euler_b / trapez, Sect. 4.1) and the translating
oscillator (Sect. 4.3) through the C ABI against the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import TOL, as_dtype, dev, rel_l2

pytestmark = pytest.mark.gpu
FCT, IGA = 1, 2


def _case(shape, seed, with_g):
    gen = synth.rng(seed)
    c = synth.small_advector(shape, 0.45, gen) if len(shape) > 1 else [np.full(shape[0] + 1, 0.4)]
    g = gen.uniform(0.7, 1.3, size=shape) if with_g else None
    psi = gen.uniform(0.2, 1.0, size=shape)
    return gen, psi, c, g


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape,with_g", [((300,), False), ((150, 197), False), ((150, 197), True),
                                          ((20, 17, 70), True)])
@pytest.mark.parametrize("scheme", ["euler_a", "euler_b", "trapez"])
def test_step_rhs_vs_oracle(scheme, shape, with_g, dtype):
    gen, psi, c, g = _case(shape, 5 + len(shape), with_g)
    r0 = gen.normal(scale=0.1, size=shape)
    r1 = gen.normal(scale=0.1, size=shape)
    dt = 0.7
    kw = {"euler_a": dict(r_post=r0, a_post=dt), "euler_b": dict(r_pre=r0, a_pre=dt),
          "trapez": dict(r_pre=r0, a_pre=dt / 2, r_post=r1, a_post=dt / 2)}[scheme]
    psi, c, g = as_dtype(psi, dtype), [as_dtype(x, dtype) for x in c], as_dtype(g, dtype)
    kwo = {k: (as_dtype(v, dtype) if isinstance(v, np.ndarray) else v) for k, v in kw.items()}
    ref = oracle.step_rhs(psi, c, g=g, n_iters=3, opts=FCT, **kwo)
    plan = mpdata.Plan(shape, dtype=dtype, n_iters=3, opts=FCT, has_g=with_g)
    p = dev(psi, dtype)
    kwd = {k: (dev(v, dtype) if isinstance(v, np.ndarray) else v) for k, v in kwo.items()}
    plan.step_rhs(p, [dev(x, dtype) for x in c], g=dev(g, dtype), **kwd)
    torch.cuda.synchronize()
    assert rel_l2(p.double().cpu().numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", [(201,), (96, 80)])
def test_oscillator_vs_oracle(shape, dtype):
    """The translating oscillator of the paper's example (C = 0.5, omega =
    2 pi / 400, dt = 1, iga + fct) on a smaller grid, 60 steps."""
    n = shape[0]
    x = np.arange(n, dtype=np.float64)
    prof = np.where((x > n / 4) & (x < n / 2), 0.5 * (1 + np.cos(2 * np.pi * (x - 3 * n / 8) / (n / 4))), 0.0)
    if len(shape) == 1:
        psi = prof
        c = [np.full(n + 1, 0.5)]
    else:
        psi = np.outer(prof, np.ones(shape[1]))
        c = synth.small_advector(shape, 0.5, synth.rng(3))
    phi = np.zeros(shape)
    a = 0.5 * 1.0 * 2 * np.pi / 400
    psi, phi, c = as_dtype(psi, dtype), as_dtype(phi, dtype), [as_dtype(v, dtype) for v in c]
    rx, ry = oracle.osc_step(psi, phi, c, a, n_iters=2, opts=IGA | FCT, n_steps=60)
    plan = mpdata.Plan(shape, dtype=dtype, n_iters=2, opts=IGA | FCT)
    p, q = dev(psi, dtype), dev(phi, dtype)
    plan.osc_step(p, q, [dev(v, dtype) for v in c], a, n_steps=60)
    torch.cuda.synchronize()
    assert rel_l2(p.double().cpu().numpy(), rx) <= TOL[dtype]
    assert rel_l2(q.double().cpu().numpy(), ry) <= TOL[dtype]


def test_rhs_argument_errors():
    plan = mpdata.Plan((16, 16), n_iters=2, opts=FCT)
    p = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    c = [torch.zeros((17, 16), dtype=torch.float64, device="cuda"),
         torch.zeros((16, 17), dtype=torch.float64, device="cuda")]
    L = mpdata.lib()
    rc = L.mpdata_osc_step(plan._handle, ctypes.c_void_p(p.data_ptr()),
                           ctypes.c_void_p(p.data_ptr()), None, ctypes.c_void_p(c[0].data_ptr()),
                           ctypes.c_void_p(c[1].data_ptr()), None, 0.1, 1)
    assert rc == mpdata.EINVAL
    rc = L.mpdata_step_rhs(plan._handle, None, None, ctypes.c_void_p(c[0].data_ptr()),
                           ctypes.c_void_p(c[1].data_ptr()), None, None, 0.0, None, 0.0)
    assert rc == mpdata.EINVAL


@pytest.mark.parametrize("kind", ["osc", "plain"])
def test_resident_1d_large_lds(kind):
    """1-D grids whose resident working set exceeds 64 KB of LDS (gfx950 gives
    a workgroup up to 160 KB): the paper's 1001-cell oscillator and a
    1500-cell plain run go through the single-launch resident kernel and
    match the oracle."""
    if kind == "osc":
        case = synth.case_osc(n_steps=150)
        a = case.extra["a"]
        plan = mpdata.Plan(case.psi.shape, n_iters=2, opts=case.opts)
        p, q = dev(case.psi, torch.float64), dev(case.extra["phi"], torch.float64)
        c = [dev(x, torch.float64) for x in case.c]
        plan.timing(1)
        plan.osc_step(p, q, c, a, n_steps=case.n_steps)
        _, n_launch, name = plan.timing_read()
        rx, ry = oracle.osc_step(case.psi, case.extra["phi"], case.c, a, n_iters=2,
                                 opts=case.opts, n_steps=case.n_steps)
        assert name == "k_resident1d" and n_launch == 1
        # the pair's norm (phi alone passes through zero every half period)
        got = np.concatenate([p.cpu().numpy(), q.cpu().numpy()])
        assert rel_l2(got, np.concatenate([rx, ry])) <= 1e-12
    else:
        n = 1500
        gen = synth.rng(99)
        psi = gen.uniform(0.0, 1.0, size=n)
        c = [np.full(n + 1, -0.35)]
        plan = mpdata.Plan((n,), n_iters=3, opts=FCT | mpdata.OPT_TOT)
        p = dev(psi, torch.float64)
        plan.timing(1)
        plan.step(p, [dev(c[0], torch.float64)], n_steps=300)
        _, n_launch, name = plan.timing_read()
        ref = oracle.step(psi, c, n_iters=3, opts=FCT | mpdata.OPT_TOT, n_steps=300)
        assert name == "k_resident1d" and n_launch == 1
        assert rel_l2(p.cpu().numpy(), ref) <= 1e-12
