"""Stop flag of the step loop (the paper's solvers stop after the current
step when a flag is raised, Sect. 3.2): the cancelled call returns
ECANCELLED with psi at the last completed step, bit for bit the state a
plain run of that many steps reaches, on every kernel path."""
import threading
import time

import numpy as np
import pytest
import torch

from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
FCT, IGA, TOT, DFL, ABS = (mpdata.OPT_FCT, mpdata.OPT_IGA, mpdata.OPT_TOT, mpdata.OPT_DFL,
                           mpdata.OPT_ABS)

# (shape, bc, n_iters, opts, kernel family)
PATHS = [((128, 96), 0, 3, FCT, "k_fused2d"), ((96, 130), 1, 2, IGA | FCT | DFL, "k_pass2d"),
         ((20, 18, 70), 1, 3, FCT, "k_step3d"), ((20, 18, 70), 1, 3, ABS | FCT, "k_step3d"),
         ((96, 130), 1, 1, 0, "staged step"),
         ((300,), 0, 2, FCT, "k_resident1d"), ((12, 20, 70), 0, 2, IGA | TOT, "k_step3d")]


def _setup(shape, bc, opts, seed):
    gen = synth.rng(seed)
    if len(shape) == 1:
        c = [np.full(shape[0] + 1, 0.4)]
    elif bc == 0:
        c = synth.small_advector(shape, 0.45, gen)
    else:
        c = synth.random_advector(shape, 0.45, gen)
    psi = gen.uniform(-0.5, 1.0, size=shape) if opts & IGA else gen.uniform(0.1, 1.0, size=shape)
    return psi, c


@pytest.mark.parametrize("shape,bc,n_iters,opts,family", PATHS)
@pytest.mark.parametrize("n_steps", [4, 5])
def test_polled_run_equals_plain_run(shape, bc, n_iters, opts, family, n_steps):
    psi, c = _setup(shape, bc, opts, seed=len(shape) + n_steps)
    cd = [dev(x, torch.float64) for x in c]
    plan = mpdata.Plan(shape, n_iters=n_iters, opts=opts, bc=bc)
    a = dev(psi, torch.float64)
    plan.timing(1)
    plan.step(a, cd, n_steps=n_steps)
    assert plan.timing_read()[2] == family
    plan.timing(0)
    flag = np.zeros(1, dtype=np.int32)
    plan.set_cancel_flag(flag)
    b = dev(psi, torch.float64)
    plan.step(b, cd, n_steps=n_steps)
    assert plan.steps_done() == n_steps
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("shape,bc,n_iters,opts,family", PATHS)
def test_raised_flag_stops_before_the_first_step(shape, bc, n_iters, opts, family):
    psi, c = _setup(shape, bc, opts, seed=3)
    plan = mpdata.Plan(shape, n_iters=n_iters, opts=opts, bc=bc)
    flag = np.ones(1, dtype=np.int32)
    plan.set_cancel_flag(flag)
    b = dev(psi, torch.float64)
    with pytest.raises(mpdata.MPDATAError) as ei:
        plan.step(b, [dev(x, torch.float64) for x in c], n_steps=3)
    assert ei.value.code == mpdata.ECANCELLED
    assert plan.steps_done() == 0
    assert np.array_equal(b.cpu().numpy(), psi)
    plan.set_cancel_flag(None)
    plan.step(b, [dev(x, torch.float64) for x in c], n_steps=1)
    assert plan.steps_done() == 1


@pytest.mark.parametrize("shape,bc,opts", [((512, 512), 0, FCT), ((256, 300), 1, IGA | FCT)])
def test_flag_raised_mid_run(shape, bc, opts):
    """Another thread raises the flag while a long call runs: the call stops
    after the step in progress, and psi equals a plain run of the completed
    steps bit for bit (odd counts included: the state is copied back)."""
    psi, c = _setup(shape, bc, opts, seed=11)
    cd = [dev(x, torch.float64) for x in c]
    plan = mpdata.Plan(shape, n_iters=2, opts=opts, bc=bc)
    flag = np.zeros(1, dtype=np.int32)
    plan.set_cancel_flag(flag)
    b = dev(psi, torch.float64)
    n = 200000
    t = threading.Thread(target=lambda: (time.sleep(0.05), flag.__setitem__(0, 1)))
    t.start()
    with pytest.raises(mpdata.MPDATAError) as ei:
        plan.step(b, cd, n_steps=n)
    t.join()
    assert ei.value.code == mpdata.ECANCELLED
    done = plan.steps_done()
    assert 0 < done < n
    ref = mpdata.Plan(shape, n_iters=2, opts=opts, bc=bc)
    a = dev(psi, torch.float64)
    ref.step(a, cd, n_steps=done)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
