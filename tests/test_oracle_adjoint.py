"""Pins of the oracle's hand-written reverse mode (an extension of the
method, not in the paper).

* Linear cases (donor cell only; infinite gauge without the limiter): the
  step is a linear map L of psi, so <L^T lam, v> == <lam, L v> to round-off.
* Every option: the directional derivative from the adjoint equals central
  finite differences of the forward oracle (the misfit J = 1/2 ||psi_T -
  psi_obs||^2), for psi-only, advector-only and joint directions.  A
  direction whose one-sided differences disagree (a kink of the limiter or
  of [u]^+- straddled) is redrawn.
* The gradient does not depend on the checkpoint interval (bitwise).
"""
import numpy as np
import pytest

import oracle
from paper_1407_1309_amd import synth

FCT, IGA, TOT = oracle.OPT_FCT, oracle.OPT_IGA, oracle.OPT_TOT


def _setup(shape, bc, opts, seed, with_g=True):
    gen = synth.rng(seed)
    nd = len(shape)
    g = gen.uniform(0.7, 1.3, size=shape) if with_g else None
    c = synth.random_advector(shape, 0.4, gen)
    if bc == 0:
        c = synth.periodic_fix(c)
    m = min(shape)
    psi = synth.blob_field(shape, 4, (m / 6, m / 3), "normal" if opts & IGA else "uniform", gen,
                           periodic=(bc == 0)) + (0.0 if opts & IGA else 0.05)
    return gen, psi, c, g


@pytest.mark.parametrize("shape,bc", [((40,), 0), ((12, 10), 0), ((12, 10), 1), ((6, 5, 7), 0),
                                      ((6, 5, 7), 1)])
@pytest.mark.parametrize("n_iters,opts", [(1, 0), (2, IGA), (2, IGA | TOT)])
def test_dot_product_linear(shape, bc, n_iters, opts):
    gen, psi, c, g = _setup(shape, bc, opts, seed=3)
    lam = gen.normal(size=shape)
    v = gen.normal(size=shape)
    n_steps = 4
    gpsi, _ = oracle.adjoint(psi, c, lam, g=g, n_iters=n_iters, opts=opts, bc=bc,
                             n_steps=n_steps, ckpt_every=2)
    Lv = oracle.step(v, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=n_steps)
    a, b = np.vdot(gpsi, v), np.vdot(lam, Lv)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def _J(psi, c, g, obs, kw):
    out = oracle.step(psi, c, g=g, **kw)
    return 0.5 * np.sum((out - obs) ** 2), out


def _central(psi, c, g, obs, kw, dpsi, dc, h):
    Jp, _ = _J(psi + h * dpsi, [a + h * b for a, b in zip(c, dc)], g, obs, kw)
    Jm, _ = _J(psi - h * dpsi, [a - h * b for a, b in zip(c, dc)], g, obs, kw)
    return (Jp - Jm) / (2 * h)


def _fd_check(psi, c, g, obs, kw, dpsi, dc, grad_psi, grad_c, gen, tries=4):
    """Central difference along (dpsi, dc).  A smooth J makes the central
    difference converge like h^2; if the values at h and h/4 disagree the
    direction straddles a kink (limiter or [u]^+- switch) and is redrawn."""
    for _ in range(tries):
        scale = np.sqrt(np.sum(psi ** 2) + sum(np.sum(x ** 2) for x in c))
        dn = np.sqrt(np.sum(dpsi ** 2) + sum(np.sum(x ** 2) for x in dc))
        h = 1e-5 * scale / dn
        fd = _central(psi, c, g, obs, kw, dpsi, dc, h)
        fd4 = _central(psi, c, g, obs, kw, dpsi, dc, h / 4)
        ad = np.vdot(grad_psi, dpsi) + sum(np.vdot(a, b) for a, b in zip(grad_c, dc))
        if abs(fd - fd4) > 1e-7 * max(abs(fd), abs(fd4)):
            dpsi = gen.normal(size=psi.shape) if np.any(dpsi) else dpsi
            dc = [gen.normal(size=x.shape) if np.any(x) else x for x in dc]
            if kw.get("bc", 0) == 0:
                dc = synth.periodic_fix(dc)
            continue
        return fd4, ad
    pytest.skip("every direction straddled a kink")


CASES = []
for shape, bc in [((30,), 0), ((30,), 1), ((10, 9), 0), ((10, 9), 1), ((6, 5, 5), 0), ((5, 6, 5), 1)]:
    for n_iters, opts in [(2, 0), (3, FCT), (2, FCT), (3, TOT), (2, TOT | FCT), (2, IGA),
                          (2, IGA | FCT), (2, IGA | TOT | FCT)]:
        CASES.append((shape, bc, n_iters, opts))


@pytest.mark.parametrize("shape,bc,n_iters,opts", CASES)
@pytest.mark.parametrize("which", ["psi", "c", "joint"])
def test_adjoint_vs_central_fd(shape, bc, n_iters, opts, which):
    gen, psi, c, g = _setup(shape, bc, opts, seed=len(shape) * 10 + bc + opts)
    kw = dict(n_iters=n_iters, opts=opts, bc=bc, n_steps=3)
    obs = oracle.step(psi * 1.05 + 0.01, c, g=g, **kw)
    _, out = _J(psi, c, g, obs, kw)
    gpsi, gc = oracle.adjoint(psi, c, out - obs, g=g, n_iters=n_iters, opts=opts, bc=bc,
                              n_steps=3, ckpt_every=2)
    dpsi = gen.normal(size=shape) if which in ("psi", "joint") else np.zeros(shape)
    dc = [gen.normal(size=x.shape) if which in ("c", "joint") else np.zeros(x.shape) for x in c]
    if bc == 0:
        dc = synth.periodic_fix(dc)
    fd, ad = _fd_check(psi, c, g, obs, kw, dpsi, dc, gpsi, gc, gen)
    assert abs(fd - ad) <= 1e-6 * max(abs(fd), abs(ad)), (fd, ad)


def test_adjoint_checkpoint_independent():
    gen, psi, c, g = _setup((14, 11), 0, FCT, seed=9)
    lam = gen.normal(size=psi.shape)
    ref = oracle.adjoint(psi, c, lam, g=g, n_iters=3, opts=FCT, n_steps=7, ckpt_every=7)
    for k in (1, 2, 3, 5):
        got = oracle.adjoint(psi, c, lam, g=g, n_iters=3, opts=FCT, n_steps=7, ckpt_every=k)
        np.testing.assert_array_equal(got[0], ref[0])
        for a, b in zip(got[1], ref[1]):
            np.testing.assert_array_equal(a, b)


def test_periodic_duplicate_wall_gradient_is_zero():
    gen, psi, c, g = _setup((9, 8), 0, FCT, seed=2)
    lam = gen.normal(size=psi.shape)
    _, gc = oracle.adjoint(psi, c, lam, g=g, n_iters=2, opts=FCT, n_steps=2)
    assert np.all(gc[0][-1, :] == 0) and np.all(gc[1][:, -1] == 0)
