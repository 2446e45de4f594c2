"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the property it checks and the passage it rests on.  None of
them re-types the oracle's formulae: they use hand-derived worked examples,
closed forms (upwind scheme, Fourier amplification factors), invariants of the
method (conservation, sign preservation, constant-state preservation, exact
shifts, boundedness, homogeneity, linearity of the infinite gauge, the gauge
limit), symmetry, convergence orders, and an exact-rational second coding on
tiny grids.
"""
import json
import math
import os
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle
from paper_1407_1309_amd import synth
from tests.bruteforce import mpdata_exact

FCT, IGA, TOT = oracle.OPT_FCT, oracle.OPT_IGA, oracle.OPT_TOT
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL_OPTS = [0, FCT, TOT, FCT | TOT, IGA, IGA | FCT, IGA | TOT, IGA | TOT | FCT]
KAHAN = oracle.OPT_KAHAN
KAHAN_OPTS = [KAHAN, FCT | KAHAN, IGA | TOT | KAHAN, FCT | TOT | KAHAN]
ABS = oracle.OPT_ABS
ABS_OPTS = [ABS, ABS | FCT, ABS | TOT, ABS | TOT | FCT]
DFL = oracle.OPT_DFL
DFL_OPTS = [DFL, DFL | FCT, DFL | TOT, DFL | IGA | TOT | FCT]


def _fr(s):
    return float(Fraction(s))


# ---------------------------------------------------------------- worked example
def test_worked_example_1d():
    """Hand-derived one-step values (eqs. upstream, F, adf_vel; Sects. 3.1.4-3.1.5)."""
    gold = json.load(open(os.path.join(GOLDEN, "worked_1d.json")))
    psi0 = np.array(gold["psi0"], dtype=float)
    c = [np.full(5, 0.5)]
    p1 = oracle.step(psi0, c, n_iters=1)
    np.testing.assert_array_equal(p1, [_fr(s) for s in gold["psi1"]])
    for key, opts in (("basic", 0), ("fct", FCT), ("iga", IGA)):
        out = oracle.step(psi0, c, n_iters=2, opts=opts)
        np.testing.assert_allclose(out, [_fr(s) for s in gold[key]["psi2"]], rtol=0, atol=4e-16)


# ---------------------------------------------------------------- P1 upwind closed form
@pytest.mark.parametrize("cour", [0.3, -0.7, 1.0])
def test_donor_cell_is_upwind_1d(cour):
    """n_iters=1 is the first-order upwind scheme (eq. upstream with eq. F)."""
    gen = synth.rng(11)
    psi = gen.uniform(0.1, 2.0, size=37)
    out = oracle.step(psi, [np.full(38, cour)], n_iters=1)
    if cour > 0:
        ref = psi - cour * (psi - np.roll(psi, 1))
    else:
        ref = psi - cour * (np.roll(psi, -1) - psi)
    np.testing.assert_allclose(out, ref, rtol=4e-16, atol=4e-16)


def test_donor_cell_is_upwind_2d_variable_g():
    """Donor pass with divergent, sign-varying walls and variable G equals the
    upwind flux-form update computed with np.roll (periodic)."""
    gen = synth.rng(12)
    shape = (9, 7)
    psi = gen.uniform(0.1, 2.0, size=shape)
    g = gen.uniform(0.5, 2.0, size=shape)
    c = synth.periodic_fix(synth.random_advector(shape, 0.8, gen))
    out = oracle.step(psi, c, g=g, n_iters=1)
    tend = np.zeros(shape)
    for d in range(2):
        cd = np.take(c[d], range(shape[d]), axis=d)       # wall f (left wall of cell f)
        left = np.roll(psi, 1, axis=d)
        flux = np.maximum(cd, 0) * left + np.minimum(cd, 0) * psi
        tend += np.roll(flux, -1, axis=d) - flux
    np.testing.assert_allclose(out, psi - tend / g, rtol=1e-14, atol=1e-15)


# ---------------------------------------------------------------- brute force (P14)
def _to_frac_case(shape, bc, seed, with_g, sign):
    gen = synth.rng(seed)
    psi = gen.integers(1, 9, size=shape).astype(float)
    if sign:
        psi = psi - 5.0
    psi = psi / 8.0
    c = []
    for d in range(len(shape)):
        s = list(shape)
        s[d] += 1
        c.append(gen.integers(-3, 4, size=s).astype(float) / 16.0)
    if bc == 0:
        c = synth.periodic_fix(c)
    g = gen.integers(2, 6, size=shape).astype(float) / 4.0 if with_g else None
    return psi, c, g


def _dict(a):
    return {tuple(int(v) for v in idx): Fraction(float(a[idx])) for idx in np.ndindex(a.shape)}


BF_CASES = [((8,), 0), ((8,), 1), ((5, 4), 0), ((5, 4), 1), ((4, 3, 3), 0), ((3, 4, 3), 1)]
# exact rationals grow fast through the limiter's divisions: keep the number
# of passes x steps small in 2-D / 3-D


@pytest.mark.parametrize("shape,bc", BF_CASES)
@pytest.mark.parametrize("opts", ALL_OPTS + KAHAN_OPTS + ABS_OPTS + DFL_OPTS)
def test_bruteforce_exact(shape, bc, opts):
    """Oracle == exact-rational second coding, every option, 1/2/3-D, both BCs
    (variable-sign psi for the two variable-sign options, iga and abs)."""
    iga = bool(opts & IGA)
    n_iters = 2 if (iga or len(shape) == 3) else 3
    with_g = len(shape) != 1 or bc == 1
    psi, c, g = _to_frac_case(shape, bc, seed=hash((shape, bc, opts)) % 1000, with_g=with_g,
                              sign=iga or bool(opts & ABS))
    n_steps = 2 if len(shape) == 1 else 1
    exact = mpdata_exact(_dict(psi), [_dict(x) for x in c], _dict(g) if g is not None else None,
                         shape, bc, n_iters, bool(opts & FCT), iga, bool(opts & TOT), n_steps,
                         absf=bool(opts & ABS), dfl=bool(opts & DFL))
    ref = np.zeros(shape)
    for k, v in exact.items():
        ref[k] = float(v)
    out = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=n_steps)
    scale = max(1.0, np.abs(ref).max())
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-13 * scale)


# ------------------------------------------------- compensated donor summation
@pytest.mark.parametrize("shape", [(24, 20), (10, 9, 8)])
def test_kahan_donor_update_is_compensated(shape):
    """With the Kahan option the donor-cell update is Kahan's compensated sum
    of psi and the per-dimension terms -(F(i+1/2) - F(i-1/2)) (Sect. 3.1.1).
    Check against the exact rational sum of those terms (recomputed from
    eq. F in plain floats: one product per flux, one difference per
    dimension), correctly rounded: a compensated sum of three or four terms
    of very different size is within one ulp of it everywhere and equal to
    it almost everywhere.  The uncompensated left-to-right sum, as a foil,
    misses the rounded value in far more cells, so a lost or mis-signed
    compensation fails the test."""
    gen = synth.rng(41)
    nd = len(shape)
    psi = gen.uniform(1.0, 2.0, size=shape)
    c = synth.periodic_fix([gen.uniform(-0.2 / nd, 0.2 / nd, size=tuple(
        s + (1 if d == e else 0) for e, s in enumerate(shape))) for d in range(nd)])
    k = oracle.step(psi, c, n_iters=1, opts=KAHAN, n_steps=1)

    def flux(u, xl, xr):
        return (u if u > 0 else 0.0) * xl + (u if u < 0 else 0.0) * xr

    hit = hit_naive = 0
    worst = 0.0
    for idx in np.ndindex(shape):
        x = psi[idx]
        terms = []
        for d in range(nd):
            lo = list(idx)
            hi = list(idx)
            hi[d] += 1
            m = list(idx)
            m[d] = (idx[d] - 1) % shape[d]
            p = list(idx)
            p[d] = (idx[d] + 1) % shape[d]
            fhi = flux(c[d][tuple(hi)], x, psi[tuple(p)])
            flo = flux(c[d][tuple(lo)], psi[tuple(m)], x)
            terms.append(-(fhi - flo))
        exact = float(Fraction(x) + sum(Fraction(t) for t in terms))
        naive = x
        for t in terms:
            naive = naive + t
        hit += k[idx] == exact
        hit_naive += naive == exact
        worst = max(worst, abs(k[idx] - exact) / np.spacing(exact))
    n = np.prod(shape)
    assert worst <= 1.0
    assert hit >= 0.95 * n
    assert hit_naive <= 0.9 * n          # the foil shows the test discriminates


def test_kahan_changes_only_rounding():
    """Kahan summation changes results by round-off only, for every option."""
    gen = synth.rng(42)
    shape = (20, 18)
    psi = gen.uniform(0.0, 1.0, size=shape)
    c = synth.periodic_fix(synth.random_advector(shape, 0.4, gen))
    g = gen.uniform(0.5, 1.5, size=shape)
    for opts in ALL_OPTS:
        n_iters = 2 if opts & IGA else 3
        a = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, n_steps=4)
        b = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts | KAHAN, n_steps=4)
        assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a)), opts


# ------------------------------------------------------------- abs option
@pytest.mark.parametrize("opts", [0, FCT, TOT, FCT | TOT])
@pytest.mark.parametrize("shape,bc", [((60,), 0), ((20, 18), 1), ((9, 8, 7), 0)])
def test_abs_equals_basic_for_nonnegative_psi(opts, shape, bc):
    """With psi >= 0 everywhere |psi| = psi, so the abs option reduces to the
    basic scheme bit for bit (Sect. 3.1.5)."""
    gen = synth.rng(51)
    c = synth.random_advector(shape, 0.4, gen)
    if bc == 0:
        c = synth.periodic_fix(c)
    psi = gen.uniform(0.0, 1.0, size=shape)
    a = oracle.step(psi, c, n_iters=3, opts=opts, bc=bc, n_steps=4)
    b = oracle.step(psi, c, n_iters=3, opts=opts | ABS, bc=bc, n_steps=4)
    assert np.array_equal(a, b)


def test_abs_bounded_fractions_variable_sign():
    """For a variable-sign field the basic psi-fraction (x_R - x_L)/(x_R + x_L)
    is unbounded where psi changes sign; with |psi| it is at most 1.  A
    one-pass-plus-correction step of a field that crosses zero between
    neighbouring cells therefore stays within the donor-cell bounds scaled by
    the Courant number under abs, while the basic scheme overshoots."""
    n = 64
    psi = np.where(np.arange(n) % 2 == 0, 1.0, -0.999)
    c = [np.full(n + 1, 0.25)]
    basic = oracle.step(psi, c, n_iters=2, opts=0, n_steps=1)
    absr = oracle.step(psi, c, n_iters=2, opts=ABS, n_steps=1)
    assert np.max(np.abs(absr)) <= 1.0 + 1e-12
    assert np.max(np.abs(basic)) > 1.5


def test_abs_rejected_with_iga_and_in_reverse_mode():
    psi = np.ones(16)
    c = [np.full(17, 0.2)]
    with pytest.raises(ValueError):
        oracle.step(psi, c, n_iters=2, opts=ABS | IGA)
    with pytest.raises(ValueError):
        oracle.adjoint(psi, c, np.ones(16), n_iters=2, opts=ABS, n_steps=1)
    with pytest.raises(ValueError):
        oracle.adjoint(psi, c, np.ones(16), n_iters=2, opts=DFL, n_steps=1)


# ------------------------------------------------------------ dfl option
def _divergent_1d(N, opts, with_g=False, T=0.5, cour=0.4):
    """Periodic 1-D run with the divergent advector c = (0.5 + 0.3 sin(2 pi x))
    dt/dx at fixed Courant number, optionally with G = 1 + 0.4 cos(2 pi x);
    cell averages of a smooth positive profile."""
    dx = 1.0 / N
    dt = cour * dx / 0.8
    nt = int(round(T / dt))
    dt = T / nt
    u = 0.5 + 0.3 * np.sin(2 * np.pi * np.arange(N + 1) * dx)
    C = u * dt / dx
    C[-1] = C[0]
    xs = (np.arange(N * 16) + 0.5) * dx / 16
    prof = 1.0 + 0.5 * np.sin(2 * np.pi * xs) ** 2 + np.exp(-((xs - 0.5) / 0.1) ** 2)
    G = (1.0 + 0.4 * np.cos(2 * np.pi * xs)).reshape(N, 16).mean(1) if with_g else None
    return oracle.step(prof.reshape(N, 16).mean(1), [C], g=G, n_iters=2, opts=opts, n_steps=nt)


@pytest.mark.parametrize("with_g", [False, True])
@pytest.mark.parametrize("base", [0, IGA])
def test_dfl_restores_second_order_in_divergent_flow(with_g, base):
    """In a divergent flow the donor-cell truncation error has a term in the
    velocity divergence that the basic pseudo-velocity does not remove, so
    MPDATA drops towards first order; the divergent-flow term (Sect. 3.1.3)
    restores second order, also with variable G (products of two advector
    factors divided by the wall mean of G) and under iga (where the term is
    a unit-field flux and so carries the wall mean of psi).  Self-convergence
    against a 4096-cell run."""
    for opts, lo, hi in [(base | DFL, 1.85, 2.2), (base, 0.9, 1.6)]:
        ref = _divergent_1d(4096, opts, with_g)
        errs = []
        for N in (128, 256, 512):
            r = ref.reshape(N, 4096 // N).mean(1)
            errs.append(np.sqrt(np.mean((_divergent_1d(N, opts, with_g) - r) ** 2)))
        order = np.log2(errs[1] / errs[2])
        assert lo <= order <= hi, (opts, order)


@pytest.mark.parametrize("opts", [0, FCT, TOT, IGA])
def test_dfl_vanishes_for_nondivergent_advector(opts):
    """With two passes the corrective pass uses the input advector; for an
    exactly non-divergent one the divergent-flow term is zero and the result
    equals the basic scheme bit for bit."""
    gen = synth.rng(61)
    shape = (24, 20)
    c = synth.small_advector(shape, 0.5, gen)
    psi = gen.uniform(0.0, 1.0, size=shape)
    if opts & IGA:
        psi -= 0.5
    a = oracle.step(psi, c, n_iters=2, opts=opts, n_steps=3)
    b = oracle.step(psi, c, n_iters=2, opts=opts | DFL, n_steps=3)
    assert np.array_equal(a, b)


# ------------------------------------------------------------ source terms
def test_rhs_schemes_without_advection_are_axpy():
    """With a zero advector ADV is the identity, so euler_a and euler_b both
    give psi + dt R and trapez psi + dt/2 (R^n + R^{n+1}) (Sect. 4.1)."""
    gen = synth.rng(91)
    shape = (30, 20)
    psi = gen.uniform(0.0, 1.0, size=shape)
    r0, r1 = gen.normal(size=shape), gen.normal(size=shape)
    c = [np.zeros((31, 20)), np.zeros((30, 21))]
    dt = 0.3
    ea = oracle.step_rhs(psi, c, r_post=r0, a_post=dt, n_iters=3, opts=FCT)
    eb = oracle.step_rhs(psi, c, r_pre=r0, a_pre=dt, n_iters=3, opts=FCT)
    tz = oracle.step_rhs(psi, c, r_pre=r0, a_pre=dt / 2, r_post=r1, a_post=dt / 2, n_iters=3,
                         opts=FCT)
    assert np.allclose(ea, psi + dt * r0, rtol=0, atol=1e-15)
    assert np.allclose(eb, psi + dt * r0, rtol=0, atol=1e-15)
    assert np.allclose(tz, psi + dt / 2 * (r0 + r1), rtol=0, atol=1e-15)


def test_rhs_constant_source_commutes_with_donor_cell():
    """For a spatially constant source and a non-divergent advector the
    donor-cell pass maps psi + k to ADV(psi) + k, so euler_a == euler_b."""
    gen = synth.rng(92)
    shape = (24, 20)
    c = synth.small_advector(shape, 0.5, gen)
    psi = gen.uniform(0.0, 1.0, size=shape)
    R = np.full(shape, 0.37)
    ea = oracle.step_rhs(psi, c, r_post=R, a_post=0.5, n_iters=1)
    eb = oracle.step_rhs(psi, c, r_pre=R, a_pre=0.5, n_iters=1)
    assert np.max(np.abs(ea - eb)) <= 1e-14


def _rotation(psi0, phi0, ang):
    return (psi0 * np.cos(ang) + phi0 * np.sin(ang), phi0 * np.cos(ang) - psi0 * np.sin(ang))


def test_oscillator_at_rest_is_cayley_rotation():
    """With no advection the trapezoidal oscillator step is the Cayley
    transform of the rotation generator: after N steps (psi, phi) is rotated
    by N * 2 atan(dt omega / 2) with the amplitude preserved exactly (eq.
    final_osc).  Using phi^n in place of psi^n in the second argument of
    eq. trapez_osc (as printed) breaks this."""
    gen = synth.rng(93)
    shape = (40,)
    psi0, phi0 = gen.normal(size=shape), gen.normal(size=shape)
    c = [np.zeros(41)]
    a, N = 0.5 * 1.0 * (2 * np.pi / 400), 120
    x, y = oracle.osc_step(psi0, phi0, c, a, n_iters=2, opts=IGA | FCT, n_steps=N)
    ex, ey = _rotation(psi0, phi0, N * 2 * np.arctan(a))
    assert np.max(np.abs(x - ex)) <= 1e-12 and np.max(np.abs(y - ey)) <= 1e-12
    assert np.allclose(x ** 2 + y ** 2, psi0 ** 2 + phi0 ** 2, rtol=1e-12, atol=0)


def test_oscillator_with_unit_courant_translates_and_rotates():
    """At C = 1 every MPDATA step is an exact one-cell shift (Sect. 3), so the
    oscillator's solution is the rotated initial state shifted by N cells."""
    gen = synth.rng(94)
    n = 64
    psi0, phi0 = gen.normal(size=n), gen.normal(size=n)
    c = [np.ones(n + 1)]
    a, N = 0.05, 37
    x, y = oracle.osc_step(psi0, phi0, c, a, n_iters=2, opts=IGA, n_steps=N)
    ex, ey = _rotation(np.roll(psi0, N), np.roll(phi0, N), N * 2 * np.arctan(a))
    assert np.max(np.abs(x - ex)) <= 1e-12 and np.max(np.abs(y - ey)) <= 1e-12


# ---------------------------------------------------------------- P3 conservation
@pytest.mark.parametrize("opts", ALL_OPTS + [KAHAN, FCT | KAHAN, ABS, ABS | TOT | FCT, DFL,
                                              DFL | TOT | FCT])
@pytest.mark.parametrize("shape", [(64,), (24, 20), (10, 9, 8)])
def test_conservation_periodic(opts, shape):
    """Flux form conserves sum(G psi) to round-off (Sect. 1; eq. gte)."""
    gen = synth.rng(21)
    g = gen.uniform(0.5, 1.5, size=shape)
    c = synth.periodic_fix(synth.random_advector(shape, 0.5, gen))
    psi = gen.uniform(0.0, 1.0, size=shape)
    if opts & (IGA | ABS):
        psi -= 0.5
    n_iters = 2 if opts & IGA else 3
    out = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, n_steps=5)
    s0, s1 = np.sum(g * psi), np.sum(g * out)
    assert abs(s1 - s0) / np.sum(np.abs(g * psi)) <= 1e-13


# ---------------------------------------------------------------- P4 sign preservation
@pytest.mark.parametrize("opts", [0, FCT, TOT, FCT | TOT])
@pytest.mark.parametrize("shape,cour", [((80,), 0.5), ((32, 28), 0.5), ((12, 10, 9), 0.5)])
def test_sign_preserving(opts, shape, cour):
    """Non-negative psi stays non-negative (Sect. 1 footnote; Sect. 3.1.4).
    The advector is divergent; a Courant sum of 1/2 keeps every cell's total
    outflow Courant number <= 1."""
    gen = synth.rng(31)
    c = synth.periodic_fix(synth.random_advector(shape, cour, gen))
    psi = np.where(gen.uniform(size=shape) < 0.4, 0.0, gen.uniform(0, 1, size=shape))
    out = oracle.step(psi, c, n_iters=3, opts=opts, n_steps=10)
    assert out.min() >= -4 * np.finfo(float).eps * psi.max()


# ---------------------------------------------------------------- P5 constant state
@pytest.mark.parametrize("opts", ALL_OPTS)
@pytest.mark.parametrize("shape,bc", [((40,), 0), ((40,), 1), ((20, 18), 0), ((20, 18), 1),
                                      ((10, 9, 8), 0), ((10, 9, 8), 1)])
def test_constant_state_preserved(opts, shape, bc):
    """psi = K with a non-divergent G-weighted advector stays K (eq. gte with
    eq. gte_G): every difference in the pseudo-velocity vanishes."""
    gen = synth.rng(41)
    g = gen.uniform(0.5, 1.5, size=shape)
    if len(shape) == 1:
        c = [np.full(shape[0] + 1, 0.375)]
    elif len(shape) == 2:
        c = list(synth.stream_advector_2d(shape, 0.5, gen, n_modes=4, kmax=2))
        c = [x * 0.5 for x in c]          # exact (power of two); keeps Courant/G <= 1
    else:
        c = list(synth.potential_advector_3d(shape, 0.5, gen, g=g, n_modes=3, kmax=2))
    K = 0.7
    psi = np.full(shape, K)
    n_iters = 2 if opts & IGA else 3
    out = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=4)
    # K is not dyadic, so each flux product rounds: allow a few ulp per pass
    np.testing.assert_allclose(out, K, rtol=32 * np.finfo(float).eps, atol=0)


# ---------------------------------------------------------------- P6 exact shift
@pytest.mark.parametrize("opts", ALL_OPTS)
@pytest.mark.parametrize("shape,axis,sgn", [((33,), 0, 1), ((33,), 0, -1), ((12, 11), 1, 1),
                                           ((12, 11), 0, -1), ((6, 7, 8), 2, 1), ((6, 7, 8), 0, -1)])
def test_unit_courant_shifts_one_cell(opts, shape, axis, sgn):
    """|C| = 1 along one axis: every antidiffusive coefficient vanishes and the
    step is an exact one-cell shift (eq. adf_vel at |GC| = G)."""
    gen = synth.rng(51)
    c = []
    for d in range(len(shape)):
        s = list(shape)
        s[d] += 1
        c.append(np.full(s, float(sgn) if d == axis else 0.0))
    psi = gen.uniform(0.1, 1.0, size=shape)
    if opts & IGA:
        psi -= 0.5
    n_iters = 2 if opts & IGA else 3
    out = oracle.step(psi, c, n_iters=n_iters, opts=opts)
    np.testing.assert_allclose(out, np.roll(psi, sgn, axis=axis), rtol=2 * np.finfo(float).eps,
                               atol=2 * np.finfo(float).eps)


# ---------------------------------------------------------------- P7 boundedness
@pytest.mark.parametrize("opts", [FCT, FCT | TOT, FCT | IGA, FCT | IGA | TOT])
@pytest.mark.parametrize("shape", [(120,), (40, 36), (14, 12, 10)])
def test_fct_no_new_extrema(opts, shape):
    """With the limiter (Sect. 3.1.4), and a non-divergent advector of Courant
    sum <= 1, each new value lies within the range of the old values in the
    domain of dependence (radius n_iters), and global extrema do not grow."""
    gen = synth.rng(61)
    c = synth.small_advector(shape, 0.5, gen) if len(shape) > 1 else [np.full(shape[0] + 1, 0.45)]
    psi = np.where(gen.uniform(size=shape) < 0.5, 0.0, 1.0) + 0.1 * gen.uniform(size=shape)
    if opts & IGA:
        psi -= 0.6
    n_iters = 2 if opts & IGA else 3
    out = oracle.step(psi, c, n_iters=n_iters, opts=opts)
    eps = 4 * np.finfo(float).eps * np.abs(psi).max()
    hi = np.full(shape, -np.inf)
    lo = np.full(shape, np.inf)
    r = n_iters
    for off in product(range(-r, r + 1), repeat=len(shape)):
        if sum(abs(o) for o in off) > r:
            continue
        sh = np.roll(psi, off, axis=tuple(range(len(shape))))
        hi, lo = np.maximum(hi, sh), np.minimum(lo, sh)
    assert np.all(out <= hi + eps) and np.all(out >= lo - eps)
    many = oracle.step(psi, c, n_iters=n_iters, opts=opts, n_steps=20)
    assert many.max() <= psi.max() + eps and many.min() >= psi.min() - eps


def test_fct_removes_overshoot_1d():
    """The top-hat of the 1-D workload overshoots without the limiter and does
    not with it (Sect. 3.1.4, Sect. 3.4 non-oscillatory option)."""
    case = synth.case_1d(n_steps=100)
    plain = oracle.step(case.psi, case.c, n_iters=2, n_steps=100)
    lim = oracle.step(case.psi, case.c, n_iters=2, opts=FCT, n_steps=100)
    assert plain.max() > case.psi.max() + 1e-3
    assert lim.max() <= case.psi.max() + 1e-15 and lim.min() >= -1e-15


# ---------------------------------------------------------------- P8 homogeneity
@pytest.mark.parametrize("opts", ALL_OPTS)
@pytest.mark.parametrize("shape", [(50,), (16, 14), (8, 7, 6)])
def test_power_of_two_homogeneity_bitwise(opts, shape):
    """step(2^k psi) == 2^k step(psi) bit for bit: psi-fractions are ratios,
    and no epsilon enters them."""
    gen = synth.rng(71)
    c = synth.periodic_fix(synth.random_advector(shape, 0.6, gen))
    psi = gen.uniform(0.0, 1.0, size=shape)
    if opts & IGA:
        psi -= 0.5
    n_iters = 2 if opts & IGA else 3
    a = oracle.step(psi, c, n_iters=n_iters, opts=opts, n_steps=3)
    b = oracle.step(psi * 2.0 ** 7, c, n_iters=n_iters, opts=opts, n_steps=3)
    np.testing.assert_array_equal(b, a * 2.0 ** 7)


# ---------------------------------------------------------------- P9 linear infinite gauge
@pytest.mark.parametrize("opts", [IGA, IGA | TOT, IGA | DFL, IGA | TOT | DFL])
@pytest.mark.parametrize("shape", [(64,), (20, 18), (9, 8, 7)])
def test_iga_is_linear(opts, shape):
    """Without the limiter the infinite-gauge scheme is linear (Sect. 3.1.5),
    also with the divergent-flow term (random, divergent advectors)."""
    gen = synth.rng(81)
    c = synth.periodic_fix(synth.random_advector(shape, 0.6, gen))
    p, q = gen.normal(size=shape), gen.normal(size=shape)
    a, b = 1.7, -0.3
    lhs = oracle.step(a * p + b * q, c, n_iters=2, opts=opts, n_steps=2)
    rhs = a * oracle.step(p, c, n_iters=2, opts=opts, n_steps=2) + \
        b * oracle.step(q, c, n_iters=2, opts=opts, n_steps=2)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13)


@pytest.mark.parametrize("opts", [IGA, IGA | TOT, IGA | FCT, IGA | FCT | TOT])
def test_iga_background_independent(opts):
    """Ripples of the infinite-gauge option do not depend on the constant
    background (Sect. 3.4 variable-sign example); with the limiter too."""
    gen = synth.rng(82)
    shape = (30, 26)
    c = synth.small_advector(shape, 0.5, gen)
    psi = np.where(gen.uniform(size=shape) < 0.5, -1.0, 1.0)
    K = 3.0
    a = oracle.step(psi, c, n_iters=2, opts=opts, n_steps=5)
    b = oracle.step(psi + K, c, n_iters=2, opts=opts, n_steps=5)
    np.testing.assert_allclose(b - K, a, rtol=0, atol=1e-13)


# ---------------------------------------------------------------- P10 gauge limit
@pytest.mark.parametrize("tot", [0, TOT])
@pytest.mark.parametrize("shape", [(48,), (16, 14), (8, 8, 6)])
def test_gauge_limit(tot, shape):
    """[step(psi + K) - K] of the standard scheme tends to the infinite-gauge
    step with an error ~ 1/K (the gauge is the limit of infinite background)."""
    gen = synth.rng(91)
    # non-divergent, so a constant background is itself a steady solution
    c = synth.small_advector(shape, 0.5, gen)
    psi = gen.normal(size=shape)
    ref = oracle.step(psi, c, n_iters=2, opts=IGA | tot)
    errs = []
    for K in (2.0 ** 12, 2.0 ** 14, 2.0 ** 16):
        out = oracle.step(psi + K, c, n_iters=2, opts=tot) - K
        errs.append(np.abs(out - ref).max())
    assert errs[0] < 1e-2
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.0 < e0 / e1 < 5.5        # one factor 4 in K -> error / 4


# ---------------------------------------------------------------- P11 Fourier
def _amplification(shape, cvec, theta_idx, opts):
    """Numerical amplification factor of one step on the Fourier mode with
    integer wavenumber vector theta_idx (constant advector, G = 1)."""
    nd = len(shape)
    c = []
    for d in range(nd):
        s = list(shape)
        s[d] += 1
        c.append(np.full(s, cvec[d]))
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = sum(2 * math.pi * k * x / n for k, x, n in zip(theta_idx, grids, shape))
    oc = oracle.step(np.cos(phase), c, n_iters=2, opts=opts)
    os_ = oracle.step(np.sin(phase), c, n_iters=2, opts=opts)
    g = (oc + 1j * os_) / np.exp(1j * phase)
    return g.mean(), np.abs(g - g.mean()).max()


def test_fourier_closed_form_1d():
    """Infinite-gauge step on a Fourier mode, 1-D: the composition of the donor
    factor and the corrective-flux factor (linear scheme, constant c)."""
    for U in (0.3, -0.6):
        for tot in (0, TOT):
            n, k = 64, 5
            th = 2 * math.pi * k / n
            gnum, spread = _amplification((n,), [U], [k], IGA | tot)
            assert spread < 1e-13
            e = np.exp(1j * th)
            if U >= 0:
                g1 = 1 - U * (1 - 1 / e)
            else:
                g1 = 1 - U * (e - 1)
            alpha = (3 * U * abs(U) - 2 * U ** 3 - U) / 3 if tot else 0.0
            corr = (abs(U) - U * U) * (e - 1) / 2 + alpha * (e * e - e - 1 + 1 / e) / 4
            gcf = g1 * (1 - (1 - 1 / e) * corr)
            assert abs(gnum - gcf) < 1e-14


@pytest.mark.parametrize("cvec", [(0.3,), (-0.55,), (0.3, 0.2), (-0.25, 0.35), (0.2, -0.15, 0.25),
                                  (-0.3, -0.2, 0.1)])
@pytest.mark.parametrize("tot", [0, TOT])
def test_fourier_order_conditions(cvec, tot):
    """Local error of one step on a mode is O(theta^3) (second order, Sect.
    3.1.1) and O(theta^4) with the third-order terms (Sect. 3.1.2) for the
    infinite-gauge scheme; checked by halving the wavenumber."""
    nd = len(cvec)
    n = 256 if nd == 1 else (128 if nd == 2 else 32)
    shape = (n,) * nd
    dirs = [(1,), (1, 1), (1, 1, 1)][nd - 1], [(1,), (1, -1), (1, -1, 1)][nd - 1]
    want = 4.0 if tot else 3.0
    for dvec in dirs:
        errs = []
        for m in (4, 2, 1):
            kk = [m * v for v in dvec]
            g, _ = _amplification(shape, cvec, kk, IGA | tot)
            th = [2 * math.pi * k / n for k in kk]
            exact = np.exp(-1j * sum(c * t for c, t in zip(cvec, th)))
            errs.append(abs(g - exact))
        orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
        assert orders[-1] > want - 0.25, (dvec, errs, orders)


# ---------------------------------------------------------------- P12 convergence
def _cell_gauss(x_lo, x_hi, x0, sigma):
    from scipy.special import erf
    s = sigma * math.sqrt(2.0)
    return 0.5 * (erf((x_hi - x0) / s) - erf((x_lo - x0) / s)) / (x_hi - x_lo)


def _conv_error(k, C, n_iters, opts):
    """Truncation error (eq. trerr) of the 1-D convergence test (Sect. 3.5):
    X = 44, T = 1, u = 1, sigma = 1.5, x0 = X/2, cell-integrated profiles,
    periodic; NT = round(T / dt) and the exact solution at NT dt."""
    X, sigma = 44.0, 1.5
    dx = 2.0 ** -k
    nx = int(round(X / dx))
    dt = C * dx
    nt = int(round(1.0 / dt))
    t = nt * dt
    edges = np.arange(nx + 1) * dx
    psi0 = _cell_gauss(edges[:-1], edges[1:], X / 2, sigma)
    ex = _cell_gauss(edges[:-1], edges[1:], X / 2 + t, sigma)
    out = oracle.step(psi0, [np.full(nx + 1, C)], n_iters=n_iters, opts=opts, n_steps=nt)
    return math.sqrt(np.mean((ex - out) ** 2)) / 1.0


@pytest.mark.slow
@pytest.mark.parametrize("label,n_iters,opts,lo,hi", [
    ("donor", 1, 0, 0.8, 1.2),
    ("basic", 2, 0, 1.8, 2.3),
    ("three-pass", 3, 0, 1.8, 2.6),
    ("tot three-pass", 3, TOT, 2.7, 3.4),
    ("fct", 2, FCT, 1.5, 2.2),
    ("iga", 2, IGA, 1.8, 2.3),
    ("iga tot", 2, IGA | TOT, 2.7, 3.4),
])
@pytest.mark.parametrize("C", [0.25, 0.75])
def test_convergence_orders(label, n_iters, opts, lo, hi, C):
    """Orders of the convergence test of Sect. 3.5: donor-cell 1, MPDATA 2,
    third-order variant 3, limiter about 1.8, infinite gauge 2 (3 with tot)."""
    e5 = _conv_error(5, C, n_iters, opts)
    e6 = _conv_error(6, C, n_iters, opts)
    order = math.log2(e5 / e6)
    assert lo < order < hi, (label, C, e5, e6, order)


def test_iga_as_accurate_as_three_pass():
    """Sect. 3.5: the infinite gauge is about as accurate as three-pass MPDATA."""
    e_iga = _conv_error(5, 0.5 - 0.25, 2, IGA)
    e_3 = _conv_error(5, 0.25, 3, 0)
    e_2 = _conv_error(5, 0.25, 2, 0)
    assert e_iga < e_2 and 0.3 < e_iga / e_3 < 3.0


def test_variable_g_second_order():
    """1-D, G = 1 + 0.3 sin(2 pi x / X), constant G-weighted advector: the
    exact solution moves the mass coordinate m(x) = int G dx uniformly, and the
    scheme (with the mean G at walls) converges at second order."""
    X, a = 32.0, 0.3

    def m_of(x):
        return x + a * X / (2 * math.pi) * (1 - np.cos(2 * math.pi * x / X))

    def x_of(m):
        x = m.copy()
        for _ in range(60):
            x = x - (m_of(x) - m) / (1 + a * np.sin(2 * math.pi * x / X))
        return x

    def prof(x):
        d = (x - X / 2 + X / 2) % X - X / 2
        return np.exp(-d * d / (2 * 2.0 ** 2))

    errs = []
    for k in (4, 5, 6):
        dx = 2.0 ** -k
        nx = int(X / dx)
        x = (np.arange(nx) + 0.5) * dx
        g = 1 + a * np.sin(2 * math.pi * x / X)
        Q = 0.4                      # G-weighted Courant number per step
        nt = int(round(4.0 / (Q * dx)))
        psi = oracle.step(prof(x), [np.full(nx + 1, Q)], g=g, n_iters=2, n_steps=nt)
        shift = nt * Q * dx
        ex = prof(x_of((m_of(x) - shift) % X))
        errs.append(math.sqrt(np.mean((psi - ex) ** 2)))
    orders = [math.log2(e0 / e1) for e0, e1 in zip(errs, errs[1:])]
    assert 1.8 < orders[-1] < 2.3, (errs, orders)


# ---------------------------------------------------------------- P13 symmetry
@pytest.mark.parametrize("opts", ALL_OPTS)
@pytest.mark.parametrize("shape", [(30,), (12, 10), (7, 6, 5)])
def test_translation_equivariance_bitwise(opts, shape):
    gen = synth.rng(101)
    g = gen.uniform(0.5, 1.5, size=shape)
    c = synth.periodic_fix(synth.random_advector(shape, 0.5, gen))
    psi = gen.uniform(0.0, 1.0, size=shape) - (0.5 if opts & IGA else 0.0)
    n_iters = 2 if opts & IGA else 3
    shift = tuple(range(1, len(shape) + 1))
    axes = tuple(range(len(shape)))
    a = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, n_steps=2)

    def roll_wall(x, d):
        core = np.take(x, range(shape[d]), axis=d)
        core = np.roll(core, shift, axis=axes)
        first = np.take(core, [0], axis=d)
        return np.concatenate([core, first], axis=d)

    b = oracle.step(np.roll(psi, shift, axis=axes), [roll_wall(x, d) for d, x in enumerate(c)],
                    g=np.roll(g, shift, axis=axes), n_iters=n_iters, opts=opts, n_steps=2)
    np.testing.assert_array_equal(b, np.roll(a, shift, axis=axes))


@pytest.mark.parametrize("opts", ALL_OPTS)
@pytest.mark.parametrize("shape,bc", [((30,), 1), ((12, 10), 0), ((12, 10), 1), ((7, 6, 5), 1)])
def test_mirror_symmetry(opts, shape, bc):
    """Reflecting the grid along an axis (and negating that velocity
    component) reflects the result (Arakawa-C staggering, Sect. 2.3)."""
    gen = synth.rng(111)
    g = gen.uniform(0.5, 1.5, size=shape)
    c = synth.random_advector(shape, 0.5, gen)
    if bc == 0:
        c = synth.periodic_fix(c)
    psi = gen.uniform(0.0, 1.0, size=shape) - (0.5 if opts & IGA else 0.0)
    n_iters = 2 if opts & IGA else 3
    a = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=2)
    for ax in range(len(shape)):
        cm = [np.flip(x, axis=ax) * (-1.0 if d == ax else 1.0) for d, x in enumerate(c)]
        b = oracle.step(np.flip(psi, axis=ax), cm, g=np.flip(g, axis=ax), n_iters=n_iters,
                        opts=opts, bc=bc, n_steps=2)
        np.testing.assert_allclose(np.flip(b, axis=ax), a, rtol=0, atol=1e-13)


@pytest.mark.parametrize("opts", ALL_OPTS)
def test_transpose_symmetry(opts):
    """Swapping the two axes of a 2-D problem swaps the result."""
    gen = synth.rng(121)
    shape = (11, 9)
    g = gen.uniform(0.5, 1.5, size=shape)
    c = synth.periodic_fix(synth.random_advector(shape, 0.5, gen))
    psi = gen.uniform(0.0, 1.0, size=shape) - (0.5 if opts & IGA else 0.0)
    n_iters = 2 if opts & IGA else 3
    a = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, n_steps=2)
    b = oracle.step(psi.T.copy(), [c[1].T.copy(), c[0].T.copy()], g=g.T.copy(), n_iters=n_iters,
                    opts=opts, n_steps=2)
    np.testing.assert_allclose(b.T, a, rtol=0, atol=1e-13)


# ---------------------------------------------------------------- workload sanity
def test_1d_workload_one_period():
    """1000 steps at C = 0.5 move the 1-D workload once round the 500-cell ring;
    MPDATA keeps it close to the initial field (accuracy report, not parity)."""
    case = synth.case_1d()
    out = oracle.step(case.psi, case.c, n_iters=2, n_steps=1000)
    err = math.sqrt(np.mean((out - case.psi) ** 2))
    donor = oracle.step(case.psi, case.c, n_iters=1, n_steps=1000)
    err_d = math.sqrt(np.mean((donor - case.psi) ** 2))
    assert err < 0.6 * err_d


def test_diag_and_courant():
    psi = np.array([[1.0, -2.0], [np.nan, 4.0]])
    g = np.array([[2.0, 1.0], [1.0, 0.5]])
    s, mn, mx, bad = oracle.diag(psi, g)
    assert (s, mn, mx, bad) == (2.0, -2.0, 4.0, 1)
    c0 = np.array([[0.1, 0.2], [0.3, -0.4], [0.1, 0.2]])
    c1 = np.array([[0.05, 0.0, 0.05], [-0.25, 0.1, -0.25]])
    cm = oracle.courant_max((2, 2), [c0, c1], g=g)
    # cell (1,1): max(0.4, 0.2) + max(0.1, 0.25) = 0.65, / 0.5
    assert abs(cm - 1.3) < 1e-15


# ---------------------------------------------------------------- compensated sum of diag
def test_diag_sum_is_compensated():
    """The conservation diagnostic (Sect. 1: the scheme conserves sum G psi)
    sums with compensation.  Cancellation cases that plain left-to-right
    summation gets wrong: [2^53, 1, -2^53, 1] sums to 1 uncompensated and 2
    exactly; [1, 2^100, 1, -2^100] defeats Kahan's form (the compensation
    is lost when a later term dwarfs the running sum) but not Neumaier's.
    A dropped or mis-signed compensation term fails one of them."""
    for vals, exact in (([2.0 ** 53, 1.0, -2.0 ** 53, 1.0], 2.0),
                        ([1.0, 2.0 ** 100, 1.0, -2.0 ** 100], 2.0),
                        ([1e16, 3.0, 3.0, -1e16], 6.0),
                        ([-2.0 ** 60, 7.0, 2.0 ** 60, -1.0, 1.0], 7.0)):
        psi = np.array(vals)
        s, mn, mx, bad = oracle.diag(psi)
        assert s == exact, (vals, s)
        assert (mn, mx, bad) == (min(vals), max(vals), 0)
        # the same values as G * psi products (exact ones: G = 0.5, psi doubled)
        s2, _, _, _ = oracle.diag(2.0 * psi, np.full(psi.shape, 0.5))
        assert s2 == exact
        # plain summation really differs here (the pin has teeth)
        naive = 0.0
        for v in vals:
            naive += v
        assert naive != exact


def test_diag_sum_matches_exact_summation():
    """On ill-conditioned data (terms of random sign spanning 2^-40..2^40,
    sum of order 1) the compensated sum of the rounded G*psi products stays
    within 2 ulp of their exactly rounded sum (math.fsum, an exact
    summation), where plain summation is off by many orders more.  Neumaier's
    bound: |error| <= 2u|S| + O(n u^2) sum|x|."""
    gen = np.random.default_rng(123)
    n = 4096
    mag = 2.0 ** gen.uniform(-40, 40, size=n)
    gm = gen.uniform(0.5, 2.0, size=n)
    small = gen.uniform(-1, 1, size=n)
    # pairs +x, -x under the same G cancel exactly; the small terms remain
    psi = np.concatenate([mag, -mag, small])
    g = np.concatenate([gm, gm, np.ones(n)])
    perm = gen.permutation(psi.size)
    psi, g = psi[perm], g[perm]
    terms = g * psi                       # the products the sum is defined over
    exact = math.fsum(terms.tolist())
    s, _, _, _ = oracle.diag(psi.reshape(96, 128), g.reshape(96, 128))
    assert abs(s - exact) <= 2 * np.spacing(abs(exact)), (s, exact)
    naive = float(np.sum(terms[:0]))
    for t in terms:
        naive += t
    assert abs(naive - exact) > 1e3 * np.spacing(abs(exact))


# ---------------------------------------------------------------- multi-core build
@pytest.mark.parametrize("shape,bc,opts", [((37, 29), 0, FCT), ((9, 7, 11), 1, IGA | TOT),
                                           ((64,), 0, FCT | TOT), ((20, 30), 1, FCT | KAHAN)])
def test_openmp_build_same_bits(shape, bc, opts):
    """The OpenMP build of the oracle (the multi-core CPU baseline) shares
    each stage's outermost loop among threads; every iteration writes only its
    own cells, so the result is the single-threaded one bit for bit."""
    gen = synth.rng(17)
    g = gen.uniform(0.7, 1.3, size=shape)
    c = synth.random_advector(shape, 0.4, gen)
    if bc == 0:
        c = synth.periodic_fix(c)
    psi = gen.uniform(0.0, 1.0, size=shape) if not opts & IGA else gen.normal(size=shape)
    n_iters = 2 if opts & IGA else 3
    a = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=4)
    b = oracle.step(psi, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=4, parallel=True)
    assert np.array_equal(a, b)
    assert oracle.threads(parallel=False) == 1
