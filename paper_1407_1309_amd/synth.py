"""Seeded synthetic inputs for the MPDATA step (no method arithmetic here).

Shared by the tests, the benchmark and the smoke check; used by both the HIP
path and the CPU oracle.  Everything is produced in float64 with NumPy's
PCG64 generator; FP32 runs cast the result (the advector is built so that the
cast is exact).

Layout (row-major, last dimension fastest): psi and G are cell arrays of shape
n; the advector component c[d] has n[d]+1 entries along dimension d, entry f
being the wall between cells f-1 and f.

Velocity fields are made exactly non-divergent: a stream function (2-D) or a
vector potential (3-D) is sampled at cell corners / edges, quantised to a
power-of-two grid so that every value and every difference is exact in the
target precision, and the wall values are its differences.  The discrete
divergence of every cell is then exactly zero as a real number.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

def _quantise(a: np.ndarray, mant_bits: int) -> np.ndarray:
    """Round to multiples of 2**(e - mant_bits) with 2**e >= max|a|."""
    m = float(np.max(np.abs(a)))
    if m == 0.0:
        return a.copy()
    e = math.ceil(math.log2(m))
    q = 2.0 ** (e - mant_bits)
    return np.round(a / q) * q


def courant_sum(c, g=None) -> float:
    """max over cells of sum_d max(|c_d| on the two d-walls) / G."""
    nd = len(c)
    shape = list(c[0].shape)
    shape[0] -= 1
    tot = np.zeros(shape)
    for d in range(nd):
        a = np.abs(c[d])
        lo = np.take(a, range(0, shape[d]), axis=d)
        hi = np.take(a, range(1, shape[d] + 1), axis=d)
        tot = tot + np.maximum(lo, hi)
    if g is not None:
        tot = tot / g
    return float(tot.max())


def _periodic_offsets(n: int, centre: float) -> np.ndarray:
    x = np.arange(n, dtype=np.float64) - centre
    return x - n * np.round(x / n)


def blob_field(shape, n_blobs, sigma_range, amp, gen: np.random.Generator,
               periodic=True) -> np.ndarray:
    """Sum of Gaussian blobs exp(-r^2 / (2 s^2)); amp is 'uniform' (U(0,1)) or
    'normal' (N(0,1)).  Periodic fields use the minimum-image distance.  Each
    blob is separable, so the sum over blobs is a product of per-axis profile
    matrices (the last axis split off)."""
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    profs = [[] for _ in range(nd)]
    amps = []
    for _ in range(n_blobs):
        centre = [gen.uniform(0, s) for s in shape]
        s = gen.uniform(*sigma_range)
        a = gen.uniform(0.0, 1.0) if amp == "uniform" else gen.normal()
        amps.append(a)
        for d, n in enumerate(shape):
            if periodic:
                x = _periodic_offsets(n, centre[d])
            else:
                x = np.arange(n, dtype=np.float64) - centre[d]
            profs[d].append(np.exp(-x * x / (2.0 * s * s)))
    amps = np.array(amps)
    if nd == 1:
        return np.array(profs[0]).T @ amps
    lead = np.array(profs[0]).T * amps                     # (n0, B)
    for d in range(1, nd - 1):
        P = np.array(profs[d]).T                            # (nd, B)
        lead = (lead[:, None, :] * P[None, :, :]).reshape(-1, n_blobs)
    out = lead @ np.array(profs[nd - 1])                    # (prod lead, n_last)
    return out.reshape(shape)


# --------------------------------------------------------------------------
# non-divergent advectors
# --------------------------------------------------------------------------

def _modes(gen, nd, n_modes, kmax):
    ks = []
    while len(ks) < n_modes:
        k = tuple(int(v) for v in gen.integers(-kmax, kmax + 1, size=nd))
        if any(k):
            ks.append(k)
    amps = gen.normal(size=n_modes)
    phases = gen.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return ks, amps, phases


def _sum_of_sines(coords, lengths, ks, amps, phases):
    """sum_m a_m sin(2 pi sum_d k_md x_d / L_d + phi_m) on the outer grid of
    the 1-D coordinate vectors.  With the last axis split off,
    sin(P + Q) = sin P cos Q + cos P sin Q turns the sum over modes into one
    matrix product."""
    shape = tuple(len(x) for x in coords)
    nd = len(coords)
    lead_cols_s, lead_cols_c, last_c, last_s = [], [], [], []
    for k, a, ph in zip(ks, amps, phases):
        P = np.full((1,), ph)
        for d in range(nd - 1):
            ang = 2.0 * math.pi * k[d] * coords[d] / lengths[d]
            P = (P[:, None] + ang[None, :]).reshape(-1)
        q = 2.0 * math.pi * k[nd - 1] * coords[nd - 1] / lengths[nd - 1]
        lead_cols_s.append(a * np.sin(P))
        lead_cols_c.append(a * np.cos(P))
        last_c.append(np.cos(q))
        last_s.append(np.sin(q))
    lead = np.stack(lead_cols_s + lead_cols_c, axis=1)      # (prod lead, 2M)
    last = np.stack(last_c + last_s, axis=0)                # (2M, n_last)
    return (lead @ last).reshape(shape)


def stream_advector_2d(shape, courant, gen, n_modes=8, kmax=4, mant_bits=23):
    """Periodic non-divergent (c0, c1) from a random stream function.

    Psi sampled at corners (a-1/2, b-1/2), a in [0, n0], b in [0, n1];
    c0[f, j] = Psi[f, j+1] - Psi[f, j];  c1[i, f] = -(Psi[i+1, f] - Psi[i, f]).
    Integer wavenumbers make wall n_d equal wall 0 exactly."""
    n0, n1 = (int(s) for s in shape)
    ks, amps, phases = _modes(gen, 2, n_modes, kmax)
    xa = np.arange(n0 + 1, dtype=np.float64) - 0.5
    xb = np.arange(n1 + 1, dtype=np.float64) - 0.5
    psi_c = _sum_of_sines([xa, xb], [n0, n1], ks, amps, phases)

    def walls(p):
        c0 = p[:, 1:] - p[:, :-1]
        c1 = -(p[1:, :] - p[:-1, :])
        return c0, c1

    c0, c1 = walls(psi_c)
    s = courant_sum([c0, c1])
    psi_c = _quantise(psi_c * (courant / s), mant_bits)
    # periodic corners: the last row/column repeats the first bit for bit, so
    # wall n_d equals wall 0 and every cell stays exactly non-divergent
    psi_c[n0, :] = psi_c[0, :]
    psi_c[:, n1] = psi_c[:, 0]
    return walls(psi_c)


def potential_advector_3d(shape, courant, gen, g=None, n_modes=8, kmax=4,
                          mant_bits=50):
    """Non-divergent (c0, c1, c2) = discrete curl of a random vector potential
    sampled on cell edges (all walls, including boundary walls, are curls).

    Edge arrays: A0[i, b, c] at (i, b-1/2, c-1/2); A1[a, j, c] at
    (a-1/2, j, c-1/2); A2[a, b, k] at (a-1/2, b-1/2, k).  The scale is set so
    that the Courant sum (walls / G) equals `courant`."""
    n = [int(s) for s in shape]
    cell = [np.arange(m, dtype=np.float64) for m in n]
    edge = [np.arange(m + 1, dtype=np.float64) - 0.5 for m in n]
    A = []
    for comp in range(3):
        ks, amps, phases = _modes(gen, 3, n_modes, kmax)
        coords = [cell[d] if d == comp else edge[d] for d in range(3)]
        A.append(_sum_of_sines(coords, n, ks, amps, phases))

    def curl(A0, A1, A2):
        c0 = (A2[:, 1:, :] - A2[:, :-1, :]) - (A1[:, :, 1:] - A1[:, :, :-1])
        c1 = (A0[:, :, 1:] - A0[:, :, :-1]) - (A2[1:, :, :] - A2[:-1, :, :])
        c2 = (A1[1:, :, :] - A1[:-1, :, :]) - (A0[:, 1:, :] - A0[:, :-1, :])
        return c0, c1, c2

    c = curl(*A)
    s = courant_sum(list(c), g)
    A = [_quantise(a * (courant / s), mant_bits) for a in A]
    return curl(*A)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

@dataclass
class Case:
    name: str
    psi: np.ndarray
    c: list
    g: np.ndarray | None
    n_iters: int
    opts: int            # bit 0 fct, bit 1 iga, bit 2 tot
    bc: int              # 0 periodic, 1 open
    n_steps: int
    extra: dict = field(default_factory=dict)


OPT_FCT, OPT_IGA, OPT_TOT, OPT_DFL = 1, 2, 4, 16


def case_1d(nx=500, n_steps=1000) -> Case:
    """1-D periodic: Gaussian (centre 250, sigma 20, peak 1) plus a top-hat of
    value 1 on cells 50..100 inclusive; constant Courant number 0.5."""
    i = np.arange(nx, dtype=np.float64)
    psi = np.exp(-((i - 250.0) ** 2) / (2.0 * 20.0 ** 2)) + ((i >= 50) & (i <= 100))
    c0 = np.full(nx + 1, 0.5)
    return Case("1d_periodic", psi, [c0], None, 2, 0, 0, n_steps)


def case_osc(nx=1001, n_steps=1400, courant=0.5, omega=2 * np.pi / 400, dt=1.0) -> Case:
    """Translating oscillator (the paper's inhomogeneous example): 1-D
    periodic, psi = 0.5 (1 + cos(2 pi x / 100)) for 50 < x < 150 and 0
    elsewhere (x = cell index), phi = 0, constant Courant number 0.5,
    omega = 2 pi / 400, dt = 1; iga with the limiter, n_iters = 2 (the
    library's default options for a variable-sign pair)."""
    x = np.arange(nx, dtype=np.float64)
    psi = np.where((x > 50) & (x < 150), 0.5 * (1.0 + np.cos(2 * np.pi * x / 100.0)), 0.0)
    c0 = np.full(nx + 1, float(courant))
    return Case("osc_1d_periodic", psi, [c0], None, 2, OPT_FCT | OPT_IGA, 0, n_steps,
                extra={"phi": np.zeros(nx), "a": 0.5 * dt * omega})


def drop_coords(shape, half):
    """Cell-centre coordinates of a box [-half, half]^nd split into `shape`
    cells, and the spacing per dimension."""
    dx = [2.0 * half / n for n in shape]
    axes = [(np.arange(n) + 0.5) * d - half for n, d in zip(shape, dx)]
    return np.meshgrid(*axes, indexing="ij"), dx


def case_sw(n=2048, half=6.0, n_steps=100) -> Case:
    """Shallow-water drop (the paper's 2-D prognosed-velocity example): an
    n x n box [-6, 6]^2, open boundaries, depth 1 - r^2 inside r < 1 and 0
    outside, at rest; dt = dx / 5, g = 1, eps = 1e-8; iga + fct + dfl with
    n_iters = 2.  extra: q (momenta), dt, dx, grav, eps."""
    shape = (n, n)
    X, dx = drop_coords(shape, half)
    h = np.maximum(1.0 - X[0] ** 2 - X[1] ** 2, 0.0)
    return Case(f"sw_2d_open_{n}x{n}", h, [], None, 2, OPT_FCT | OPT_IGA | OPT_DFL, 1, n_steps,
                extra={"q": [np.zeros(shape), np.zeros(shape)], "dt": dx[0] / 5.0, "dx": dx,
                       "grav": 1.0, "eps": 1e-8})


def sw_state(shape, seed, half=2.0, ring=True):
    """A perturbed shallow-water state in motion at two time levels:
    depth (R^2 - r^2)+ (R = 0.8 half) times (1 + 5% noise), with `ring` a
    ring of cells outside the drop with depths in [0, 2e-8) (around the
    usual cut-off), outward velocity 0.4 x_d / half plus 5% noise, momenta
    = velocity x depth; the previous level is the same with 2%
    multiplicative noise.  Returns (h, q, h_prev, q_prev, dx)."""
    gen = rng(seed)
    X, dx = drop_coords(shape, half)
    r2 = sum(x * x for x in X)
    R2 = (0.8 * half) ** 2
    h = np.maximum(R2 - r2, 0.0) / R2 * (1.0 + 0.05 * gen.uniform(-1, 1, size=shape))
    band = (r2 >= R2) & (r2 < 1.2 * R2) & ring
    h = np.where(band, gen.uniform(0.0, 2e-8, size=shape), h)
    u = [0.4 * x / half + 0.05 * gen.uniform(-1, 1, size=shape) for x in X]
    q = [ud * h for ud in u]
    h_prev = h * (1.0 + 0.02 * gen.uniform(-1, 1, size=shape))
    q_prev = [qd * (1.0 + 0.02 * gen.uniform(-1, 1, size=shape)) for qd in q]
    return h, q, h_prev, q_prev, dx


def case_2d(n=2048, seed=2, courant=0.5, sigma=(32.0, 128.0), n_blobs=64,
            n_iters=3, opts=OPT_FCT, n_steps=200, shape=None) -> Case:
    """2-D periodic: stream-function advector (8 modes, wavenumbers -4..4),
    64 non-negative Gaussian blobs, n_iters=3 with the limiter."""
    shape = tuple(shape) if shape is not None else (n, n)
    gen = rng(seed)
    c0, c1 = stream_advector_2d(shape, courant, gen)
    psi = blob_field(shape, n_blobs, sigma, "uniform", gen, periodic=True)
    return Case(f"2d_periodic_{shape[0]}x{shape[1]}", psi, [c0, c1], None,
                n_iters, opts, 0, n_steps)


def case_3d(shape=(384, 384, 256), seed=3, courant=0.6, n_steps=100,
            sigma=(8.0, 32.0), n_blobs=64) -> Case:
    """3-D open: G(k) = exp(-(k+1/2)/H), H = nz/2 along the last axis; curl
    advector with Courant sum 0.6; variable-sign blobs; tot + iga, n_iters=2."""
    shape = tuple(int(s) for s in shape)
    gen = rng(seed)
    H = 0.5 * shape[2]
    gz = np.exp(-(np.arange(shape[2], dtype=np.float64) + 0.5) / H)
    g = np.broadcast_to(gz, shape).copy()
    c = potential_advector_3d(shape, courant, gen, g=g)
    psi = blob_field(shape, n_blobs, sigma, "normal", gen, periodic=False)
    return Case(f"3d_open_{shape[0]}x{shape[1]}x{shape[2]}", psi, list(c), g,
                2, OPT_TOT | OPT_IGA, 1, n_steps)


def batch_shapes(n_grids=1024, lo=64, hi=768, seed=4):
    gen = rng(seed)
    return [tuple(int(v) for v in gen.integers(lo, hi + 1, size=2)) for _ in range(n_grids)]


def case_batch(n_grids=1024, lo=64, hi=768, seed=4, courant=0.4, n_steps=100,
               grids=None):
    """Many independent 2-D periodic grids of uneven size.  Returns a list of
    Case (one per grid); grid i uses the i-th spawned child of the seed."""
    shapes = batch_shapes(n_grids, lo, hi, seed)
    children = np.random.SeedSequence(seed).spawn(n_grids)
    idx = range(n_grids) if grids is None else grids
    out = []
    for i in idx:
        shape = shapes[i]
        gen = np.random.Generator(np.random.PCG64(children[i]))
        c0, c1 = stream_advector_2d(shape, courant, gen)
        m = min(shape)
        psi = blob_field(shape, 16, (m / 32.0, m / 8.0), "uniform", gen, periodic=True)
        out.append(Case(f"batch_{i}_{shape[0]}x{shape[1]}", psi, [c0, c1], None,
                        2, OPT_FCT, 0, n_steps))
    return out


def case_adjoint(n=1024, seed=5, n_steps=200) -> dict:
    """2-D periodic 1024^2 adjoint workload: forward set-up as the 2-D case
    (Courant sum 0.5, sigma in [16, 64]); the observation comes from a run
    started at psi0 + 0.05 * (blob field, seed 52) with advector c + dc, dc
    from an independent stream function (seed 53) of Courant sum 0.05."""
    base = case_2d(n=n, seed=seed, courant=0.5, sigma=(16.0, 64.0), n_iters=2,
                   opts=OPT_FCT, n_steps=n_steps)
    dpsi = blob_field((n, n), 64, (16.0, 64.0), "uniform", rng(52), periodic=True)
    dc0, dc1 = stream_advector_2d((n, n), 0.05, rng(53))
    return {"case": base, "psi_perturbed": base.psi + 0.05 * dpsi,
            "c_perturbed": [base.c[0] + dc0, base.c[1] + dc1]}


# --------------------------------------------------------------------------
# small generic inputs for tests
# --------------------------------------------------------------------------

def small_advector(shape, courant, gen, periodic=True, g=None):
    """Non-divergent advector for any 1/2/3-D shape (1-D: a constant)."""
    nd = len(shape)
    if nd == 1:
        c = np.full(shape[0] + 1, float(courant) * (1 if gen.uniform() < 0.5 else -1))
        if g is not None:
            c = c * float(np.min(g))
        return [c]
    if nd == 2:
        c = list(stream_advector_2d(shape, courant, gen, n_modes=4, kmax=2))
        if g is not None:
            s = courant_sum(c, g)
            c = [x * (courant / s) for x in c]
        return c
    return list(potential_advector_3d(shape, courant, gen, g=g, n_modes=3, kmax=2))


def random_advector(shape, courant, gen):
    """Divergent random advector (walls independent, uniform signs)."""
    nd = len(shape)
    c = []
    for d in range(nd):
        s = list(shape)
        s[d] += 1
        c.append(gen.uniform(-1.0, 1.0, size=s))
    sc = courant_sum(c)
    c = [x * (courant / sc) for x in c]
    return c


def periodic_fix(c):
    """Copy wall 0 into wall n along each dimension (periodic convention)."""
    out = []
    for d, x in enumerate(c):
        x = x.copy()
        idx_last = [slice(None)] * x.ndim
        idx_first = [slice(None)] * x.ndim
        idx_last[d] = x.shape[d] - 1
        idx_first[d] = 0
        x[tuple(idx_last)] = x[tuple(idx_first)]
        out.append(x)
    return out
