"""FP64 CPU oracle of the MPDATA time step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path (the HIP library and its Python
binding) never imports it.

Thin ctypes wrapper over liboracle.so (built from mpdata_oracle*.c by
oracle/build.py); the source-term schemes, the translating oscillator, the
prognosed-velocity advector and the shallow-water step (step_rhs, osc_step,
vip_advector, sw_step) are plain compositions of its step with numpy
arithmetic.  Arrays are numpy float64, C-contiguous, last dimension
fastest.  The advector component c[d] has n[d]+1 entries along dimension d.
"""
import ctypes
import os

import numpy as np

from . import build as _build

BC_PERIODIC, BC_OPEN = 0, 1
OPT_FCT, OPT_IGA, OPT_TOT, OPT_ABS, OPT_DFL, OPT_KAHAN = 1, 2, 4, 8, 16, 32

_LIBS = {}
_DP = ctypes.POINTER(ctypes.c_double)


def _lib(parallel=False):
    """The oracle library: single-threaded, or (parallel=True) the same
    source built with OpenMP over each stage's outermost loop (same bits)."""
    if parallel not in _LIBS:
        path = _build.OUT_OMP if parallel else _build.OUT
        srcs = [os.path.join(_build.HERE, s) for s in _build.SOURCES]
        newest = max(os.path.getmtime(s) for s in srcs if os.path.exists(s))
        if not os.path.exists(path) or os.path.getmtime(path) < newest:
            _build.build()
        lib = ctypes.CDLL(path)
        L3 = ctypes.c_long * 3
        I3 = ctypes.c_int * 3
        lib.orc_step.argtypes = [ctypes.c_int, L3, I3, ctypes.c_int, ctypes.c_uint,
                                 _DP, _DP, _DP, _DP, _DP, ctypes.c_long]
        lib.orc_diag.argtypes = [ctypes.c_int, L3, _DP, _DP, _DP,
                                 ctypes.POINTER(ctypes.c_long)]
        lib.orc_courant_max.argtypes = [ctypes.c_int, L3, I3, _DP, _DP, _DP, _DP, _DP]
        if hasattr(lib, "orc_adjoint"):
            lib.orc_adjoint.argtypes = [ctypes.c_int, L3, I3, ctypes.c_int, ctypes.c_uint,
                                        _DP, _DP, _DP, _DP, _DP, ctypes.c_long, ctypes.c_long,
                                        _DP, _DP, _DP, _DP, _DP]
        lib.orc_threads.restype = ctypes.c_int
        _LIBS[parallel] = lib
    return _LIBS[parallel]


def threads(parallel=True):
    """Threads the stage loops of step() use in the given build."""
    return int(_lib(parallel).orc_threads())


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_DP)


def _f64(a):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(psi_shape, bc):
    ndims = len(psi_shape)
    n = [int(s) for s in psi_shape] + [1] * (3 - ndims)
    if isinstance(bc, int):
        bc = [bc] * ndims
    bcs = list(bc) + [0] * (3 - ndims)
    return ndims, (ctypes.c_long * 3)(*n), (ctypes.c_int * 3)(*bcs)


def _check_c(psi_shape, c):
    ndims = len(psi_shape)
    if len(c) != ndims:
        raise ValueError("need one advector component per dimension")
    for d, cd in enumerate(c):
        want = list(psi_shape)
        want[d] += 1
        if tuple(cd.shape) != tuple(want):
            raise ValueError(f"c[{d}] has shape {cd.shape}, expected {tuple(want)}")


def step(psi, c, g=None, n_iters=2, opts=0, bc=BC_PERIODIC, n_steps=1, parallel=False):
    """Return psi advanced by n_steps MPDATA steps (input not modified).
    parallel=True runs the OpenMP build of the same source (same bits)."""
    psi = np.array(psi, dtype=np.float64, copy=True, order="C")
    c = [_f64(x) for x in c]
    _check_c(psi.shape, c)
    g = _f64(g)
    ndims, n, bcs = _dims(psi.shape, bc)
    cc = c + [None] * (3 - ndims)
    rc = _lib(parallel).orc_step(ndims, n, bcs, int(n_iters), int(opts), _ptr(psi), _ptr(g),
                         _ptr(cc[0]), _ptr(cc[1]), _ptr(cc[2]), int(n_steps))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return psi


def step_rhs(psi, c, r_pre=None, a_pre=0.0, r_post=None, a_post=0.0, g=None, n_iters=2,
             opts=0, bc=BC_PERIODIC):
    """One step of the inhomogeneous transport equation (Sect. 4.1, eq.
    gte_final_rhs): psi <- ADV(psi + a_pre r_pre) + a_post r_post, ADV one
    MPDATA step.  The paper's schemes: euler_a (eq. euler_a) r_post = R^n,
    a_post = dt; euler_b (eq. euler_b) r_pre = R^n, a_pre = dt; trapez (eq.
    trapez) r_pre = R^n, a_pre = dt/2, r_post = R^{n+1}, a_post = dt/2."""
    x = np.array(psi, dtype=np.float64, copy=True)
    if r_pre is not None:
        x = x + a_pre * _f64(r_pre)
    x = step(x, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=1)
    if r_post is not None:
        x = x + a_post * _f64(r_post)
    return x


def osc_step(psi, phi, c, a, g=None, n_iters=2, opts=0, bc=BC_PERIODIC, n_steps=1):
    """Translating oscillator d(psi)/dt + div(u psi) = omega phi,
    d(phi)/dt + div(u phi) = -omega psi under the trapezoidal rule (Sect. 4.3,
    eqs. osc_disc, trapez_osc, final_osc) with a = dt omega / 2:
    psi* = ADV(psi + a phi), phi* = ADV(phi - a psi), then
    psi = (psi* + a phi*) / (1 + a^2), phi = (phi* - a psi*) / (1 + a^2).
    The printed trapez_osc has phi^n where psi^n belongs in the second
    argument (the explicit half of -omega psi); psi^n is used here."""
    x = np.array(psi, dtype=np.float64, copy=True)
    y = np.array(phi, dtype=np.float64, copy=True)
    for _ in range(int(n_steps)):
        xs = step(x + a * y, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=1)
        ys = step(y - a * x, c, g=g, n_iters=n_iters, opts=opts, bc=bc, n_steps=1)
        den = 1.0 + a * a
        x = (xs + a * ys) / den
        y = (ys - a * xs) / den
    return x, y


def _cell_shift(a, d, s, bc):
    """a at cell i + s along d through the boundary map (open: clamp)."""
    n = a.shape[d]
    idx = np.arange(n) + s
    idx = np.clip(idx, 0, n - 1) if bc == BC_OPEN else idx % n
    return np.take(a, idx, axis=d)


def _spacing(dx, nd):
    return [float(dx)] * nd if np.isscalar(dx) else [float(v) for v in dx]


def vip_advector(num, den, num_prev, den_prev, dt, dx, eps, bc=BC_OPEN):
    """Advector at n+1/2 from prognosed velocity (Sect. 5.1-5.2).

    Velocity component d at a cell is num[d] / den (den None: num[d] is the
    velocity itself), set to 0 where den <= eps; it is extrapolated linearly
    in time, u^{n+1/2} = 1.5 u^n - 0.5 u^{n-1}, interpolated linearly to the
    walls (mean of the wall's two cells through the boundary map: open
    clamps, so an edge wall takes its cell's value) and multiplied by
    dt / dx_d.  Returns the advector components (n_d + 1 walls along d)."""
    nd = len(num)
    sp = _spacing(dx, nd)

    def vel(nm, dn):
        nm = _f64(nm)
        if dn is None:
            return nm
        dn = _f64(dn)
        ok = dn > eps
        return np.where(ok, nm / np.where(ok, dn, 1.0), 0.0)
    out = []
    for d in range(nd):
        ue = 1.5 * vel(num[d], den) - 0.5 * vel(num_prev[d], den_prev)
        n = ue.shape[d]
        f = np.arange(n + 1)
        left = np.clip(f - 1, 0, n - 1) if bc == BC_OPEN else (f - 1) % n
        right = np.clip(f, 0, n - 1) if bc == BC_OPEN else f % n
        out.append(dt / sp[d] * (0.5 * (np.take(ue, left, axis=d) +
                                         np.take(ue, right, axis=d))))
    return out


def sw_forcing(h, d, dx_d, grav=1.0, bc=BC_OPEN):
    """Pressure-gradient forcing of momentum component d in the shallow-water
    equations (eqs. shw1d, shw2d): -g h dh/dx_d, the derivative as a centred
    difference through the boundary map."""
    return -grav * h * (_cell_shift(h, d, 1, bc) - _cell_shift(h, d, -1, bc)) / (2.0 * dx_d)


def sw_step(h, q, h_prev, q_prev, dt, dx, eps=1e-8, grav=1.0, n_iters=2,
            opts=OPT_IGA | OPT_FCT | OPT_DFL, bc=BC_OPEN):
    """One step of the shallow-water system (Sect. 5.3-5.4): depth h and
    momenta q_d = u_d h, advector from vip_advector (den = h), then with the
    trapezoidal source-term scheme (Sect. 4.1)
        h^{n+1}   = ADV(h^n)                       (no source term)
        q_d^{n+1} = ADV(q_d^n + dt/2 R_d(h^n)) + dt/2 R_d(h^{n+1})
    where R_d = sw_forcing: the equation for h has no source, so the forcing
    at n+1 is known once h is advected.  Returns (h^{n+1}, [q_d^{n+1}]); the
    caller keeps (h^n, q^n) as the next step's previous level (before the
    first step the previous level equals the current one)."""
    nd = h.ndim
    sp = _spacing(dx, nd)
    C = vip_advector(q, h, q_prev, h_prev, dt, sp, eps, bc)
    hn = step(h, C, n_iters=n_iters, opts=opts, bc=bc, n_steps=1)
    qn = []
    for d in range(nd):
        x = q[d] + 0.5 * dt * sw_forcing(h, d, sp[d], grav, bc)
        x = step(x, C, n_iters=n_iters, opts=opts, bc=bc, n_steps=1)
        qn.append(x + 0.5 * dt * sw_forcing(hn, d, sp[d], grav, bc))
    return hn, qn


def sw_run(h, q, n_steps, dt, dx, **kw):
    """n_steps of sw_step from a state at rest in time (previous level =
    current level).  Returns (h, [q_d])."""
    h = _f64(h)
    q = [_f64(x) for x in q]
    hp, qp = h, q
    for _ in range(n_steps):
        hn, qn = sw_step(h, q, hp, qp, dt, dx, **kw)
        hp, qp, h, q = h, q, hn, qn
    return h, q


def diag(psi, g=None):
    """(sum of G*psi, min, max, count of non-finite values)."""
    psi = _f64(psi)
    g = _f64(g)
    ndims, n, _ = _dims(psi.shape, 0)
    out = np.zeros(3)
    bad = ctypes.c_long(0)
    rc = _lib().orc_diag(ndims, n, _ptr(psi), _ptr(g), _ptr(out), ctypes.byref(bad))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return float(out[0]), float(out[1]), float(out[2]), int(bad.value)


def courant_max(psi_shape, c, g=None, bc=BC_PERIODIC):
    c = [_f64(x) for x in c]
    _check_c(psi_shape, c)
    g = _f64(g)
    ndims, n, bcs = _dims(psi_shape, bc)
    cc = c + [None] * (3 - ndims)
    out = ctypes.c_double(0.0)
    rc = _lib().orc_courant_max(ndims, n, bcs, _ptr(g), _ptr(cc[0]), _ptr(cc[1]),
                                _ptr(cc[2]), ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return float(out.value)


def adjoint(psi0, c, lambda_T, g=None, n_iters=2, opts=0, bc=BC_PERIODIC, n_steps=1,
            ckpt_every=0, parallel=False):
    """Reverse-mode gradient of J through n_steps steps, given dJ/dpsi_T.
    parallel=True runs the OpenMP build (its forward recomputations share
    their stage loops among threads; same bits).

    Returns (grad_psi0, [grad_c0, grad_c1, ...])."""
    psi0 = _f64(psi0)
    c = [_f64(x) for x in c]
    _check_c(psi0.shape, c)
    g = _f64(g)
    lam = _f64(lambda_T)
    ndims, n, bcs = _dims(psi0.shape, bc)
    gpsi = np.zeros_like(psi0)
    gc = [np.zeros_like(x) for x in c]
    cc = c + [None] * (3 - ndims)
    gg = gc + [None] * (3 - ndims)
    lib = _lib(parallel)
    if not hasattr(lib, "orc_adjoint"):
        raise RuntimeError("oracle built without the adjoint")
    rc = lib.orc_adjoint(ndims, n, bcs, int(n_iters), int(opts), _ptr(psi0), _ptr(g),
                         _ptr(cc[0]), _ptr(cc[1]), _ptr(cc[2]), int(n_steps),
                         int(ckpt_every if ckpt_every else n_steps or 1), _ptr(lam),
                         _ptr(gpsi), _ptr(gg[0]), _ptr(gg[1]), _ptr(gg[2]))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return gpsi, gc
