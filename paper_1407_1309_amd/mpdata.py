"""Thin Python binding of libmpdata (the C ABI in include/mpdata.h).

Argument marshalling only: shapes, dtypes and devices are checked, torch
tensors are passed as raw device pointers together with torch's current HIP
stream, and every step of the computation runs in the library's kernels.
PyTorch supplies device memory (including the plan's workspace) and streams.

The library is loaded on first use from this package directory; if it is
missing the binding raises instead of computing anything another way.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpdata.so")

OK, EINVAL, EWORKSPACE, EHIP, ENONFINITE, ECANCELLED, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
OPT_FCT, OPT_IGA, OPT_TOT, OPT_ABS, OPT_DFL, OPT_KAHAN = 1, 2, 4, 8, 16, 32
BC_PERIODIC, BC_OPEN = 0, 1
F32, F64 = 0, 1
KERNEL_AUTO, KERNEL_STAGED, KERNEL_FUSED, KERNEL_PASS = 0, 1, 2, 3

EXPORTS = [
    "mpdata_workspace_bytes", "mpdata_init", "mpdata_set_stream", "mpdata_set_kernel",
    "mpdata_set_tile_rows", "mpdata_autotune",
    "mpdata_step", "mpdata_diag", "mpdata_courant_max", "mpdata_adv_adj",
    "mpdata_adj_workspace_bytes", "mpdata_batched_workspace_bytes", "mpdata_batched_init",
    "mpdata_step_batched", "mpdata_step_per_grid", "mpdata_set_batched_tiling",
    "mpdata_autotune_batched", "mpdata_timing", "mpdata_timing_read", "mpdata_step_rhs",
    "mpdata_osc_step", "mpdata_vip_advector", "mpdata_sw_step", "mpdata_set_cancel_flag",
    "mpdata_steps_done", "mpdata_tlm_step", "mpdata_tlm_workspace_bytes",
    "mpdata_diag_noalloc", "mpdata_set_step_diag", "mpdata_step_diag",
    "mpdata_destroy", "mpdata_last_error",
]


class MPDATAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmpdata status {code}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("n_dims", ctypes.c_int), ("shape", ctypes.c_int64 * 3), ("dtype", ctypes.c_int),
                ("n_iters", ctypes.c_int), ("opts", ctypes.c_uint32), ("bc", ctypes.c_int * 3),
                ("has_g", ctypes.c_int)]


_lib = None
_VP = ctypes.c_void_p


def lib():
    """Load libmpdata.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the MPDATA step has no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        DP = ctypes.POINTER(Desc)
        L.mpdata_workspace_bytes.argtypes = [DP]
        L.mpdata_workspace_bytes.restype = ctypes.c_size_t
        L.mpdata_init.argtypes = [DP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]
        L.mpdata_set_stream.argtypes = [_VP, _VP]
        L.mpdata_set_kernel.argtypes = [_VP, ctypes.c_int]
        L.mpdata_set_tile_rows.argtypes = [_VP, ctypes.c_int]
        L.mpdata_autotune.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int)]
        L.mpdata_step.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int]
        L.mpdata_diag.argtypes = [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int64)]
        L.mpdata_courant_max.argtypes = [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_double)]
        L.mpdata_set_step_diag.argtypes = [_VP, ctypes.c_int]
        L.mpdata_step_diag.argtypes = [_VP, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
        L.mpdata_diag_noalloc.argtypes = [ctypes.c_int, ctypes.c_int64, _VP, _VP, _VP,
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]
        L.mpdata_adv_adj.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_int,
                                     _VP, _VP, _VP, _VP, _VP]
        L.mpdata_adj_workspace_bytes.argtypes = [DP, ctypes.c_int, ctypes.c_int]
        L.mpdata_adj_workspace_bytes.restype = ctypes.c_size_t
        I64P = ctypes.POINTER(ctypes.c_int64)
        L.mpdata_batched_workspace_bytes.argtypes = [ctypes.c_int, I64P, ctypes.c_int, ctypes.c_int,
                                                     ctypes.c_uint32, ctypes.c_int]
        L.mpdata_batched_workspace_bytes.restype = ctypes.c_size_t
        L.mpdata_batched_init.argtypes = [ctypes.c_int, I64P, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_uint32, ctypes.c_int, _VP, ctypes.c_size_t, _VP,
                                          ctypes.POINTER(_VP)]
        L.mpdata_step_batched.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_int]
        L.mpdata_step_per_grid.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_int]
        L.mpdata_set_batched_tiling.argtypes = [_VP, ctypes.c_int, ctypes.c_int]
        L.mpdata_autotune_batched.argtypes = [_VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int)]
        L.mpdata_step_rhs.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP,
                                      ctypes.c_double]
        L.mpdata_osc_step.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_double,
                                      ctypes.c_int]
        _P3 = _VP * 3
        _D3 = ctypes.c_double * 3
        L.mpdata_vip_advector.argtypes = [_VP, _P3, _VP, _P3, _VP, ctypes.c_double, _D3,
                                          ctypes.c_double, _P3]
        L.mpdata_sw_step.argtypes = [_VP, _VP, _P3, _VP, _P3, _P3, ctypes.c_double, _D3,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.mpdata_set_cancel_flag.argtypes = [_VP, _VP]
        L.mpdata_tlm_step.argtypes = [_VP] + [_VP] * 9 + [ctypes.c_int]
        L.mpdata_tlm_workspace_bytes.argtypes = [DP]
        L.mpdata_tlm_workspace_bytes.restype = ctypes.c_size_t
        L.mpdata_steps_done.argtypes = [_VP, ctypes.POINTER(ctypes.c_int64)]
        L.mpdata_timing.argtypes = [_VP, ctypes.c_int]
        L.mpdata_timing_read.argtypes = [_VP, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_char_p)]
        L.mpdata_destroy.argtypes = [_VP]
        L.mpdata_destroy.restype = None
        L.mpdata_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise MPDATAError(rc, lib().mpdata_last_error().decode())


def _dtype_code(dtype):
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {dtype}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _wall_shape(shape, d):
    s = list(shape)
    s[d] += 1
    return tuple(s)


def _tune_key(device, kind, dtype, shape, opts, n_iters, bc, has_g):
    """Autotune cache key: device architecture and everything that selects
    a kernel and its launch shape."""
    arch = torch.cuda.get_device_properties(device).gcnArchName
    return json.dumps([arch, kind, str(dtype), shape, int(opts), int(n_iters), bc, bool(has_g)],
                      default=list)


def _cache_get(path, key):
    try:
        with open(path) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def _cache_put(path, key, value):
    """Add one entry (read-modify-write through a temporary file and an
    atomic rename, so a concurrent reader never sees a partial file)."""
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[key] = value
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class Plan:
    """A single-grid plan: validated descriptor + workspace + stream.

    shape: cells per dimension (1-3 entries); bc: int or per-dimension list.
    adj_steps / ckpt_every: size the workspace for mpdata_adv_adj as well;
    tlm: size it for mpdata_tlm_step as well."""

    def __init__(self, shape, dtype=torch.float64, n_iters=2, opts=0, bc=BC_PERIODIC,
                 has_g=False, device="cuda", kernel=KERNEL_AUTO, adj_steps=None, ckpt_every=None,
                 tlm=False):
        self.shape = tuple(int(s) for s in shape)
        self.nd = len(self.shape)
        self.dtype = dtype
        self.device = torch.device(device)
        bcs = [bc] * self.nd if isinstance(bc, int) else list(bc)
        d = Desc()
        d.n_dims = self.nd
        for k in range(3):
            d.shape[k] = self.shape[k] if k < self.nd else 1
            d.bc[k] = bcs[k] if k < self.nd else 0
        d.dtype = _dtype_code(dtype)
        d.n_iters = int(n_iters)
        d.opts = int(opts)
        d.has_g = 1 if has_g else 0
        self.desc = d
        L = lib()
        need = L.mpdata_workspace_bytes(ctypes.byref(d))
        if need == 0:
            # let init report the reason
            self._handle = _VP()
            _check(L.mpdata_init(ctypes.byref(d), None, 0, None, ctypes.byref(self._handle)))
        if adj_steps is not None:
            adj = L.mpdata_adj_workspace_bytes(ctypes.byref(d), int(adj_steps), int(ckpt_every))
            if adj == 0:
                raise ValueError("bad adjoint sizing (need 1 <= ckpt_every <= adj_steps)")
            need = max(need, adj)
        if tlm:
            need = max(need, L.mpdata_tlm_workspace_bytes(ctypes.byref(d)))
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self._ws_bytes = need
        self._handle = _VP()
        _check(L.mpdata_init(ctypes.byref(d), ctypes.c_void_p(self._ws_ptr), need,
                             _stream(self.device), ctypes.byref(self._handle)))
        if kernel != KERNEL_AUTO:
            self.set_kernel(kernel)

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h and _lib is not None:
            _lib.mpdata_destroy(h)
            self._handle = None

    def set_kernel(self, kernel):
        _check(lib().mpdata_set_kernel(self._handle, int(kernel)))

    def set_cancel_flag(self, flag):
        """Stop flag for step(): a host numpy int32 array of one element (kept
        referenced here), or None to remove it.  While set, step() waits for
        each step before launching the next and returns early, raising
        MPDATAError with code ECANCELLED, once flag[0] != 0."""
        if flag is None:
            self._cancel = None
            _check(lib().mpdata_set_cancel_flag(self._handle, None))
            return
        if flag.dtype != np.int32 or flag.size != 1 or not flag.flags["C_CONTIGUOUS"]:
            raise ValueError("flag: need a contiguous numpy int32 array of one element")
        self._cancel = flag
        _check(lib().mpdata_set_cancel_flag(self._handle, ctypes.c_void_p(flag.ctypes.data)))

    def steps_done(self):
        """Steps completed by the last step() call."""
        out = ctypes.c_int64(0)
        _check(lib().mpdata_steps_done(self._handle, ctypes.byref(out)))
        return int(out.value)

    def set_tile_rows(self, rows):
        _check(lib().mpdata_set_tile_rows(self._handle, int(rows)))

    def timing(self, max_launches):
        """Time the next max_launches step launches with a pair of HIP events
        around them (0 switches timing off)."""
        _check(lib().mpdata_timing(self._handle, int(max_launches)))

    def timing_read(self):
        """(mean milliseconds per launch, launches, kernel name) of the timed
        launches; waits for them."""
        tot = ctypes.c_double(0.0)
        n = ctypes.c_int(0)
        name = ctypes.c_char_p()
        _check(lib().mpdata_timing_read(self._handle, ctypes.byref(tot), ctypes.byref(n),
                                        ctypes.byref(name)))
        return (tot.value / n.value if n.value else float("nan"), n.value,
                (name.value or b"").decode())

    def autotune(self, psi, c, g=None, cache=None):
        """Pick the fused kernel's chunk length by timing candidates on these
        inputs (psi is not modified); returns the chosen rows per chunk.
        cache: path of a JSON file of earlier choices keyed by device
        architecture, dtype, shape, options, pass count and boundaries; a
        hit sets the stored chunk length without timing, a miss times and
        stores."""
        self._check_cell(psi, "psi")
        self._check_cell(g, "g")
        cp = self._check_walls(c)
        key = None
        if cache is not None:
            key = _tune_key(self.device, "single", self.dtype, self.shape, self.desc.opts,
                            self.desc.n_iters, list(self.desc.bc)[: self.nd], self.desc.has_g)
            hit = _cache_get(cache, key)
            if hit is not None:
                self.set_tile_rows(int(hit["tile_rows"]))
                return int(hit["tile_rows"])
        self._bind_stream()
        out = ctypes.c_int(0)
        _check(lib().mpdata_autotune(self._handle, _ptr(psi), _ptr(g), cp[0], cp[1], cp[2],
                                     ctypes.byref(out)))
        if key is not None:
            _cache_put(cache, key, {"tile_rows": int(out.value)})
        return out.value

    def _bind_stream(self):
        _check(lib().mpdata_set_stream(self._handle, _stream(self.device)))

    def _check_cell(self, t, name):
        if t is None:
            return
        if t.device != self.device and not (t.is_cuda and self.device.type == "cuda"):
            raise ValueError(f"{name} must be on {self.device}")
        if t.dtype != self.dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name}: need contiguous {self.dtype} of shape {self.shape}, got "
                             f"{t.dtype} {tuple(t.shape)} contiguous={t.is_contiguous()}")

    def _check_walls(self, c):
        if len(c) != self.nd:
            raise ValueError(f"need {self.nd} advector components")
        for d, cd in enumerate(c):
            want = _wall_shape(self.shape, d)
            if cd.dtype != self.dtype or tuple(cd.shape) != want or not cd.is_contiguous() \
                    or not cd.is_cuda:
                raise ValueError(f"c[{d}]: need contiguous {self.dtype} of shape {want} on the GPU")
        return [_ptr(x) for x in c] + [None] * (3 - self.nd)

    def step(self, psi, c, g=None, n_steps=1):
        """Advance psi in place by n_steps steps on torch's current stream."""
        self._check_cell(psi, "psi")
        self._check_cell(g, "g")
        cp = self._check_walls(c)
        self._bind_stream()
        _check(lib().mpdata_step(self._handle, _ptr(psi), _ptr(g), cp[0], cp[1], cp[2],
                                 int(n_steps)))
        return psi

    def step_rhs(self, psi, c, r_pre=None, a_pre=0.0, r_post=None, a_post=0.0, g=None):
        """One step of the inhomogeneous transport equation in place:
        psi <- ADV(psi + a_pre r_pre) + a_post r_post."""
        self._check_cell(psi, "psi")
        self._check_cell(g, "g")
        self._check_cell(r_pre, "r_pre")
        self._check_cell(r_post, "r_post")
        cp = self._check_walls(c)
        self._bind_stream()
        _check(lib().mpdata_step_rhs(self._handle, _ptr(psi), _ptr(g), cp[0], cp[1], cp[2],
                                     _ptr(r_pre), float(a_pre), _ptr(r_post), float(a_post)))
        return psi

    def osc_step(self, psi, phi, c, a, n_steps=1, g=None):
        """n_steps trapezoidal steps of the translating oscillator (in place),
        a = dt * omega / 2."""
        self._check_cell(psi, "psi")
        self._check_cell(phi, "phi")
        self._check_cell(g, "g")
        cp = self._check_walls(c)
        self._bind_stream()
        _check(lib().mpdata_osc_step(self._handle, _ptr(psi), _ptr(phi), _ptr(g), cp[0], cp[1],
                                     cp[2], float(a), int(n_steps)))
        return psi, phi

    def _cells3(self, ts, name):
        if len(ts) != self.nd:
            raise ValueError(f"{name}: need {self.nd} cell arrays")
        for d, t in enumerate(ts):
            if t is None:
                raise ValueError(f"{name}[{d}] is None")
            self._check_cell(t, f"{name}[{d}]")
        return (_VP * 3)(*([x.data_ptr() for x in ts] + [None] * (3 - self.nd)))

    def _spacing(self, dx):
        sp = [float(dx)] * self.nd if isinstance(dx, (int, float)) else [float(v) for v in dx]
        if len(sp) != self.nd:
            raise ValueError(f"need {self.nd} grid spacings")
        return (ctypes.c_double * 3)(*(sp + [1.0] * (3 - self.nd)))

    def vip_advector(self, num, den, num_prev, den_prev, dt, dx, eps, c):
        """Advector at n+1/2 from prognosed velocity num[d] / den (den None:
        num[d] is the velocity) at levels n and n-1, written into c."""
        self._check_cell(den, "den")
        self._check_cell(den_prev, "den_prev")
        self._check_walls(c)
        cp = (_VP * 3)(*([x.data_ptr() for x in c] + [None] * (3 - self.nd)))
        self._bind_stream()
        _check(lib().mpdata_vip_advector(self._handle, self._cells3(num, "num"), _ptr(den),
                                         self._cells3(num_prev, "num_prev"), _ptr(den_prev),
                                         float(dt), self._spacing(dx), float(eps), cp))
        return c

    def sw_step(self, h, q, h_prev, q_prev, c, dt, dx, grav=1.0, eps=1e-8, n_steps=1):
        """n_steps shallow-water steps in place (depth h, momenta q, previous
        level h_prev, q_prev; c receives the last step's advector)."""
        self._check_cell(h, "h")
        self._check_cell(h_prev, "h_prev")
        self._check_walls(c)
        cp = (_VP * 3)(*([x.data_ptr() for x in c] + [None] * (3 - self.nd)))
        self._bind_stream()
        _check(lib().mpdata_sw_step(self._handle, _ptr(h), self._cells3(q, "q"), _ptr(h_prev),
                                    self._cells3(q_prev, "q_prev"), cp, float(dt),
                                    self._spacing(dx), float(grav), float(eps), int(n_steps)))
        return h, q

    def diag(self, psi, g=None):
        """(sum G psi, min, max, n_nonfinite); waits for the result."""
        self._check_cell(psi, "psi")
        self._check_cell(g, "g")
        self._bind_stream()
        out = (ctypes.c_double * 3)()
        bad = ctypes.c_int64(0)
        rc = lib().mpdata_diag(self._handle, _ptr(psi), _ptr(g), out, ctypes.byref(bad))
        if rc not in (OK, ENONFINITE):
            _check(rc)
        return out[0], out[1], out[2], int(bad.value)

    def set_step_diag(self, on=True):
        """Have every later step call form the diagnostics of its result."""
        _check(lib().mpdata_set_step_diag(self._handle, 1 if on else 0))

    def step_diag(self):
        """(sum G psi, min, max, n_nonfinite) of the last step call's result."""
        self._bind_stream()
        out = (ctypes.c_double * 3)()
        bad = ctypes.c_int64(0)
        rc = lib().mpdata_step_diag(self._handle, out, ctypes.byref(bad))
        if rc not in (OK, ENONFINITE):
            _check(rc)
        return out[0], out[1], out[2], int(bad.value)

    def courant_max(self, c, g=None):
        self._check_cell(g, "g")
        cp = self._check_walls(c)
        self._bind_stream()
        out = ctypes.c_double(0.0)
        _check(lib().mpdata_courant_max(self._handle, _ptr(g), cp[0], cp[1], cp[2],
                                        ctypes.byref(out)))
        return out.value

    def tlm_step(self, psi, dpsi, c, dc=None, g=None, n_steps=1):
        """n_steps tangent-linear steps in place: psi advances, dpsi becomes
        the derivative of the result along (dpsi, dc) (dc None: zero)."""
        self._check_cell(psi, "psi")
        self._check_cell(dpsi, "dpsi")
        self._check_cell(g, "g")
        cp = self._check_walls(c)
        dp = [None] * 3 if dc is None else self._check_walls(dc)
        self._bind_stream()
        _check(lib().mpdata_tlm_step(self._handle, _ptr(psi), _ptr(dpsi), _ptr(g), cp[0], cp[1],
                                     cp[2], dp[0], dp[1], dp[2], int(n_steps)))
        return psi, dpsi

    def adv_adj(self, psi0, c, lambda_T, g=None, n_steps=1, ckpt_every=None):
        """Gradient of J w.r.t. psi0 and c, given lambda_T = dJ/dpsi_T."""
        ckpt_every = int(ckpt_every or n_steps)
        self._check_cell(psi0, "psi0")
        self._check_cell(lambda_T, "lambda_T")
        self._check_cell(g, "g")
        cp = self._check_walls(c)
        gpsi = torch.empty_like(psi0)
        gc = [torch.empty_like(x) for x in c]
        gp = [_ptr(x) for x in gc] + [None] * (3 - self.nd)
        self._bind_stream()
        _check(lib().mpdata_adv_adj(self._handle, _ptr(psi0), _ptr(g), cp[0], cp[1], cp[2],
                                    int(n_steps), ckpt_every, _ptr(lambda_T), _ptr(gpsi),
                                    gp[0], gp[1], gp[2]))
        return gpsi, gc


class BatchedPlan:
    """Many independent 2-D grids of uneven size in packed buffers."""

    def __init__(self, shapes, dtype=torch.float32, n_iters=2, opts=OPT_FCT, bc=BC_PERIODIC,
                 device="cuda"):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.n = len(self.shapes)
        self.dtype = dtype
        self.device = torch.device(device)
        self.n_iters, self.opts, self.bc = int(n_iters), int(opts), int(bc)
        flat = (ctypes.c_int64 * (2 * self.n))(*[v for s in self.shapes for v in s])
        L = lib()
        need = L.mpdata_batched_workspace_bytes(self.n, flat, _dtype_code(dtype), int(n_iters),
                                                int(opts), int(bc))
        if need == 0:
            raise ValueError("invalid batched shapes (each side must be >= 3)")
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = base + (-base) % 256
        self._handle = _VP()
        _check(L.mpdata_batched_init(self.n, flat, _dtype_code(dtype), int(n_iters), int(opts),
                                     int(bc), ctypes.c_void_p(self._ws_ptr), need,
                                     _stream(self.device), ctypes.byref(self._handle)))
        self.n_psi = sum(a * b for a, b in self.shapes)
        self.n_c0 = sum((a + 1) * b for a, b in self.shapes)
        self.n_c1 = sum(a * (b + 1) for a, b in self.shapes)

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h and _lib is not None:
            _lib.mpdata_destroy(h)
            self._handle = None

    def _check(self, psi, c0, c1):
        for t, n, name in ((psi, self.n_psi, "psi"), (c0, self.n_c0, "c0"), (c1, self.n_c1, "c1")):
            if t.dtype != self.dtype or t.numel() != n or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name}: need {n} contiguous {self.dtype} values on the GPU")
        _check(lib().mpdata_set_stream(self._handle, _stream(self.device)))

    def step(self, psi, c0, c1, n_steps=1, use_graph=True):
        self._check(psi, c0, c1)
        _check(lib().mpdata_step_batched(self._handle, _ptr(psi), _ptr(c0), _ptr(c1),
                                         int(n_steps), 1 if use_graph else 0))
        return psi

    def set_tiling(self, tile_rows=0, xcd_order=False):
        """Chunk length (0 = default) and tile order of the batched launch."""
        _check(lib().mpdata_set_stream(self._handle, _stream(self.device)))
        _check(lib().mpdata_set_batched_tiling(self._handle, int(tile_rows), 1 if xcd_order else 0))

    def autotune(self, psi, c0, c1, cache=None):
        """Pick chunk length and tile order by timing one batched step per
        candidate on these buffers (psi is not modified); returns both.
        cache: JSON file of earlier choices (see Plan.autotune), keyed here
        by the list of grid shapes as well."""
        self._check(psi, c0, c1)
        key = None
        if cache is not None:
            key = _tune_key(self.device, "batched", self.dtype, self.shapes, self.opts,
                            self.n_iters, self.bc, False)
            hit = _cache_get(cache, key)
            if hit is not None:
                self.set_tiling(int(hit["tile_rows"]), bool(hit["xcd_order"]))
                return int(hit["tile_rows"]), bool(hit["xcd_order"])
        rows, xcd = ctypes.c_int(0), ctypes.c_int(0)
        _check(lib().mpdata_autotune_batched(self._handle, _ptr(psi), _ptr(c0), _ptr(c1),
                                             ctypes.byref(rows), ctypes.byref(xcd)))
        if key is not None:
            _cache_put(cache, key, {"tile_rows": int(rows.value), "xcd_order": bool(xcd.value)})
        return rows.value, bool(xcd.value)

    def step_per_grid(self, psi, c0, c1, n_steps=1):
        self._check(psi, c0, c1)
        _check(lib().mpdata_step_per_grid(self._handle, _ptr(psi), _ptr(c0), _ptr(c1),
                                          int(n_steps)))
        return psi

    def pack(self, arrays, which):
        """Concatenate per-grid arrays (cells / c0 walls / c1 walls) into one
        packed device tensor."""
        return torch.cat([torch.as_tensor(a, dtype=self.dtype).reshape(-1) for a in arrays]) \
            .to(self.device).contiguous()

    def unpack(self, packed, which):
        out, off = [], 0
        for a, b in self.shapes:
            shp = {"psi": (a, b), "c0": (a + 1, b), "c1": (a, b + 1)}[which]
            n = shp[0] * shp[1]
            out.append(packed[off:off + n].reshape(shp))
            off += n
        return out


def diag_noalloc(psi, g=None):
    """(sum G psi, min, max, n_nonfinite) of a contiguous device field
    without a plan or workspace (mpdata_diag_noalloc: the library's fixed
    scratch array); runs on torch's current stream and waits."""
    if not (psi.is_cuda and psi.is_contiguous()):
        raise ValueError("psi must be a contiguous device tensor")
    if g is not None and (g.dtype != psi.dtype or g.shape != psi.shape or not g.is_contiguous()):
        raise ValueError("g must match psi")
    out = (ctypes.c_double * 3)()
    bad = ctypes.c_int64(0)
    rc = lib().mpdata_diag_noalloc(_dtype_code(psi.dtype), psi.numel(), _ptr(psi), _ptr(g),
                                   _stream(psi.device), out, ctypes.byref(bad))
    if rc not in (OK, ENONFINITE):
        _check(rc)
    return out[0], out[1], out[2], int(bad.value)


def step(psi, c, g=None, n_iters=2, opts=0, bc=BC_PERIODIC, n_steps=1, kernel=KERNEL_AUTO):
    """One-shot convenience: build a plan and advance psi in place."""
    p = Plan(tuple(psi.shape), dtype=psi.dtype, n_iters=n_iters, opts=opts, bc=bc,
             has_g=g is not None, device=psi.device, kernel=kernel)
    return p.step(psi, c, g=g, n_steps=n_steps)


class MPDATAFunction(torch.autograd.Function):
    """psi_T = n_steps MPDATA steps of psi0 with the advector c (G constant).

    Backward runs mpdata_adv_adj (checkpointed reverse sweep in the library),
    giving gradients with respect to psi0 and every advector component;
    forward mode (torch.func.jvp, forward-mode AD) runs mpdata_tlm_step."""

    @staticmethod
    def forward(ctx, psi0, plan, n_steps, ckpt_every, g, *c):
        psi = psi0.detach().clone().contiguous()
        cs = [x.detach().contiguous() for x in c]
        plan.step(psi, cs, g=g, n_steps=n_steps)
        ctx.save_for_backward(psi0.detach(), *cs)
        ctx.save_for_forward(psi0.detach(), *cs)
        ctx.plan, ctx.n_steps, ctx.ckpt, ctx.g = plan, n_steps, ckpt_every, g
        return psi

    @staticmethod
    def jvp(ctx, dpsi0, _plan, _n, _ck, _g, *dc):
        """Forward mode: mpdata_tlm_step along (dpsi0, dc) (the plan needs
        tlm=True)."""
        psi0, *c = ctx.saved_tensors
        psi = psi0.clone()
        dpsi = (torch.zeros_like(psi0) if dpsi0 is None else dpsi0.detach().clone()).contiguous()
        dcs = None
        if any(x is not None for x in dc):
            dcs = [torch.zeros_like(cd) if x is None else x.detach().contiguous()
                   for x, cd in zip(dc, c)]
        ctx.plan.tlm_step(psi, dpsi, c, dc=dcs, g=ctx.g, n_steps=ctx.n_steps)
        return dpsi

    @staticmethod
    def backward(ctx, grad_out):
        psi0, *c = ctx.saved_tensors
        gpsi, gc = ctx.plan.adv_adj(psi0, c, grad_out.contiguous(), g=ctx.g,
                                    n_steps=ctx.n_steps, ckpt_every=ctx.ckpt)
        return (gpsi, None, None, None, None, *gc)


def advance(psi0, c, plan, n_steps, ckpt_every=None, g=None):
    """Differentiable n_steps advance (see MPDATAFunction); the plan must be
    created with adj_steps >= n_steps and the same ckpt_every."""
    return MPDATAFunction.apply(psi0, plan, int(n_steps), int(ckpt_every or n_steps), g, *c)
