"""Helpers for the GPU parity tests (HIP path via the C ABI vs the oracle)."""
import numpy as np
import torch

from paper_1407_1309_amd import mpdata

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def rel_l2(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return np.linalg.norm((a - ref).ravel()) / (den if den > 0 else 1.0)


def as_dtype(x, dtype):
    """Round to the run's dtype and widen back (what the oracle consumes)."""
    if x is None:
        return None
    if dtype == torch.float32:
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)


def dev(x, dtype):
    if x is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype).contiguous()


def gpu_run(psi, c, g, dtype, n_iters, opts, bc, n_steps, kernel=mpdata.KERNEL_AUTO):
    plan = mpdata.Plan(psi.shape, dtype=dtype, n_iters=n_iters, opts=opts, bc=bc,
                       has_g=g is not None, kernel=kernel)
    p = dev(psi, dtype)
    cd = [dev(x, dtype) for x in c]
    gd = dev(g, dtype)
    plan.step(p, cd, g=gd, n_steps=n_steps)
    torch.cuda.synchronize()
    return p.double().cpu().numpy()
