"""Shared plumbing of the GPU parity tests: run the HIP library through its
C ABI and the FP64 oracle on the same seeded inputs, and compare."""
import sys

import numpy as np
import pytest
import torch

import oracle


def need_gpu():
    """GPU tests fail loudly (not skip) when the library or the GPU is missing."""
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1111_2142_amd import lwacm as L
    L.load_library()
    return L


def banner(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def gpu_run(q, shape, omega, drho, u, steps, storage=0, mask=None, wall_u=None, g=None,
            variant=0, fp16_scales=None, omega_p=None):
    """Run `steps` steps on the GPU; returns (drho, u) float64 numpy, diag, solver."""
    L = need_gpu()
    nz, ny, nx = shape
    s = L.Solver(q, nx, ny, nz, omega, storage=storage,
                 mask=None if mask is None else to_dev(mask, torch.uint8),
                 wall_u=None if wall_u is None else [list(r) for r in wall_u], g=g,
                 variant=variant, fp16_scales=fp16_scales, omega_p=omega_p)
    s.set_state(to_dev(drho), to_dev(u))
    s.step(steps)
    dr, uu = s.moments()
    torch.cuda.synchronize()
    return dr.double().cpu().numpy(), uu.double().cpu().numpy(), s


def oracle_run(q, shape, omega, drho, u, steps, mask=None, wall_u=None, g=None, rho0=1.0,
               omega_p=None):
    nz, ny, nx = shape
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=omega, mask=mask, wall_u=wall_u, g=g,
                       rho0=rho0, omega_p=omega_p)
    r, uu = oracle.run(p, 1.0 + np.asarray(drho, dtype=np.float64), u, steps)
    return r - 1.0, uu


def rel_l2(x, ref, fluid=None):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if fluid is not None:
        x = x[..., fluid]
        ref = ref[..., fluid]
    den = np.sqrt((ref ** 2).sum())
    return float(np.sqrt(((x - ref) ** 2).sum()) / (den if den > 0 else 1.0))


def fluid_of(mask, shape):
    return np.ones(shape, dtype=bool) if mask is None else (np.asarray(mask) == 0)
