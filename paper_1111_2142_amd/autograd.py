"""Differentiable LW-ACM runs: ``torch.autograd.Function`` over the HIP
forward step and the hand-written reverse step of the library.

Forward: run ``nsteps`` steps from (rho0 - 1, u0), saving the state (storage
format) every ``K`` steps.  Backward: seed mu from the loss cotangent of the
final state, then for each segment from last to first recompute the
segment's states from its checkpoint into a K-slot buffer (one library call)
and apply the K reverse steps (one call; two per launch where the library
supports it).  The omega gradient is accumulated in FP64 on the
device.  Every arithmetic step runs in the library's kernels; this module
only sequences the calls.
"""
from typing import Optional, Sequence

import torch

from . import lwacm as L


class _Run(torch.autograd.Function):
    @staticmethod
    def forward(ctx, drho0, u0, omega, lattice, shape, nsteps, K, storage, mask, wall_u, g):
        nz, ny, nx = shape
        om = float(omega.detach().cpu()) if torch.is_tensor(omega) else float(omega)
        solver = L.Solver(lattice, nx, ny, nz, om, storage=storage, mask=mask, wall_u=wall_u,
                          g=g, device=u0.device)
        solver.set_state(drho0.detach(), u0.detach())
        checkpoints = []
        t = 0
        while t < nsteps:
            checkpoints.append((t, solver.save_state()))
            k = min(K, nsteps - t)
            solver.step(k)
            t += k
        drho_T, u_T = solver.moments()
        ctx.solver = solver
        ctx.checkpoints = checkpoints
        ctx.final_state = solver.save_state()
        ctx.nsteps, ctx.K = nsteps, K
        ctx.omega_is_tensor = torch.is_tensor(omega)
        ctx.omega_shape = omega.shape if torch.is_tensor(omega) else None
        ctx.omega_dtype = omega.dtype if torch.is_tensor(omega) else None
        return drho_T, u_T

    @staticmethod
    def backward(ctx, g_drho, g_u):
        solver = ctx.solver
        dev = solver.device
        shape = solver.shape
        D = solver.D
        lam = torch.zeros((D + 1,) + shape, dtype=torch.float32, device=dev)
        if g_drho is not None:
            lam[0] = g_drho
        if g_u is not None:
            lam[1:] = g_u
        mu = torch.empty_like(lam)
        mu_next = torch.empty_like(lam)
        dw = torch.zeros(1, dtype=torch.float64, device=dev)
        L.lwacm_adjoint_seed(solver.ctx, ctx.final_state, lam, mu)
        # the segment's states, slot j = the state at step t0 + j: the
        # checkpoint, then the recomputed ones (lwacm_forward_states), then the
        # segment's reverse steps in one call (lwacm_adjoint_sweep, two per
        # launch where the library can; bitwise the separate calls' result)
        sb = solver.state_bytes
        seg = torch.empty(min(ctx.K, max(ctx.nsteps, 1)) * sb, dtype=torch.uint8, device=dev)
        for (t0, ckpt) in reversed(ctx.checkpoints):
            nseg = min(ctx.K, ctx.nsteps - t0)
            seg[:sb].copy_(ckpt)
            if nseg > 1:
                L.lwacm_forward_states(solver.ctx, ckpt, t0, nseg - 1, seg[sb:nseg * sb])
            L.lwacm_adjoint_sweep(solver.ctx, seg, t0, nseg, mu, mu_next, dw)
        if ctx.nsteps == 0:
            mu = lam
        grad_drho0 = mu[0].clone()
        grad_u0 = mu[1:].clone()
        grad_omega = None
        if ctx.omega_is_tensor:
            # accumulated in FP64 on the device; handed back in omega's own dtype
            grad_omega = dw.to(ctx.omega_dtype).reshape(ctx.omega_shape)
        solver.close()
        ctx.solver = None
        return (grad_drho0, grad_u0, grad_omega, None, None, None, None, None, None, None, None)


def lwacm_run(drho0: torch.Tensor, u0: torch.Tensor, omega, nsteps: int, lattice: int,
              K: int = 100, storage: int = L.LWACM_FP32, mask: Optional[torch.Tensor] = None,
              wall_u: Optional[Sequence[Sequence[float]]] = None,
              g: Optional[Sequence[float]] = None):
    """Differentiable run of ``nsteps`` LW-ACM steps; returns (rho_T - 1, u_T).

    ``drho0`` has shape (nz, ny, nx), ``u0`` shape (D, nz, ny, nx) (float32,
    on the GPU); ``omega`` is a float or a 0-dim tensor (then it receives
    dL/domega in its own dtype).  Gradients reach ``drho0``, ``u0`` and
    ``omega``.  With moving walls, the density rho0 of the wall term (Eq.
    ACM2.0ccccbb: the mean fluid density, computed once from the initial state)
    is a constant of the problem, as the paper holds it: dL/d(drho0) is the
    derivative through the steps with rho0 fixed, and carries no term from
    rho0's own dependence on drho0.
    """
    if nsteps < 0 or K < 1:
        raise ValueError("nsteps must be >= 0 and K >= 1")
    shape = tuple(drho0.shape)
    if len(shape) != 3:
        raise ValueError("drho0 must have shape (nz, ny, nx)")
    return _Run.apply(drho0, u0, omega, lattice, shape, int(nsteps), int(K), storage, mask,
                      wall_u, g)
