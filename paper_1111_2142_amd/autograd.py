"""Differentiable LW-ACM runs: ``torch.autograd.Function`` over the HIP
forward step and the hand-written reverse step of the library.

Forward: run ``nsteps`` steps from (rho0 - 1, u0), saving the state (storage
format) every ``K`` steps.  Backward: seed mu from the loss cotangent of the
final state, then for each segment from last to first recompute the
segment's states from its checkpoint into a K-slot buffer (one library call)
and apply the K reverse steps (one call; two per launch where the library
supports it).  The omega gradient is accumulated in FP64 on the
device.  ``lwacm_run_thermal`` does the same for a flow with its temperature
field.  Every arithmetic step runs in the library's kernels; this module
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


class _ThermalRun(torch.autograd.Function):
    """Flow and temperature together (lwacm_set_thermal).  Checkpoints hold the
    state and T every K steps; the backward pass recomputes a segment one
    step at a time (states and temperatures of every step) and runs, for each
    step from the last, the flow's reverse step and then the temperature's
    (lwacm_adjoint_thermal_step), which adds the flow cotangent dL/du_t of
    the temperature step to the flow sweep."""

    @staticmethod
    def forward(ctx, drho0, u0, T0, omega, omega_t, lattice, shape, nsteps, K, mask, wall_u,
                wall_T, q_t, g):
        nz, ny, nx = shape
        om = float(omega.detach().cpu()) if torch.is_tensor(omega) else float(omega)
        solver = L.Solver(lattice, nx, ny, nz, om, mask=mask, wall_u=wall_u, g=g,
                          device=u0.device)
        solver.set_state(drho0.detach(), u0.detach())
        solver.set_thermal(omega_t, T0.detach(), wall_T=wall_T, q_t=q_t)
        checkpoints = []
        t = 0
        while t < nsteps:
            checkpoints.append((t, solver.save_state(), solver.temperature()))
            k = min(K, nsteps - t)
            solver.step(k)
            t += k
        drho_T, u_T = solver.moments()
        T_T = solver.temperature()
        ctx.solver = solver
        ctx.checkpoints = checkpoints
        ctx.final_state = solver.save_state()
        ctx.nsteps, ctx.K = nsteps, K
        ctx.thermal = (omega_t, wall_T, q_t)
        ctx.omega_is_tensor = torch.is_tensor(omega)
        ctx.omega_shape = omega.shape if torch.is_tensor(omega) else None
        ctx.omega_dtype = omega.dtype if torch.is_tensor(omega) else None
        return drho_T, u_T, T_T

    @staticmethod
    def backward(ctx, g_drho, g_u, g_T):
        solver = ctx.solver
        dev = solver.device
        shape = solver.shape
        D = solver.D
        lam = torch.zeros((D + 1,) + shape, dtype=torch.float32, device=dev)
        if g_drho is not None:
            lam[0] = g_drho
        if g_u is not None:
            lam[1:] = g_u
        lamT = torch.zeros(shape, dtype=torch.float32, device=dev)
        if g_T is not None:
            lamT.copy_(g_T)
        lamT_next = torch.empty_like(lamT)
        mu = torch.empty_like(lam)
        mu_next = torch.empty_like(lam)
        dw = torch.zeros(1, dtype=torch.float64, device=dev)
        L.lwacm_adjoint_seed(solver.ctx, ctx.final_state, lam, mu)
        omega_t, wall_T, q_t = ctx.thermal
        for (t0, ckpt, Tck) in reversed(ctx.checkpoints):
            nseg = min(ctx.K, ctx.nsteps - t0)
            solver.load_state(ckpt, t0)
            solver.set_thermal(omega_t, Tck, wall_T=wall_T, q_t=q_t)
            states, temps = [], []
            for j in range(nseg):
                states.append(solver.save_state())
                temps.append(solver.temperature())
                if j + 1 < nseg:
                    solver.step(1)
            for j in range(nseg - 1, -1, -1):
                final = t0 + j == 0
                L.lwacm_adjoint_step(solver.ctx, states[j], mu, mu_next, dw, final)
                L.lwacm_adjoint_thermal_step(solver.ctx, states[j], temps[j], lamT, lamT_next,
                                             mu_next, final)
                mu, mu_next = mu_next, mu
                lamT, lamT_next = lamT_next, lamT
        if ctx.nsteps == 0:
            mu = lam
        grad_omega = None
        if ctx.omega_is_tensor:
            grad_omega = dw.to(ctx.omega_dtype).reshape(ctx.omega_shape)
        grads = (mu[0].clone(), mu[1:].clone(), lamT.clone(), grad_omega)
        solver.close()
        ctx.solver = None
        return grads + (None,) * 10


def lwacm_run_thermal(drho0: torch.Tensor, u0: torch.Tensor, T0: torch.Tensor, omega,
                      omega_t: float, nsteps: int, lattice: int, K: int = 100,
                      mask: Optional[torch.Tensor] = None,
                      wall_u: Optional[Sequence[Sequence[float]]] = None,
                      wall_T: Optional[Sequence[float]] = None, q_t: int = 0,
                      g: Optional[Sequence[float]] = None):
    """Differentiable run of ``nsteps`` steps of the flow and its temperature
    field (thermal LW-ACM, FP32); returns (rho_T - 1, u_T, T_T).

    Arguments as for lwacm_run, plus ``T0`` (nz, ny, nx), the temperature
    relaxation ``omega_t``, the walls' temperatures ``wall_T`` by mask id
    (NaN: adiabatic) and the temperature lattice ``q_t`` (0: the flow's; 5 or
    7: D2Q5 / D3Q7).  Gradients reach ``drho0``, ``u0``, ``T0`` and
    ``omega``; omega_t and the wall temperatures are constants.
    """
    if nsteps < 0 or K < 1:
        raise ValueError("nsteps must be >= 0 and K >= 1")
    shape = tuple(drho0.shape)
    if len(shape) != 3 or tuple(T0.shape) != shape:
        raise ValueError("drho0 and T0 must have shape (nz, ny, nx)")
    return _ThermalRun.apply(drho0, u0, T0, omega, float(omega_t), lattice, shape, int(nsteps),
                             int(K), mask, wall_u, wall_T, int(q_t), g)


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
