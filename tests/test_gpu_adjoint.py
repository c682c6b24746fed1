"""GPU parity of the hand-written reverse step and of the checkpointed
differentiable run against the FP64 oracle's reverse mode and against
central finite differences of the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from gpu_helpers import banner, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _single_step_case(case):
    rng = np.random.Generator(np.random.PCG64(31))
    mask = wall = g = None
    if case.startswith("d2q9"):
        q, d, shape = 9, 2, (1, 40, 52)
    else:
        q, d, shape = 19, 3, (12, 14, 18)
    nz, ny, nx = shape
    if "walls" in case:
        mask = (wl.channel_mask(nx, ny, moving_top=True) if q == 9
                else wl.slab_mask_3d(nx, ny, nz, moving_top=True))
        wall = wl.wall_table((0.05, 0.0, 0.02))
    if "force" in case:
        g = (2e-3, -1e-3) if q == 9 else (2e-3, -1e-3, 5e-4)
    drho, u = wl.random_state(shape, d, seed=8, du=0.05, drho=0.02)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    lam = rng.standard_normal((d + 1,) + shape).astype(np.float32).astype(np.float64)
    if mask is not None:
        lam[:, mask != 0] = 0
    return q, d, shape, mask, wall, g, drho, u, lam


@pytest.mark.parametrize("case", ["d2q9_periodic", "d2q9_walls_force", "d3q19_periodic",
                                  "d3q19_walls_force"])
@pytest.mark.parametrize("final", [True, False])
def test_single_reverse_step_matches_oracle(case, final):
    """lwacm_adjoint_seed + lwacm_adjoint_step on one step reproduce the
    oracle's reverse mode (cotangents of the inputs and dL/domega)."""
    L = need_gpu()
    banner(f"reverse step {case} final={final}")
    q, d, shape, mask, wall, g, drho, u, lam = _single_step_case(case)
    nz, ny, nx = shape
    omega = 1.55
    s = L.Solver(q, nx, ny, nz, omega, mask=None if mask is None else to_dev(mask, torch.uint8),
                 wall_u=None if wall is None else [list(r) for r in wall], g=g)
    # state_t and state_{t+1} on the device (the reverse step needs both)
    s.set_state(to_dev(drho), to_dev(u))
    st0 = s.save_state()
    s.step(1)
    st1 = s.save_state()
    dr1, u1 = s.moments()
    mu = torch.empty((d + 1,) + shape, dtype=torch.float32, device="cuda")
    out = torch.empty_like(mu)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    L.lwacm_adjoint_seed(s.ctx, st1, to_dev(lam), mu)
    L.lwacm_adjoint_step(s.ctx, st0, mu, out, dw, final)
    torch.cuda.synchronize()
    rho0 = 1.0 if mask is None else 1.0 + drho[mask == 0].mean()
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=omega, mask=mask, wall_u=wall, g=g,
                       rho0=rho0)
    lr, lu, dwo = oracle.vjp(p, 1 + drho, u, lam[0], lam[1:])
    got = out.double().cpu().numpy()
    if final:
        assert rel_l2(got[0], lr) < 1e-5
        assert rel_l2(got[1:], lu) < 1e-5
    else:
        # mu of the previous step: fold u = J/rho with the oracle's own state
        inv = 1.0 / (1.0 + drho)
        mu_r = lr - (lu * u).sum(0) * inv
        mu_j = lu * inv
        if mask is not None:
            mu_r[mask != 0] = 0
            mu_j[:, mask != 0] = 0
        assert rel_l2(got[0], mu_r) < 1e-5
        assert rel_l2(got[1:], mu_j) < 1e-5
    assert abs(dw.item() - dwo) < 1e-5 * abs(dwo)


def _loss_setup(n, kmax, seed_init=0, seed_tgt=1):
    drho, u0 = wl.divergence_free_field(n, kmax, 0.01, seed=seed_init)
    _, u_tgt = wl.divergence_free_field(n, kmax, 0.01, seed=seed_tgt)
    return drho, u0, u_tgt


def _gpu_gradient(n, drho, u0, u_tgt, steps, K, omega):
    need_gpu()
    from paper_1111_2142_amd.autograd import lwacm_run
    u0_t = to_dev(u0).requires_grad_(True)
    om = torch.tensor(omega, dtype=torch.float64, requires_grad=True)
    dr_T, u_T = lwacm_run(to_dev(drho), u0_t, om, steps, 9, K=K)
    loss = ((u_T.double() - to_dev(u_tgt, torch.float64)) ** 2).sum()
    loss.backward()
    return loss.item(), u0_t.grad.double().cpu().numpy(), om.grad.item()


def test_gradient_32_matches_oracle_and_finite_differences():
    """32x32, k <= 2 seeded fields, 200 steps, checkpoint every 10: the GPU
    gradient (FP32 reverse steps) matches the oracle's FP64 reverse sweep
    and FP64 central differences of the oracle within 1e-4."""
    n, kmax, steps, K, omega = 32, 2, 200, 10, 1.6
    banner("gradient 32x32")
    drho, u0, u_tgt = _loss_setup(n, kmax)
    loss, gu, gw = _gpu_gradient(n, drho, u0, u_tgt, steps, K, omega)
    p = oracle.Problem(q=9, nx=n, ny=n, omega=omega)
    u0_32 = u0.astype(np.float32).astype(np.float64)
    gr_o, gu_o, gw_o, _ = oracle.gradient(
        p, 1 + drho, u0_32, steps, lambda r, uu: (np.zeros_like(r), 2 * (uu - u_tgt)), K=K)
    assert rel_l2(gu, gu_o) < 1e-4
    assert abs(gw - gw_o) < 1e-4 * abs(gw_o)

    def L_of(om, uu0):
        _, uT = oracle.run(oracle.Problem(q=9, nx=n, ny=n, omega=om), 1 + drho, uu0, steps)
        return float(((uT - u_tgt) ** 2).sum())

    rng = np.random.Generator(np.random.PCG64(4))
    for _ in range(3):
        du = rng.standard_normal(u0.shape)
        h = 1e-5
        fd = (L_of(omega, u0_32 + h * du) - L_of(omega, u0_32 - h * du)) / (2 * h)
        assert abs((gu * du).sum() - fd) < 1e-4 * abs(fd)
    h = 1e-6
    fdw = (L_of(omega + h, u0_32) - L_of(omega - h, u0_32)) / (2 * h)
    assert abs(gw - fdw) < 1e-4 * abs(fdw)


def test_gradient_512_matches_oracle():
    """The 512x512 differentiable workload (seeded k <= 8 fields, omega 1.6)
    with 200 steps and a checkpoint every 20: GPU vs oracle reverse sweep."""
    c = wl.ADJOINT_512
    steps, K = 200, 20
    banner("gradient 512x512 (200 steps)")
    drho, u0, u_tgt = _loss_setup(c.nx, 8)
    loss, gu, gw = _gpu_gradient(c.nx, drho, u0, u_tgt, steps, K, c.omega)
    p = oracle.Problem(q=9, nx=c.nx, ny=c.ny, omega=c.omega)
    u0_32 = u0.astype(np.float32).astype(np.float64)
    _, gu_o, gw_o, _ = oracle.gradient(
        p, 1 + drho, u0_32, steps, lambda r, uu: (np.zeros_like(r), 2 * (uu - u_tgt)), K=K)
    err = rel_l2(gu, gu_o)
    banner(f"gradient 512: rel-L2 du0 {err:.3e}, domega {gw:.6e} vs {gw_o:.6e}")
    assert err < 1e-4
    assert abs(gw - gw_o) < 1e-4 * abs(gw_o)


def test_gradient_with_zero_steps_is_identity():
    need_gpu()
    from paper_1111_2142_amd.autograd import lwacm_run
    banner("gradient zero steps")
    drho, u0, u_tgt = _loss_setup(16, 2)
    u0_t = to_dev(u0).requires_grad_(True)
    _, u_T = lwacm_run(to_dev(drho), u0_t, 1.6, 0, 9, K=4)
    (u_T * to_dev(u_tgt)).sum().backward()
    assert np.allclose(u0_t.grad.cpu().numpy(), u_tgt.astype(np.float32), rtol=0, atol=1e-7)
