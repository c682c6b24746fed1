"""Reverse mode of the temperature step on the GPU
(lwacm_adjoint_thermal_step) against the oracle's thermal_vjp.

- One step: dL/dT_t and the flow cotangent dL/du_t, added to the flow
  sweep's mu in both of its layouts (node-interleaved mu_{t-1}; field-major
  gradient of the initial state), for the flow's lattice and D2Q5 / D3Q7,
  with and without walls held at fixed temperatures and adiabatic ones.
- Several steps chained with the flow's reverse steps (lwacm_adjoint_seed,
  lwacm_adjoint_step): the gradient of L = sum a T_N + sum b . u_N with
  respect to the initial T, rho - 1 and u against the oracle's chain of
  vjp and thermal_vjp over the oracle's own forward run.
- lwacm_run_thermal (torch.autograd over flow and temperature, checkpoints
  and ragged segments): gradients of T0, rho0 - 1, u0 and omega against the
  oracle's chain.
- FP16 flow states: the step reads u and rho through the FP16 load scales.
- Argument checks.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from gpu_helpers import banner, fluid_of, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu

WALL_T = [np.nan, 0.2, np.nan, 0.9]  # ids 1 and 3 fixed, id 2 adiabatic
OMEGA, OMEGA_T = 1.6, 1.3


def _walls(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 4, int(mask.sum())).astype(np.uint8)
    return mask


def _setup(L, q, qt, masked, shape, seed):
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=seed, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    T = rng.uniform(0.2, 1.0, shape).astype(np.float32).astype(np.float64)
    mask = _walls(shape, seed + 2) if masked else None
    if mask is not None:
        u[:, mask != 0] = 0.0
    table = np.zeros((4, 3))
    s = L.Solver(q, nx, ny, nz, OMEGA, mask=None if mask is None else to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table])
    s.set_state(to_dev(drho), to_dev(u))
    s.set_thermal(OMEGA_T, to_dev(T), wall_T=WALL_T, q_t=qt or 0)
    p = oracle.Problem(q, nx, ny, nz, omega=OMEGA, mask=mask, wall_u=table)
    return s, p, d, drho, u, T, mask


CASES = [(9, None, False, (1, 24, 40)), (9, 5, True, (1, 24, 40)), (9, None, True, (1, 24, 40)),
         (19, None, False, (8, 16, 32)), (19, 7, True, (8, 16, 32)), (19, None, True, (6, 10, 12))]


@pytest.mark.parametrize("q,qt,masked,shape", CASES)
def test_one_reverse_temperature_step_matches_oracle(q, qt, masked, shape):
    L = need_gpu()
    banner(f"thermal reverse step q={q} qt={qt} masked={masked} shape={shape}")
    s, p, d, drho, u, T, mask = _setup(L, q, qt, masked, shape, 91)
    nz, ny, nx = shape
    n = nx * ny * nz
    st = s.save_state()
    Tt = s.temperature()
    rng = np.random.Generator(np.random.PCG64(94))
    lam = rng.standard_normal(shape).astype(np.float32)
    lam_in = to_dev(lam)
    lam_out = torch.empty_like(lam_in)
    # field-major: the u fields gain dL/du
    mu_f = torch.zeros((d + 1,) + shape, dtype=torch.float32, device="cuda")
    L.lwacm_adjoint_thermal_step(s.ctx, st, Tt, lam_in, lam_out, mu_f, True)
    # node-interleaved mu_{t-1}: a random sweep value plus the folded cotangent
    mu0 = rng.standard_normal(n * (d + 1)).astype(np.float32)
    mu_i = to_dev(mu0)
    lam_out2 = torch.empty_like(lam_in)
    L.lwacm_adjoint_thermal_step(s.ctx, st, Tt, lam_in, lam_out2, mu_i, False)
    torch.cuda.synchronize()
    lt, lu = oracle.thermal_vjp(p, T, u, lam.astype(np.float64), OMEGA_T, wall_T=WALL_T, qt=qt)
    got_T = lam_out.double().cpu().numpy()
    got_u = mu_f.double().cpu().numpy()
    e_T, e_u = rel_l2(got_T, lt), rel_l2(got_u[1:], lu)
    banner(f"thermal reverse step: rel-L2 dL/dT {e_T:.3e}, dL/du {e_u:.3e}")
    assert e_T < 1e-6 and e_u < 1e-5
    assert not got_u[0].any()
    assert torch.equal(lam_out, lam_out2)
    inv = 1.0 / (1.0 + drho)
    exp_r = -(lu * u).sum(0) * inv
    exp_j = lu * inv
    got_i = mu_i.double().cpu().numpy().reshape(n, d + 1).T.reshape((d + 1,) + shape)
    base = mu0.astype(np.float64).reshape(n, d + 1).T.reshape((d + 1,) + shape)
    assert rel_l2(got_i[0] - base[0], exp_r) < 1e-5
    assert rel_l2(got_i[1:] - base[1:], exp_j) < 1e-5
    if mask is not None:
        sol = mask != 0
        assert np.array_equal(got_T[sol], lam.astype(np.float64)[sol])
        assert not got_u[1:, sol].any()
        assert np.array_equal(got_i[:, sol], base[:, sol])
    s.close()


@pytest.mark.parametrize("q,qt,masked", [(9, None, True), (19, 7, False), (19, None, True)])
def test_reverse_temperature_step_on_fp16_states(q, qt, masked):
    """FP16 flow storage: the reverse temperature step reads u and rho from
    the FP16 state; against thermal_vjp at the dequantized state."""
    L = need_gpu()
    banner(f"thermal reverse step on an FP16 state q={q} qt={qt} masked={masked}")
    shape = (1, 24, 40) if q == 9 else (6, 10, 12)
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    n = nx * ny * nz
    drho, u = wl.random_state(shape, d, seed=121, du=0.03, drho=0.01)
    rng = np.random.Generator(np.random.PCG64(122))
    T = rng.uniform(0.2, 1.0, shape).astype(np.float32)
    mask = _walls(shape, 123) if masked else None
    s = L.Solver(q, nx, ny, nz, OMEGA, storage=1,
                 mask=None if mask is None else to_dev(mask, torch.uint8),
                 wall_u=[[0.0, 0.0, 0.0]] * 4)
    s.set_state(to_dev(drho), to_dev(u))
    s.set_thermal(OMEGA_T, to_dev(T), wall_T=WALL_T, q_t=qt or 0)
    st = s.save_state()
    dr_t, u_t = (x.double().cpu().numpy() for x in s.moments())
    lam = rng.standard_normal(shape).astype(np.float32)
    lam_out = torch.empty(shape, dtype=torch.float32, device="cuda")
    mu_f = torch.zeros((d + 1,) + shape, dtype=torch.float32, device="cuda")
    L.lwacm_adjoint_thermal_step(s.ctx, st, to_dev(T), to_dev(lam), lam_out, mu_f, True)
    mu_i = torch.zeros(n * (d + 1), dtype=torch.float32, device="cuda")
    L.lwacm_adjoint_thermal_step(s.ctx, st, to_dev(T), to_dev(lam), torch.empty_like(lam_out),
                                 mu_i, False)
    torch.cuda.synchronize()
    s.close()
    p = oracle.Problem(q, nx, ny, nz, omega=OMEGA, mask=mask, wall_u=np.zeros((4, 3)))
    lt, lu = oracle.thermal_vjp(p, T.astype(np.float64), u_t, lam.astype(np.float64), OMEGA_T,
                                wall_T=WALL_T, qt=qt)
    e_T = rel_l2(lam_out.double().cpu().numpy(), lt)
    e_u = rel_l2(mu_f.double().cpu().numpy()[1:], lu)
    got_i = mu_i.double().cpu().numpy().reshape(n, d + 1).T.reshape((d + 1,) + shape)
    inv = 1.0 / (1.0 + dr_t)
    e_r = rel_l2(got_i[0], -(lu * u_t).sum(0) * inv)
    banner(f"thermal reverse step, FP16 state: rel-L2 dL/dT {e_T:.3e}, dL/du {e_u:.3e}, "
           f"mu_R {e_r:.3e}")
    assert e_T < 1e-6 and e_u < 1e-5 and e_r < 1e-5


@pytest.mark.parametrize("q,qt,masked,shape", [(9, None, True, (1, 24, 40)), (9, 5, False, (1, 24, 40)),
                                                (19, None, False, (8, 16, 32)),
                                                (19, 7, True, (8, 16, 32))])
def test_chained_reverse_sweep_matches_oracle(q, qt, masked, shape):
    """N = 4 forward steps of flow and temperature, then the reverse sweep:
    seed, and for t = N-1 .. 0 the flow's reverse step followed by the
    temperature's.  L = sum a T_N + sum b . u_N."""
    L = need_gpu()
    banner(f"thermal reverse sweep q={q} qt={qt} masked={masked} shape={shape}")
    N = 4
    s, p, d, drho, u, T, mask = _setup(L, q, qt, masked, shape, 101)
    states, temps = [], []
    for _ in range(N):
        states.append(s.save_state())
        temps.append(s.temperature())
        s.step(1)
    stN = s.save_state()
    rng = np.random.Generator(np.random.PCG64(104))
    a = rng.standard_normal(shape)
    b = rng.standard_normal((d,) + shape)
    lam_flow = np.concatenate([np.zeros((1,) + shape), b]).astype(np.float32)
    mu = torch.empty((d + 1,) + shape, dtype=torch.float32, device="cuda")
    L.lwacm_adjoint_seed(s.ctx, stN, to_dev(lam_flow), mu)
    lamT = to_dev(a)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    for t in range(N - 1, -1, -1):
        mu_next = torch.empty_like(mu)
        lamT_next = torch.empty_like(lamT)
        L.lwacm_adjoint_step(s.ctx, states[t], mu, mu_next, dw, t == 0)
        L.lwacm_adjoint_thermal_step(s.ctx, states[t], temps[t], lamT, lamT_next, mu_next, t == 0)
        mu, lamT = mu_next, lamT_next
    torch.cuda.synchronize()
    g = mu.double().cpu().numpy()
    gT = lamT.double().cpu().numpy()
    s.close()
    # the oracle: forward run, then its chain of reverse steps
    rhos, us, Ts = [1.0 + drho], [u], [T]
    for _ in range(N):
        Ts.append(oracle.thermal_step(p, Ts[-1], us[-1], OMEGA_T, wall_T=WALL_T, qt=qt))
        r1, u1 = oracle.step(p, rhos[-1], us[-1])
        rhos.append(r1)
        us.append(u1)
    lr, lu, lt = np.zeros(shape), b.copy(), a.copy()
    for t in range(N - 1, -1, -1):
        lr, lu_f, _ = oracle.vjp(p, rhos[t], us[t], lr, lu)
        lt, gu = oracle.thermal_vjp(p, Ts[t], us[t], lt, OMEGA_T, wall_T=WALL_T, qt=qt)
        lu = lu_f + gu
    fl = fluid_of(mask, shape)
    e_T = rel_l2(gT, lt)
    e_r = rel_l2(g[0][fl], lr[fl])
    e_u = rel_l2(g[1:][:, fl], lu[:, fl])
    banner(f"thermal reverse sweep: rel-L2 dL/dT0 {e_T:.3e}, dL/drho0 {e_r:.3e}, dL/du0 {e_u:.3e}")
    assert e_T < 1e-5 and e_r < 1e-5 and e_u < 1e-5


def test_reverse_temperature_step_rejects_bad_arguments():
    L = need_gpu()
    s = L.Solver(9, 32, 16, 1, 1.6)
    st = s.save_state()
    lam = torch.zeros((1, 16, 32), device="cuda")
    mu = torch.zeros((3, 1, 16, 32), device="cuda")
    with pytest.raises(L.LWACMError):  # temperature off
        L.lwacm_adjoint_thermal_step(s.ctx, st, lam, lam, torch.empty_like(lam), mu, True)
    s.set_thermal(1.3, torch.ones((1, 16, 32), device="cuda"))
    with pytest.raises(L.LWACMError):  # lam buffers alias
        L.lwacm_adjoint_thermal_step(s.ctx, st, s.temperature(), lam, lam, mu, True)
    s.close()


@pytest.mark.parametrize("q,qt,masked,shape", [(9, None, True, (1, 24, 40)),
                                                (19, 7, False, (8, 16, 32))])
def test_differentiable_thermal_run_matches_oracle(q, qt, masked, shape):
    """lwacm_run_thermal through torch.autograd: 9 steps with checkpoints every
    4 (segments of 4, 4 and 1), L = sum a T_N + sum b . u_N + sum c (rho_N - 1);
    gradients with respect to T0, rho0 - 1, u0 and omega against the oracle's
    chain of vjp and thermal_vjp."""
    L = need_gpu()
    from paper_1111_2142_amd.autograd import lwacm_run_thermal
    banner(f"thermal autograd q={q} qt={qt} masked={masked} shape={shape}")
    N, K = 9, 4
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=111, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(112))
    T = rng.uniform(0.2, 1.0, shape).astype(np.float32).astype(np.float64)
    mask = _walls(shape, 113) if masked else None
    if mask is not None:
        u[:, mask != 0] = 0.0
    a = rng.standard_normal(shape)
    b = rng.standard_normal((d,) + shape)
    c = rng.standard_normal(shape)
    table = [[0.0, 0.0, 0.0]] * 4
    x_r = to_dev(drho).requires_grad_(True)
    x_u = to_dev(u).requires_grad_(True)
    x_T = to_dev(T).requires_grad_(True)
    om = torch.tensor(OMEGA, dtype=torch.float64, requires_grad=True)
    r_N, u_N, T_N = lwacm_run_thermal(x_r, x_u, x_T, om, OMEGA_T, N, q, K=K,
                                      mask=None if mask is None else to_dev(mask, torch.uint8),
                                      wall_u=table, wall_T=WALL_T, q_t=qt or 0)
    loss = (to_dev(a) * T_N).sum() + (to_dev(b) * u_N).sum() + (to_dev(c) * r_N).sum()
    loss.backward()
    p = oracle.Problem(q, nx, ny, nz, omega=OMEGA, mask=mask, wall_u=np.zeros((4, 3)))
    rhos, us, Ts = [1.0 + drho], [u], [T]
    for _ in range(N):
        Ts.append(oracle.thermal_step(p, Ts[-1], us[-1], OMEGA_T, wall_T=WALL_T, qt=qt))
        r1, u1 = oracle.step(p, rhos[-1], us[-1])
        rhos.append(r1)
        us.append(u1)
    lr, lu, lt, dw = c.copy(), b.copy(), a.copy(), 0.0
    for t in range(N - 1, -1, -1):
        lr, lu_f, dwt = oracle.vjp(p, rhos[t], us[t], lr, lu)
        lt, gu = oracle.thermal_vjp(p, Ts[t], us[t], lt, OMEGA_T, wall_T=WALL_T, qt=qt)
        lu = lu_f + gu
        dw += dwt
    fl = fluid_of(mask, shape)
    e_T = rel_l2(x_T.grad.double().cpu().numpy(), lt)
    e_r = rel_l2(x_r.grad.double().cpu().numpy()[fl], lr[fl])
    e_u = rel_l2(x_u.grad.double().cpu().numpy()[:, fl], lu[:, fl])
    e_w = abs(om.grad.item() - dw) / abs(dw)
    banner(f"thermal autograd: rel-L2 dL/dT0 {e_T:.3e}, dL/drho0 {e_r:.3e}, dL/du0 {e_u:.3e}, "
           f"dL/domega {e_w:.3e}")
    assert e_T < 1e-5 and e_r < 1e-5 and e_u < 1e-5 and e_w < 1e-5
