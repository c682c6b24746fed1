"""The semi-implicit pressure update (lwacm_set_semi_implicit, Eq.
FDcompact_si) on the GPU against the oracle's step_si.

- Random states with walls (a moving one) and a uniform body force, D2Q9 and
  D3Q19, 6 steps: u and rho - 1 against the oracle.
- The generalized Taylor-Green vortex at eps = pi/32 to t = 60 with a new
  acceleration field every step: fields and L1 errors against the oracle.
- Mass is conserved on a periodic grid; scope.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from gpu_helpers import banner, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("q,shape", [(9, (1, 40, 48)), (19, (12, 32, 32))])
def test_semi_implicit_steps_match_oracle(q, shape):
    L = need_gpu()
    banner(f"semi-implicit q={q}")
    d = 2 if q == 9 else 3
    nz, ny, nx = shape
    mask = np.zeros(shape, dtype=np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 2
    table = np.array([[0, 0, 0], [0, 0, 0], [0.03, 0.0, 0.01 if d == 3 else 0.0]])
    g = (2e-4, -1e-4, 5e-5)[:d]
    drho, u = wl.random_state(shape, d, seed=61, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    u[:, mask != 0] = 0.0
    s = L.Solver(q, nx, ny, nz, 1.6, mask=to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table], g=g)
    L.lwacm_set_semi_implicit(s.ctx, True)
    s.set_state(to_dev(drho), to_dev(u))
    steps = 6
    s.step(steps)
    dr, uu = s.moments()
    torch.cuda.synchronize()
    s.close()
    fluid = mask == 0
    rho0 = 1.0 + float(drho[fluid].astype(np.float32).mean())
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=1.6, mask=mask, wall_u=table, g=g,
                       rho0=rho0)
    r_o, u_o = 1.0 + drho, u
    for _ in range(steps):
        r_o, u_o = oracle.step_si(p, r_o, u_o)
    e_u = rel_l2(uu.cpu().numpy().astype(np.float64), u_o, fluid)
    e_r = rel_l2(dr.cpu().numpy().astype(np.float64), r_o - 1.0, fluid)
    banner(f"  rel-L2 u {e_u:.3e}, drho {e_r:.3e}")
    assert e_u < 1e-5 and e_r < 1e-4


def test_semi_implicit_generalized_taylor_green_matches_oracle():
    L = need_gpu()
    banner("semi-implicit generalized Taylor-Green pi/32 to t = 60")
    c = wl.ForcedTaylorGreen(32)
    drho, u = c.initial_state()
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    s = L.Solver(9, c.n, c.n, 1, c.omega)
    L.lwacm_set_semi_implicit(s.ctx, True)
    s.set_state(to_dev(drho), to_dev(u))
    steps = c.steps_to(60.0)
    for k in range(steps):
        s.set_force_field(to_dev(c.acceleration(k)))
        s.step(1)
    dr, uu = s.moments()
    m, _ = s.diagnostics()
    torch.cuda.synchronize()
    s.close()
    p = oracle.Problem(9, c.n, c.n, 1, omega=c.omega)
    r_o, u_o = 1.0 + drho, u
    for k in range(steps):
        r_o, u_o = oracle.step_si(p, r_o, u_o, c.acceleration(k))
    g_dr = dr.cpu().numpy().astype(np.float64)
    g_u = uu.cpu().numpy().astype(np.float64)
    e_u = rel_l2(g_u, u_o)
    e_gpu = c.l1_errors(steps, g_dr, g_u)
    e_or = c.l1_errors(steps, r_o - 1.0, u_o)
    banner(f"  rel-L2 u {e_u:.3e}; L1 GPU {e_gpu}, oracle {e_or}; mass {m:.9f}")
    assert e_u < 1e-5
    assert np.allclose(e_gpu, e_or, rtol=1e-3, atol=0)
    assert abs(m - float((1.0 + drho).astype(np.float32).sum())) < 1e-6 * c.n ** 2


def test_semi_implicit_scope():
    L = need_gpu()
    banner("semi-implicit scope")
    s = L.Solver(19, 32, 16, 8, 1.6, storage=L.LWACM_FP16_DEV)
    with pytest.raises(L.LWACMError) as e:
        L.lwacm_set_semi_implicit(s.ctx, True)
    assert e.value.code == L.LWACM_EUNSUPPORTED
    s.close()
    s = L.Solver(19, 32, 16, 8, 1.6)
    L.lwacm_set_semi_implicit(s.ctx, True)
    for v in (2, 3):
        with pytest.raises(L.LWACMError) as e:
            L.lwacm_set_variant(s.ctx, v)
        assert e.value.code == L.LWACM_EUNSUPPORTED
    with pytest.raises(L.LWACMError) as e:
        L.lwacm_set_omega_p(s.ctx, 1.2)
    assert e.value.code == L.LWACM_EUNSUPPORTED
    st = s.save_state()
    mu = torch.zeros((4, 8, 16, 32), device="cuda")
    mo = torch.zeros_like(mu)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LWACMError) as e:
        L.lwacm_adjoint_step(s.ctx, st, mu, mo, dw, False)
    assert e.value.code == L.LWACM_EUNSUPPORTED
    L.lwacm_set_semi_implicit(s.ctx, False)
    L.lwacm_set_variant(s.ctx, 3)
    s.close()
