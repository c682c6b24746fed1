"""Node-by-node body acceleration (lwacm_set_force_field; Eq. force with the
space- and time-dependent g of the paper's generalized Taylor-Green vortex)
against the oracle's field-forced step.

- A uniform field gives the uniform-g step of lwacm_init bit for bit, with
  and without walls.
- A random field on D3Q19 with walls, FP32 and FP16 storage, to the parity
  bars; a random field on D2Q9.
- The generalized Taylor-Green vortex at eps = pi/32 (64^2, 6225 steps to
  t = 60, a new field before every step): the state against the oracle's,
  and the L1 errors against the analytic solution equal to the oracle's (and
  so near the paper's printed table).
- D3Q19 (nz >= 8) runs the single-step tile kernel, which loads the field
  with the state; against the generic kernel to FP32 rounding.
- Scope: a field declines the two-step kernel and the reverse steps;
  clearing it gives back the unforced step bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from gpu_helpers import banner, fluid_of, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu

MARCH = 2


def _solver(L, q, shape, omega, storage=0, mask=None, g=None):
    nz, ny, nx = shape
    return L.Solver(q, nx, ny, nz, omega, storage=storage,
                    mask=None if mask is None else to_dev(mask, torch.uint8), g=g)


def _run(s, drho, u, steps):
    s.set_state(to_dev(drho), to_dev(u))
    s.step(steps)
    dr, uu = s.moments()
    return dr.double().cpu().numpy(), uu.double().cpu().numpy()


@pytest.mark.parametrize("q,shape", [(9, (1, 48, 64)), (19, (12, 32, 32))])
def test_uniform_field_is_the_uniform_acceleration_step(q, shape):
    L = need_gpu()
    banner(f"force field uniform q={q}")
    d = 2 if q == 9 else 3
    g = (2e-5, -1e-5, 5e-6)[:d]
    drho, u = wl.random_state(shape, d, seed=31, du=0.03, drho=0.01)
    mask = np.zeros(shape, dtype=np.uint8)
    mask[:, 0] = 1
    for m in (None, mask):
        a = _solver(L, q, shape, 1.6, mask=m, g=g)
        ra = _run(a, drho, u, 5)
        a.close()
        b = _solver(L, q, shape, 1.6, mask=m)
        b.set_force_field(torch.tensor(g, dtype=torch.float32, device="cuda").reshape(d, 1, 1, 1)
                          .expand((d,) + shape).contiguous())
        rb = _run(b, drho, u, 5)
        b.close()
        assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1])


@pytest.mark.parametrize("q,storage", [(9, 0), (19, 0), (19, 1)])
def test_random_field_matches_oracle(q, storage):
    L = need_gpu()
    banner(f"force field random q={q} storage={storage}")
    shape = (1, 48, 64) if q == 9 else (12, 32, 32)
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=32, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(33))
    gf = (1e-4 * rng.standard_normal((d,) + shape)).astype(np.float32).astype(np.float64)
    mask = None
    if q == 19:
        mask = (rng.random(shape) < 0.08).astype(np.uint8)
    s = _solver(L, q, shape, 1.5, storage=storage, mask=mask)
    s.set_force_field(to_dev(gf))
    dr, uu = _run(s, drho, u, 6)
    s.close()
    p = oracle.Problem(q, nx, ny, nz, omega=1.5, mask=mask)
    r, ru = 1.0 + drho, u
    for _ in range(6):
        r, ru = oracle.step_field(p, r, ru, gf)
    fl = fluid_of(mask, shape)
    err_u, err_r = rel_l2(uu[:, fl], ru[:, fl]), rel_l2(dr[fl], (r - 1.0)[fl])
    banner(f"force field: rel-L2 u {err_u:.3e}, drho {err_r:.3e}")
    assert err_u < (1e-5 if storage == 0 else 1e-3)
    assert err_r < (1e-4 if storage == 0 else 2e-2)


@pytest.mark.parametrize("masked", [False, True])
def test_tile_kernel_field_matches_generic(masked):
    L = need_gpu()
    banner(f"force field tile vs generic masked={masked}")
    shape = (40, 32, 64)
    drho, u = wl.random_state(shape, 3, seed=35, du=0.03, drho=0.01)
    rng = np.random.Generator(np.random.PCG64(36))
    gf = to_dev(1e-4 * rng.standard_normal((3,) + shape))
    mask = None
    if masked:
        mask = (rng.random(shape) < 0.05).astype(np.uint8)
    out = []
    for v in (MARCH, 1):
        s = _solver(L, 19, shape, 1.6, mask=mask)
        L.lwacm_set_variant(s.ctx, v)
        s.set_force_field(gf)
        out.append(_run(s, drho, u, 8))
        s.close()
    fl = fluid_of(mask, shape)
    err = rel_l2(out[0][1][:, fl], out[1][1][:, fl])
    banner(f"force field tile vs generic: rel-L2 u {err:.3e}")
    assert err < 1e-6


def test_forced_taylor_green_matches_oracle_to_t60():
    L = need_gpu()
    c = wl.ForcedTaylorGreen(32)
    steps = c.steps_to(60.0)
    banner(f"forced Taylor-Green eps=pi/32 n={c.n} steps={steps}")
    drho, u = c.initial_state()
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    s = L.Solver(9, c.n, c.n, 1, c.omega)
    s.set_state(to_dev(drho), to_dev(u))
    g = torch.empty((2, 1, c.n, c.n), dtype=torch.float32, device="cuda")
    s.set_force_field(g)
    for k in range(steps):
        g.copy_(torch.from_numpy(c.acceleration(k).astype(np.float32)))
        s.step(1)
    dr, uu = s.moments()
    dr, uu = dr.double().cpu().numpy(), uu.double().cpu().numpy()
    s.close()
    p = oracle.Problem(9, c.n, c.n, 1, omega=c.omega)
    r, ru = 1.0 + drho, u
    for k in range(steps):
        r, ru = oracle.step_field(p, r, ru, c.acceleration(k).astype(np.float32).astype(np.float64))
    e_gpu, e_ora = c.l1_errors(steps, dr, uu), c.l1_errors(steps, r - 1.0, ru)
    err_u = rel_l2(uu, ru)
    banner(f"forced Taylor-Green: rel-L2 u {err_u:.3e}; L1 (u, v, p) GPU "
           f"{e_gpu[0]:.5e} {e_gpu[1]:.5e} {e_gpu[2]:.5e}, oracle {e_ora[0]:.5e} {e_ora[1]:.5e} "
           f"{e_ora[2]:.5e}")
    assert err_u < 1e-5
    for a, b in zip(e_gpu, e_ora):
        assert abs(a - b) <= 1e-3 * b


def test_force_field_scope():
    L = need_gpu()
    banner("force field scope")
    shape = (16, 32, 64)
    drho, u = wl.random_state(shape, 3, seed=34, du=0.02, drho=0.01)
    a = _solver(L, 19, shape, 1.7)
    ref = _run(a, drho, u, 4)
    a.close()
    s = _solver(L, 19, shape, 1.7)
    s.set_force_field(torch.zeros((3,) + shape, device="cuda"))
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_set_variant(s.ctx, 3)  # the two-step kernel
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    L.lwacm_set_variant(s.ctx, MARCH)  # the single-step tile kernel takes it
    s.set_state(to_dev(drho), to_dev(u))
    st = s.save_state()
    mu = torch.zeros(shape + (4,), device="cuda")
    out = torch.zeros_like(mu)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_adjoint_step(s.ctx, st, mu, out, dw, False)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    assert not L.lwacm_adjoint_step2(s.ctx, st, st, mu, out, dw, False)
    s.set_force_field(None)
    L.lwacm_set_variant(s.ctx, 0)
    back = _run(s, drho, u, 4)
    s.close()
    assert np.array_equal(ref[0], back[0]) and np.array_equal(ref[1], back[1])
