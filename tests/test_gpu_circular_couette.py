"""Wall velocities given link by link (lwacm_set_wall_velocity_links) and the
circular Couette flow (Section "Circular Couette flow", Table
"table:circouette") on the GPU, against the oracle.

- Random walls, link-wall distances and link velocities: D2Q9 and D3Q19,
  FP32 and FP16 storage, 5 steps, against oracle.step_q with the same inputs.
- Link velocities equal to the per-id table: the table's step to FP32
  rounding (the product (2/omega - 1) 6 rho0 u_w is formed in FP32 here and in
  FP64 for the table).
- Circular Couette at eps = 1/20 and 1/40 to t = 20 (8000 and 32000 steps):
  fields, L1 errors and torque against the stored FP64 oracle runs.
- The paper's table: eps = 1/20 ... 1/160 to t = 20 on the GPU, second-order
  convergence of u_theta and p, the torque to 4 pi C nu r_i, and the errors
  at 1/80 equal to the stored oracle's.
- Scope: the reverse steps and a separate omega_p decline link velocities.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from circular_couette import exact, l1_errors
from gpu_helpers import banner, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _library_order(q, a_oracle):
    """Per-link fields (first axis: link) from the oracle's link order to the
    library's, matching links by velocity."""
    from paper_1111_2142_amd import lwacm as L
    _, v, _, _ = oracle.lattice_info(q)
    where = {tuple(int(c) for c in v[k]): k for k in range(q)}
    return np.stack([a_oracle[where[vel]] for vel in L.LINK_VELOCITIES[q]])


def _gpu(L, q, shape, omega, drho, u, steps, mask, table, qd, uwl, storage=0):
    nz, ny, nx = shape
    s = L.Solver(q, nx, ny, nz, omega, storage=storage, mask=to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table],
                 qd=None if qd is None else to_dev(_library_order(q, qd)))
    if uwl is not None:
        s.set_wall_velocity_links(to_dev(_library_order(q, uwl)))
    s.set_state(to_dev(drho), to_dev(u))
    s.step(steps)
    dr, uu = s.moments()
    torch.cuda.synchronize()
    return dr.double().cpu().numpy(), uu.double().cpu().numpy(), s


@pytest.mark.parametrize("q,shape,storage,interp", [
    (9, (1, 40, 48), 0, True), (9, (1, 40, 48), 0, False), (19, (12, 32, 32), 0, True),
    (19, (12, 32, 32), 1, True)])
def test_link_velocities_match_oracle(q, shape, storage, interp):
    L = need_gpu()
    banner(f"link velocities q={q} storage={storage} interpolated={interp}")
    d = 2 if q == 9 else 3
    rng = np.random.Generator(np.random.PCG64(77))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 3, int(mask.sum())).astype(np.uint8)
    table = np.zeros((3, 3))
    qd = rng.uniform(0.05, 1.0, (q,) + shape) if interp else None
    uwl = rng.uniform(-0.04, 0.04, (q, d) + shape)
    drho, u = wl.random_state(shape, d, seed=78, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    uwl = uwl.astype(np.float32).astype(np.float64)
    if qd is not None:
        qd = qd.astype(np.float32).astype(np.float64)
    steps = 5
    dr, uu, s = _gpu(L, q, shape, 1.6, drho, u, steps, mask, table, qd, uwl, storage)
    s.close()
    nz, ny, nx = shape
    fluid = mask == 0
    # rho0 of the moving-wall term: the mean fluid density of the initial state
    rho0 = 1.0 + float(drho[fluid].mean())
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=1.6, mask=mask, wall_u=table, rho0=rho0)
    r_o, u_o = 1 + drho, u
    for _ in range(steps):
        r_o, u_o = oracle.step_q(p, r_o, u_o, qd, uwl)
    bar = 1e-5 if storage == 0 else 1e-3
    e_u = rel_l2(uu, u_o, fluid)
    banner(f"link velocities: rel-L2 u {e_u:.3e}")
    assert e_u < bar
    assert rel_l2(dr, r_o - 1, fluid) < (1e-4 if storage == 0 else 2e-2)


def test_link_velocities_equal_to_the_table_give_the_table_step():
    L = need_gpu()
    banner("link velocities = table")
    q, shape, d = 19, (12, 32, 32), 3
    rng = np.random.Generator(np.random.PCG64(79))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 3, int(mask.sum())).astype(np.uint8)
    table = np.array([[0, 0, 0], [0, 0, 0], [0.03, -0.01, 0.02]], dtype=np.float32)
    _, v, _, _ = oracle.lattice_info(q)
    nz, ny, nx = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    uwl = np.zeros((q, d) + shape)
    for j in range(q):
        tgt = mask[(zz + v[j][2]) % nz, (yy + v[j][1]) % ny, (xx + v[j][0]) % nx]
        uwl[j] = np.moveaxis(table[tgt].astype(np.float64), -1, 0)
    drho, u = wl.random_state(shape, d, seed=80, du=0.03, drho=0.01)
    a = _gpu(L, q, shape, 1.6, drho, u, 10, mask, table, None, None)
    b = _gpu(L, q, shape, 1.6, drho, u, 10, mask, table, None, uwl)
    a[2].close()
    b[2].close()
    assert np.abs(a[1] - b[1]).max() < 1e-8 and np.abs(a[0] - b[0]).max() < 1e-8


def _circular_gpu(L, eps, t_end=20.0, storage=0):
    cc = wl.CircularCouette(eps)
    qd, uwl = cc.links(L.LINK_VELOCITIES[9])
    s = L.Solver(9, cc.n, cc.n, 1, cc.omega, storage=storage, mask=to_dev(cc.mask, torch.uint8),
                 wall_u=[[0.0, 0.0, 0.0]] * 3, qd=to_dev(qd))
    s.set_wall_velocity_links(to_dev(uwl))
    s.set_state(torch.zeros((1, cc.n, cc.n), device="cuda"),
                torch.zeros((2, 1, cc.n, cc.n), device="cuda"))
    s.step(cc.steps_to(t_end))
    dr, uu = s.moments()
    _, T = s.wall_force(1, cc.center)
    torch.cuda.synchronize()
    s.close()
    return cc, 1.0 + dr.double().cpu().numpy(), uu.double().cpu().numpy(), T[2]


def test_circular_couette_matches_the_oracle(golden_dir):
    L = need_gpu()
    ref = np.load(os.path.join(golden_dir, "circular_couette_oracle.npz"))
    for k in (20, 40):
        banner(f"circular Couette eps = 1/{k}, t = 20")
        cc, rho, u, tz = _circular_gpu(L, 1.0 / k)
        e = l1_errors(cc, rho, u, tz)
        fluid = cc.fluid[None]
        e_u = rel_l2(u, ref[f"u_{k}"], fluid)
        e_r = rel_l2(rho - 1, ref[f"rho_{k}"] - 1, fluid)
        banner(f"  rel-L2 u {e_u:.3e}, drho {e_r:.3e}; L1 {e}, oracle {ref[f'errors_{k}']}; "
               f"T_z {tz:.9f} vs {float(ref[f'torque_{k}']):.9f}")
        assert e_u < 1e-5
        assert e_r < 1e-3
        assert abs(tz - float(ref[f"torque_{k}"])) < 1e-5 * abs(tz)
        assert np.allclose(e, ref[f"errors_{k}"], rtol=2e-2, atol=0)


def test_circular_couette_table(golden_dir):
    """The paper's table on the GPU: eps = 1/20 ... 1/160 to t = 20."""
    L = need_gpu()
    ref = np.load(os.path.join(golden_dir, "circular_couette_oracle.npz"))
    paper = json.load(open(os.path.join(golden_dir, "circular_couette_table.json")))
    errs = {}
    for k in (20, 40, 80, 160):
        cc, rho, u, tz = _circular_gpu(L, 1.0 / k)
        errs[k] = l1_errors(cc, rho, u, tz)
        banner(f"circular Couette eps = 1/{k} ({cc.n}^2, {cc.steps_to(20.0)} steps): "
               f"L1 u_theta {errs[k][0]:.5e}, p {errs[k][1]:.5e}, |T| {errs[k][2]:.5e} "
               f"(T_z {tz:.7f}, exact {exact(cc)[2]:.7f})")
    for a, b in ((20, 40), (40, 80), (80, 160)):
        for i in range(2):
            assert errs[a][i] / errs[b][i] > 2.8, (a, b, i, errs)
        assert errs[a][2] > errs[b][2]
    assert np.allclose(errs[80], ref["errors_80"], rtol=2e-2, atol=0)
    for col, k in enumerate((20, 40, 80, 160)):
        for i, name in enumerate(("u_theta", "p", "torque")):
            assert 0.1 < errs[k][i] / paper[name][col] < 10, (k, name)


def test_scope_of_link_velocities():
    L = need_gpu()
    banner("link velocities scope")
    shape = (1, 16, 16)
    mask = np.zeros(shape, dtype=np.uint8)
    mask[0, 0, :] = 1
    s = L.Solver(9, 16, 16, 1, 1.6, mask=to_dev(mask, torch.uint8))
    uw = torch.zeros((9, 2, 1, 16, 16), device="cuda")
    s.set_wall_velocity_links(uw)
    st = s.save_state()
    mu = torch.zeros((3, 1, 16, 16), device="cuda")
    mo = torch.zeros_like(mu)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LWACMError) as e:
        L.lwacm_adjoint_step(s.ctx, st, mu, mo, dw, False)
    assert e.value.code == L.LWACM_EUNSUPPORTED
    with pytest.raises(L.LWACMError) as e:
        L.lwacm_set_omega_p(s.ctx, 1.3)
    assert e.value.code == L.LWACM_EUNSUPPORTED
    s.set_wall_velocity_links(None)
    L.lwacm_set_omega_p(s.ctx, 1.3)
    with pytest.raises(L.LWACMError) as e:
        s.set_wall_velocity_links(uw)
    assert e.value.code == L.LWACM_EUNSUPPORTED
    s.close()
    s = L.Solver(9, 16, 16, 1, 1.6)  # no mask: nothing to apply the velocities to
    with pytest.raises(L.LWACMError) as e:
        s.set_wall_velocity_links(uw)
    assert e.value.code == L.LWACM_EINVAL
    s.close()
