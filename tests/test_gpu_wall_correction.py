"""Interpolated walls (d_q) and link-by-link wall velocities on the D3Q19
tile kernels: the halfway terms of the tile kernel plus the per-step wall
correction (lwacm_walls.hip) against the generic kernel, which applies Eqs.
ACM2.0cc and ACM2.0move link by link, and against the oracle.

- Random walls with moving ids and random q: the rolled kernel (chunks of
  planes, ragged last chunk), the unrolled kernel of thin grids (nz = 3), a
  uniform body force (the forced rolled kernel), FP32 and FP16 storage.
- Random link velocities, with and without q.
- The 192^3 cavity with q = 0.3 on every wall: one step against the generic
  kernel at every node and against the oracle at sampled nodes.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from gpu_helpers import banner, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu

GENERIC = 1


def _library_order(q, a_oracle):
    from paper_1111_2142_amd import lwacm as L
    _, v, _, _ = oracle.lattice_info(q)
    where = {tuple(int(c) for c in v[k]): k for k in range(q)}
    return np.stack([a_oracle[where[vel]] for vel in L.LINK_VELOCITIES[q]])


def _walls(shape, seed, moving=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 3, int(mask.sum())).astype(np.uint8)
    table = np.array([[0, 0, 0], [0, 0, 0], [0.03, -0.01, 0.02] if moving else [0, 0, 0]])
    return mask, table, rng


def _run(L, shape, omega, drho, u, steps, mask, table, qd_lib, uwl_lib, storage=0, variant=0,
         g=None):
    nz, ny, nx = shape
    s = L.Solver(19, nx, ny, nz, omega, storage=storage, mask=to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table], variant=variant, g=g,
                 qd=None if qd_lib is None else to_dev(qd_lib))
    if uwl_lib is not None:
        s.set_wall_velocity_links(to_dev(uwl_lib))
    s.set_state(to_dev(drho), to_dev(u))
    s.step(steps)
    dr, uu = s.moments()
    torch.cuda.synchronize()
    s.close()
    return dr.double().cpu().numpy(), uu.double().cpu().numpy()


@pytest.mark.parametrize("shape,storage,force,links", [
    ((20, 32, 64), 0, False, False), ((20, 32, 64), 1, False, False),
    ((3, 16, 32), 0, False, False), ((12, 32, 32), 0, True, False),
    ((20, 32, 64), 0, False, True), ((12, 32, 32), 1, False, True)])
def test_tile_kernel_with_wall_correction_matches_generic_and_oracle(shape, storage, force,
                                                                      links):
    L = need_gpu()
    banner(f"wall correction shape={shape} storage={storage} force={force} links={links}")
    mask, table, rng = _walls(shape, 51)
    qd = rng.uniform(0.05, 1.0, (19,) + shape).astype(np.float32).astype(np.float64)
    uwl = None
    if links:
        uwl = rng.uniform(-0.04, 0.04, (19, 3) + shape).astype(np.float32).astype(np.float64)
    drho, u = wl.random_state(shape, 3, seed=52, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    g = (2e-4, -1e-4, 5e-5) if force else None
    steps = 6
    qd_l = _library_order(19, qd)
    uwl_l = None if uwl is None else _library_order(19, uwl)
    dr_t, u_t = _run(L, shape, 1.6, drho, u, steps, mask, table, qd_l, uwl_l, storage, g=g)
    dr_g, u_g = _run(L, shape, 1.6, drho, u, steps, mask, table, qd_l, uwl_l, storage,
                     variant=GENERIC, g=g)
    fluid = mask == 0
    e_tg = rel_l2(u_t, u_g, fluid)
    nz, ny, nx = shape
    rho0 = 1.0 + float(drho[fluid].astype(np.float32).mean())
    p = oracle.Problem(q=19, nx=nx, ny=ny, nz=nz, omega=1.6, mask=mask, wall_u=table,
                       rho0=rho0, g=g)
    r_o, u_o = 1.0 + drho, u
    for _ in range(steps):
        r_o, u_o = oracle.step_q(p, r_o, u_o, qd, uwl)
    e_to = rel_l2(u_t, u_o, fluid)
    banner(f"  tile vs generic {e_tg:.3e}, tile vs oracle {e_to:.3e}")
    if storage == 0:
        assert e_tg < 1e-6
        assert e_to < 1e-5
        assert rel_l2(dr_t, r_o - 1.0, fluid) < 1e-4
    else:
        assert e_to < 1e-3


def test_cavity_192_interpolated_one_step():
    """The 192^3 cavity with every wall at q = 0.3 (the bench's workload):
    one tile step against the generic kernel and the FP64 oracle at every
    fluid node (q is the same on every link, so no link reordering)."""
    L = need_gpu()
    banner("cavity 192^3 q = 0.3, one step")
    c4 = wl.CAVITY_192
    n = c4.nx
    mask = wl.cavity_mask(n)
    table = wl.wall_table(c4.lid)
    qd = np.full((19, n, n, n), 0.3, dtype=np.float32)
    drho, u = wl.random_state((n, n, n), 3, seed=54, du=0.02, drho=0.005)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    out = []
    for variant in (0, GENERIC):
        s = L.Solver(19, n, n, n, c4.omega, mask=to_dev(mask, torch.uint8),
                     wall_u=[list(r) for r in table], variant=variant, qd=to_dev(qd))
        s.set_state(to_dev(drho), to_dev(u))
        s.step(1)
        dr, uu = s.moments()
        out.append((dr.cpu().numpy().astype(np.float64), uu.cpu().numpy().astype(np.float64)))
        s.close()
        torch.cuda.synchronize()
    fluid = mask == 0
    e_tg = rel_l2(out[0][1], out[1][1], fluid)
    rho0 = 1.0 + float(drho[fluid].mean())
    p = oracle.Problem(q=19, nx=n, ny=n, nz=n, omega=c4.omega, mask=mask, wall_u=table,
                       rho0=rho0)
    r_o, u_o = oracle.step_q(p, 1.0 + drho, u, qd.astype(np.float64))
    e_to = rel_l2(out[0][1], u_o, fluid)
    banner(f"  tile vs generic rel-L2 u {e_tg:.3e}, tile vs oracle {e_to:.3e}")
    assert e_tg < 1e-6
    assert e_to < 1e-6
    assert rel_l2(out[0][0], r_o - 1.0, fluid) < 1e-4
