"""Force and torque on a wall by momentum exchange (lwacm_wall_force; Eqs.
MEA3-MEA5) against the oracle's wall_force.

- Random walls with two ids, random states, halfway and interpolated walls
  (random q), D2Q9 and D3Q19: F and T of each id on the same state.
- The 192^3 cavity mask with a seeded random state (the bench's wall
  geometry at full size), halfway and q = 0.3: F and T of the lid and of the
  other walls.
- Steady plane Couette flow run on the GPU: the tangential force on the wall
  at rest is the shear stress rho nu U / H per wall node, halfway and
  off-lattice walls.
- Scope: FP16 storage declines it; no mask or id 0 is an error.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from gpu_helpers import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _library_order(q, qd_oracle):
    from paper_1111_2142_amd import lwacm as L
    _, v, _, _ = oracle.lattice_info(q)
    where = {tuple(int(c) for c in v[k]): k for k in range(q)}
    return np.stack([qd_oracle[where[vel]] for vel in L.LINK_VELOCITIES[q]])


def _compare(L, q, shape, mask, drho, u, qd, center, ids, omega=1.5):
    nz, ny, nx = shape
    s = L.Solver(q, nx, ny, nz, omega, mask=to_dev(mask, torch.uint8),
                 wall_u=[[0, 0, 0]] * (int(mask.max()) + 1),
                 qd=None if qd is None else to_dev(_library_order(q, qd)))
    s.set_state(to_dev(drho), to_dev(u))
    p = oracle.Problem(q, nx, ny, nz, omega=omega, mask=mask)
    worst = (0.0, 0.0)
    for wid in ids:
        Fg, Tg = s.wall_force(wid, center)
        Fo, To = oracle.wall_force(p, 1.0 + drho, u, wid, center=center, qd=qd)
        dF = float(np.abs(np.array(Fg) - Fo).max())
        dT = float(np.abs(np.array(Tg) - To).max())
        banner(f"wall force id {wid}: F {np.round(Fo, 6)}, |dF| {dF:.2e}, |dT| {dT:.2e}")
        assert dF < 1e-5 and dT < 2e-4
        worst = (max(worst[0], dF), max(worst[1], dT))
    s.close()
    return worst


@pytest.mark.parametrize("q,interp", [(9, False), (9, True), (19, False), (19, True)])
def test_random_walls_match_oracle(q, interp):
    L = need_gpu()
    banner(f"wall force random q={q} interp={interp}")
    shape = (1, 40, 48) if q == 9 else (12, 32, 32)
    d = 2 if q == 9 else 3
    rng = np.random.Generator(np.random.PCG64(61))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 3, int(mask.sum())).astype(np.uint8)
    drho, u = wl.random_state(shape, d, seed=62, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    qd = rng.uniform(0.05, 1.0, (q,) + shape).astype(np.float32).astype(np.float64) if interp else None
    _compare(L, q, shape, mask, drho, u, qd, (20.0, 15.0, 5.0), (1, 2))


@pytest.mark.parametrize("interp", [False, True])
def test_cavity_192_matches_oracle(interp):
    L = need_gpu()
    banner(f"wall force cavity 192^3 interp={interp}")
    n = 192
    mask = wl.cavity_mask(n)
    shape = mask.shape
    drho, u = wl.random_state(shape, 3, seed=63, du=0.02, drho=0.005)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    qd = np.full((19,) + shape, 0.3) if interp else None
    c = (n - 1) / 2.0
    _compare(L, 19, shape, mask, drho, u, qd, (c, c, c), (1, 2), omega=1.892148)


@pytest.mark.parametrize("q,qb,qt", [(9, 0.5, 0.5), (9, 0.2, 0.25), (19, 0.5, 0.5)])
def test_couette_wall_force_is_the_shear_stress(q, qb, qt):
    L = need_gpu()
    banner(f"wall force Couette q={q} qb={qb} qt={qt}")
    h, U, omega = 12, 0.01, 1.2
    d, v, _, _ = oracle.lattice_info(q)
    ax = 1 if q == 9 else 2
    shape = (1, h, 32) if q == 9 else (h, 16, 32)
    nz, ny, nx = shape
    mask = np.zeros(shape, np.uint8)
    sl = [slice(None)] * 3
    sl[2 - ax] = 0
    mask[tuple(sl)] = 1
    sl[2 - ax] = h - 1
    mask[tuple(sl)] = 2
    qd = np.full((q,) + shape, 0.5)
    for j in range(q):
        if v[j][ax] == -1:
            sl[2 - ax] = 1
            qd[(j,) + tuple(sl)] = qb
        if v[j][ax] == 1:
            sl[2 - ax] = h - 2
            qd[(j,) + tuple(sl)] = qt
    s = L.Solver(q, nx, ny, nz, omega, mask=to_dev(mask, torch.uint8),
                 wall_u=[[0, 0, 0], [0, 0, 0], [U, 0, 0]], qd=to_dev(_library_order(q, qd)))
    s.set_state(to_dev(np.zeros(shape)), to_dev(np.zeros((d,) + shape)))
    s.step(6000)
    F, T = s.wall_force(1)
    s.close()
    area = nx * (ny if q == 19 else 1)
    H = (h - 2 + qt) - (1 - qb)
    nu = (1.0 / omega - 0.5) / 3.0
    exact = nu * U / H * area
    banner(f"wall force Couette: F_x {F[0]:.6e}, exact {exact:.6e}, F_n {F[ax]:.6f}")
    assert abs(F[0] / exact - 1.0) < 1e-4
    assert abs(F[ax] / (-area / 3.0) - 1.0) < 1e-5


def test_wall_force_scope():
    L = need_gpu()
    banner("wall force scope")
    shape = (16, 32, 64)
    mask = np.zeros(shape, np.uint8)
    mask[:, 0] = 1
    s = L.Solver(19, 64, 32, 16, 1.5)
    with pytest.raises(L.LWACMError) as ei:
        s.wall_force(1)
    assert ei.value.code == L.LWACM_EINVAL
    s.close()
    s = L.Solver(19, 64, 32, 16, 1.5, mask=to_dev(mask, torch.uint8))
    with pytest.raises(L.LWACMError) as ei:
        s.wall_force(0)
    assert ei.value.code == L.LWACM_EINVAL
    s.close()
    h = L.Solver(19, 64, 32, 16, 1.5, storage=1, mask=to_dev(mask, torch.uint8))
    with pytest.raises(L.LWACMError) as ei:
        h.wall_force(1)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    h.close()
