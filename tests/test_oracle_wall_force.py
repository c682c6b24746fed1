"""Pins of the oracle's momentum-exchange force and torque on a wall
(Section "Moving complex boundaries", Eqs. MEA3, MEA4 and MEA5).

- A body at rest in fluid at rest (uniform density) feels no force and no
  torque: the hydrostatic parts of opposite faces cancel.
- A single flat wall face under fluid at rest with density rho feels the
  pressure rho/3 per wall node (the hydrostatic F_0 of the paper), exactly.
- Steady plane Couette flow (D2Q9 and D3Q19), halfway walls and walls cutting
  the links at q_b and q_t (Eq. ACM2.0cc): the tangential force on the wall at
  rest is the shear stress rho nu U / H per wall node, H the distance between
  the two wall positions and nu = (1/omega - 1/2)/3 (Eq. viscosity2), and the
  normal force is -rho/3 per node; the torque about a point on the wall's line
  of nodes is the lever arm times the force (T = r x F, sign checked).
- q = 1/2 on every link gives the halfway force bit for bit.
"""
import numpy as np
import pytest

import oracle
from oracle import Problem


def _couette(q, qb, qt, omega, steps, interp, U=0.01, h=12):
    d, v, _, _ = oracle.lattice_info(q)
    ax = 1 if q == 9 else 2
    shape = (1, h, 4) if q == 9 else (h, 4, 4)
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
    p = Problem(q, nx, ny, nz, omega=omega, mask=mask,
                wall_u=np.array([[0, 0, 0], [0, 0, 0], [U, 0, 0]]), rho0=1.0)
    rho, u = np.ones(shape), np.zeros((d,) + shape)
    for _ in range(steps):
        rho, u = oracle.step_q(p, rho, u, qd) if interp else oracle.step(p, rho, u)
    return p, rho, u, (qd if interp else None), ax, U


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("qb,qt,omega,steps,interp", [(0.5, 0.5, 1.2, 4000, False),
                                                      (0.3, 0.7, 1.0, 4000, True),
                                                      (0.7, 0.25, 1.2, 6000, True)])
def test_couette_wall_force_is_the_shear_stress(q, qb, qt, omega, steps, interp):
    p, rho, u, qd, ax, U = _couette(q, qb, qt, omega, steps, interp)
    nz, ny, nx = p.shape
    area = nx * (ny if q == 19 else 1)
    h = p.shape[2 - ax]
    H = (h - 2 + qt) - (1 - qb)
    nu = (1.0 / omega - 0.5) / 3.0
    r = float(rho[p.mask == 0].mean())
    center = ((nx - 1) / 2.0, (ny - 1) / 2.0 if q == 19 else 0.0, 0.0)
    F, T = oracle.wall_force(p, rho, u, 1, center=center, qd=qd)
    assert abs(F[0] / (r * nu * U / H * area) - 1.0) < 1e-9
    assert abs(F[ax] / (-r / 3.0 * area) - 1.0) < 1e-12
    other = [k for k in range(3) if k not in (0, ax)]
    assert all(abs(F[k]) < 1e-14 for k in other)
    if q == 9:   # wall nodes at y = 1 on the line y_c = 0: T_z = -1 * F_x
        assert abs(T[2] + F[0]) < 1e-12 and abs(T[0]) < 1e-14 and abs(T[1]) < 1e-14
    else:        # wall nodes at z = 1: T_y = +1 * F_x, T_x = T_z = 0
        assert abs(T[1] - F[0]) < 1e-12 and abs(T[0]) < 1e-12 and abs(T[2]) < 1e-12


@pytest.mark.parametrize("q,shape", [(9, (1, 16, 20)), (19, (10, 12, 14))])
def test_body_at_rest_in_fluid_at_rest(q, shape):
    d = 2 if q == 9 else 3
    nz, ny, nx = shape
    mask = np.zeros(shape, np.uint8)
    if q == 9:
        mask[0, 5:10, 6:12] = 1
        mask[0, 12, 2:5] = 2
    else:
        mask[3:7, 4:8, 5:10] = 1
    p = Problem(q, nx, ny, nz, omega=1.4, mask=mask)
    rho = np.full(shape, 1.03)
    u = np.zeros((d,) + shape)
    F, T = oracle.wall_force(p, rho, u, 1, center=(nx / 3.0, ny / 2.0, nz / 4.0))
    assert np.abs(F).max() < 1e-14 and np.abs(T).max() < 1e-13
    # one flat wall face under fluid at rest (the wall, id 1, is backed by a
    # second layer with id 2, so only the face towards the fluid across the
    # periodic wrap counts): the pressure rho/3 per node, pushing along +normal
    m2 = np.zeros(shape, np.uint8)
    if q == 9:
        m2[0, 0, :] = 1
        m2[0, 1, :] = 2
        F, _ = oracle.wall_force(Problem(q, nx, ny, nz, omega=1.4, mask=m2), rho, u, 1)
        assert abs(F[1] - 1.03 / 3.0 * nx) < 1e-13 and abs(F[0]) < 1e-14
    else:
        m2[:, :, 0] = 1
        m2[:, :, 1] = 2
        F, _ = oracle.wall_force(Problem(q, nx, ny, nz, omega=1.4, mask=m2), rho, u, 1)
        assert abs(F[0] - 1.03 / 3.0 * ny * nz) < 1e-12 and abs(F[1]) < 1e-14


@pytest.mark.parametrize("q,shape", [(9, (1, 14, 18)), (19, (8, 10, 12))])
def test_q_one_half_is_the_halfway_force(q, shape):
    d = 2 if q == 9 else 3
    nz, ny, nx = shape
    rng = np.random.Generator(np.random.PCG64(5))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 3, int(mask.sum())).astype(np.uint8)
    rho = 1.0 + 0.01 * rng.standard_normal(shape)
    u = 0.03 * rng.standard_normal((d,) + shape)
    p = Problem(q, nx, ny, nz, omega=1.5, mask=mask)
    a = oracle.wall_force(p, rho, u, 1, center=(3.0, 2.0, 1.0))
    b = oracle.wall_force(p, rho, u, 1, center=(3.0, 2.0, 1.0), qd=np.full((q,) + shape, 0.5))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
