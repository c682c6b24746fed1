"""Pins of the oracle's interpolated bounce-back (Section "Moving complex
boundaries", Eq. ACM2.0cc, moving-wall term Eq. ACM2.0move).

- q = 1/2 on every link gives the halfway rule of oracle.step, bit for bit
  (random walls with moving ids).
- Plane Couette flow between walls that cut the links at fractions q_b and
  q_t of their length (the bottom wall at rest at y = 1 - q_b, the top wall
  moving at U at y = ny - 2 + q_t): the steady state is the linear profile
  between the two wall positions, exactly (the interpolation is linear, and
  so is the profile).  D2Q9 and D3Q19, several (q_b, q_t, omega); omega >= 1
  (below 1 the run is unstable with the halfway rule as well).
"""
import numpy as np
import pytest

import oracle
from oracle import Problem


def _state(q, shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    d = 2 if q == 9 else 3
    return 1.0 + 0.01 * rng.standard_normal(shape), 0.03 * rng.standard_normal((d,) + shape)


@pytest.mark.parametrize("q,shape", [(9, (1, 14, 18)), (19, (8, 10, 12))])
def test_q_one_half_is_the_halfway_rule(q, shape):
    rho, u = _state(q, shape, 1)
    nz, ny, nx = shape
    rng = np.random.Generator(np.random.PCG64(2))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 3, int(mask.sum())).astype(np.uint8)
    table = np.array([[0, 0, 0], [0, 0, 0], [0.02, -0.01, 0.01]])
    p = Problem(q, nx, ny, nz, omega=1.5, mask=mask, wall_u=table, rho0=1.0)
    r0, u0 = oracle.step(p, rho, u)
    r1, u1 = oracle.step_q(p, rho, u, np.full((q,) + shape, 0.5))
    assert np.array_equal(r0, r1) and np.array_equal(u0, u1)


def _couette(q, qb, qt, omega, steps, U=0.01, h=12):
    """Walls normal to y (D2Q9) or z (D3Q19), h nodes across including the two
    solid layers; returns the max deviation from the linear profile / U."""
    d, v, _, _ = oracle.lattice_info(q)
    ax = 1 if q == 9 else 2  # wall-normal axis (velocity component index)
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
    table = np.array([[0, 0, 0], [0, 0, 0], [U, 0, 0]])
    p = Problem(q, nx, ny, nz, omega=omega, mask=mask, wall_u=table, rho0=1.0)
    rho, u = np.ones(shape), np.zeros((d,) + shape)
    for _ in range(steps):
        rho, u = oracle.step_q(p, rho, u, qd)
    coord = np.arange(1, h - 1)
    exact = U * (coord - (1 - qb)) / ((h - 2 + qt) - (1 - qb))
    sl[2 - ax] = slice(1, h - 1)
    ux = u[0][tuple(sl)]
    prof = ux.reshape(h - 2, -1) if ax == 2 else np.moveaxis(ux, 1, 0).reshape(h - 2, -1)
    return float(np.abs(prof - exact[:, None]).max() / U)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("qb,qt,omega,steps", [(0.3, 0.7, 1.0, 4000), (0.2, 0.8, 1.6, 12000),
                                               (0.7, 0.25, 1.2, 6000)])
def test_couette_between_off_lattice_walls_is_exact(q, qb, qt, omega, steps):
    assert _couette(q, qb, qt, omega, steps) < 1e-9
