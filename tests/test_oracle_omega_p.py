"""Pins of the oracle's step with a separate relaxation omega_p for the
continuity equation (Section "finite-difference formulation", item 3;
Appendix E: the density update takes b = 2 - 2/omega_p where the momentum
update takes a = 2 - 2/omega).

The oracle evaluates the populations of Eq. ACM2.0 once with each relaxation
and takes the density from the omega_p set, the momentum from the omega set.
These checks do not re-evaluate that: they use what the mathematics fixes.

- omega_p = omega is the single-relaxation step, bit for bit.
- The density update conserves mass exactly for any omega_p, on a periodic
  grid and with walls at rest (halfway bounce-back returns every term sent
  into a wall to its sender).
- The momentum rho u does not depend on omega_p.
- Closed form: only the odd part of the upstream equilibria carries b, so
  rho+(omega_p) - rho+(omega) = -(b - a) sum_i 3 w_i v_i . (rho u)(x - v_i).
  For rho = 1 and u_x = U cos(k x) the sum is U sin(k) sin(k x) on both
  lattices (sum of w_i v_ix^2 = 1/3).
"""
import numpy as np
import pytest

import oracle
from oracle import Problem

pytestmark = pytest.mark.filterwarnings("ignore")


def _random_state(q, shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    d = 2 if q == 9 else 3
    rho = 1.0 + 0.01 * rng.standard_normal(shape)
    u = 0.03 * rng.standard_normal((d,) + shape)
    return rho, u


@pytest.mark.parametrize("q,shape", [(9, (1, 12, 16)), (19, (6, 8, 10))])
def test_omega_p_equal_to_omega_is_the_single_relaxation_step(q, shape):
    rho, u = _random_state(q, shape, 1)
    nz, ny, nx = shape
    base = Problem(q, nx, ny, nz, omega=1.7)
    same = Problem(q, nx, ny, nz, omega=1.7, omega_p=1.7)
    r0, u0 = oracle.step(base, rho, u)
    r1, u1 = oracle.step(same, rho, u)
    assert np.array_equal(r0, r1) and np.array_equal(u0, u1)


@pytest.mark.parametrize("q,shape", [(9, (1, 12, 16)), (19, (6, 8, 10))])
@pytest.mark.parametrize("omega_p", [0.6, 1.0, 1.95])
def test_omega_p_conserves_mass_on_a_periodic_grid(q, shape, omega_p):
    rho, u = _random_state(q, shape, 2)
    nz, ny, nx = shape
    p = Problem(q, nx, ny, nz, omega=1.8, omega_p=omega_p)
    r1, _ = oracle.step(p, rho, u)
    assert abs(r1.sum() - rho.sum()) <= 1e-12 * rho.sum()


@pytest.mark.parametrize("q,shape", [(9, (1, 14, 18)), (19, (8, 10, 12))])
def test_omega_p_conserves_mass_with_walls_at_rest(q, shape):
    rho, u = _random_state(q, shape, 3)
    nz, ny, nx = shape
    rng = np.random.Generator(np.random.PCG64(4))
    mask = (rng.random(shape) < 0.12).astype(np.uint8)
    fl = mask == 0
    p = Problem(q, nx, ny, nz, omega=1.6, omega_p=0.9, mask=mask)
    r1, _ = oracle.step(p, rho, u)
    assert abs(r1[fl].sum() - rho[fl].sum()) <= 1e-12 * rho[fl].sum()
    # the same density with omega_p = omega differs: the split is not a no-op
    r0, _ = oracle.step(Problem(q, nx, ny, nz, omega=1.6, mask=mask), rho, u)
    assert np.abs(r1 - r0).max() > 1e-6


@pytest.mark.parametrize("q,shape", [(9, (1, 12, 16)), (19, (6, 8, 10))])
def test_omega_p_leaves_the_momentum_unchanged(q, shape):
    rho, u = _random_state(q, shape, 5)
    nz, ny, nx = shape
    g = (2e-4, -1e-4, 5e-5)[:2 if q == 9 else 3]
    j = []
    for omega_p in (None, 0.7, 1.9):
        p = Problem(q, nx, ny, nz, omega=1.5, omega_p=omega_p, g=g)
        r1, u1 = oracle.step(p, rho, u)
        j.append(r1 * u1)
    for jj in j[1:]:
        assert np.allclose(jj, j[0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("q,shape,axis", [(9, (1, 6, 24), 2), (19, (20, 4, 6), 0)])
@pytest.mark.parametrize("omega,omega_p", [(1.9, 1.2), (0.8, 1.7)])
def test_omega_p_density_change_closed_form(q, shape, axis, omega, omega_p):
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    n_ax = shape[axis]
    m, U = 2, 0.05
    k = 2.0 * np.pi * m / n_ax
    coord = np.arange(n_ax).reshape([-1 if a == axis else 1 for a in range(3)])
    wave = np.broadcast_to(np.cos(k * coord), shape)
    rho = np.ones(shape)
    u = np.zeros((d,) + shape)
    comp = {2: 0, 1: 1, 0: 2}[axis]  # x, y or z velocity component along the wave
    u[comp] = U * wave
    r_a, _ = oracle.step(Problem(q, nx, ny, nz, omega=omega), rho, u)
    r_b, _ = oracle.step(Problem(q, nx, ny, nz, omega=omega, omega_p=omega_p), rho, u)
    a, b = 2.0 - 2.0 / omega, 2.0 - 2.0 / omega_p
    expect = -(b - a) * U * np.sin(k) * np.broadcast_to(np.sin(k * coord), shape)
    assert np.abs((r_b - r_a) - expect).max() <= 1e-14
