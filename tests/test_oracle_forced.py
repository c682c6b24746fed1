"""Pins of the oracle's step with a body acceleration given node by node (the
space- and time-dependent forcing of the paper's generalized Taylor-Green
vortex, Eq. external-force; applied by Eq. force).

- A field that is uniform gives the uniform-g step, bit for bit.
- Eq. force adds the odd part 3 w_i rho (v_i . g) to every population: the
  density does not change, and the momentum of every node gains exactly
  rho(x, t) g(x) over the unforced step (sum of 3 w_i v_i v_i = identity).
- The generalized Taylor-Green vortex (diffusive scaling, nu = 0.1, t = 60):
  the oracle's L1 errors against the analytic solution are compared with the
  paper's printed table (tests/golden/forced_tgv_l1.json).  The paper does not
  state the norm's normalisation or the initial pressure; with the mean
  absolute error over nodes and rho = 1 + 3 eps^2 p_bar(0), the oracle's errors
  are 86-94 % of the printed ones at eps = pi/16 and 92-96 % at pi/32, and
  they converge at second order as the table does.  The band below (0.8 to
  1.05 of the printed value) is that agreement, not an exact match.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import Problem

HERE = os.path.dirname(os.path.abspath(__file__))


def _state(q, shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    d = 2 if q == 9 else 3
    return 1.0 + 0.01 * rng.standard_normal(shape), 0.03 * rng.standard_normal((d,) + shape)


@pytest.mark.parametrize("q,shape", [(9, (1, 12, 16)), (19, (6, 8, 10))])
def test_uniform_field_is_the_uniform_acceleration_step(q, shape):
    rho, u = _state(q, shape, 1)
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    g = (3e-4, -2e-4, 1e-4)[:d]
    rng = np.random.Generator(np.random.PCG64(2))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    for m in (None, mask):
        r0, u0 = oracle.step(Problem(q, nx, ny, nz, omega=1.6, g=g, mask=m), rho, u)
        field = np.broadcast_to(np.asarray(g).reshape((d, 1, 1, 1)), (d,) + shape)
        r1, u1 = oracle.step_field(Problem(q, nx, ny, nz, omega=1.6, mask=m), rho, u, field)
        assert np.array_equal(r0, r1) and np.array_equal(u0, u1)


@pytest.mark.parametrize("q,shape", [(9, (1, 12, 16)), (19, (6, 8, 10))])
def test_field_adds_rho_g_to_every_node_momentum(q, shape):
    rho, u = _state(q, shape, 3)
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    rng = np.random.Generator(np.random.PCG64(4))
    g = 1e-3 * rng.standard_normal((d,) + shape)
    p = Problem(q, nx, ny, nz, omega=1.4)
    r0, u0 = oracle.step(p, rho, u)
    r1, u1 = oracle.step_field(p, rho, u, g)
    assert np.allclose(r1, r0, rtol=0, atol=1e-15)
    assert np.allclose(r1 * u1 - r0 * u0, rho * g, rtol=0, atol=1e-15)


def test_forced_taylor_green_l1_errors_near_the_printed_table():
    ref = json.load(open(os.path.join(HERE, "golden", "forced_tgv_l1.json")))["l1_errors_at_t60"]
    errs = {}
    for m in (16, 32):
        c = wl.ForcedTaylorGreen(m)
        p = Problem(9, c.n, c.n, 1, omega=c.omega)
        drho, u = c.initial_state()
        rho = 1.0 + drho
        steps = c.steps_to(60.0)
        for s in range(steps):
            rho, u = oracle.step_field(p, rho, u, c.acceleration(s))
        errs[m] = c.l1_errors(steps, rho - 1.0, u)
        printed = ref[f"pi/{m}"]
        for k, e in zip(("u", "v", "p"), errs[m]):
            assert 0.8 <= e / printed[k] <= 1.05, (m, k, e, printed[k])
    for a, b in zip(errs[16], errs[32]):
        assert 3.0 <= a / b <= 4.5  # second order: halving eps divides the error by ~4
