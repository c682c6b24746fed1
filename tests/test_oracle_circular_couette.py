"""Oracle pins of wall velocities given link by link and of the circular
Couette flow (Section "Circular Couette flow": interpolated bounce-back,
Eq. ACM2.0cc, with the moving-wall term of Eq. ACM2.0move on a turning
cylinder, and the torque by momentum exchange, Eqs. MEA3 and MEA5).

- Link velocities equal to the per-id table give the table's step bit for
  bit (halfway and interpolated walls; D2Q9 and D3Q19): the link-by-link
  input only changes where u_w comes from, and the table path is pinned by
  exact plane Couette flow (test_oracle_interpolated_bb.py).
- The circular Couette run converges to the exact solution of Eqs.
  circcouttesol / circcouttesolC at second order in eps for u_theta and p,
  and the torque on the inner cylinder to 4 pi C nu r_i.
- The L1 errors are of the size the paper prints (within a factor of 3 of
  its table at eps = 1/20 and 1/40; the radii, the node placement and the
  norm are readings, see tests/circular_couette.py and workloads).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as wl
from circular_couette import exact, l1_errors


def _walls(q, shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = (rng.random(shape) < 0.12).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 4, int(mask.sum())).astype(np.uint8)
    table = np.array([[0, 0, 0], [0, 0, 0], [0.03, -0.01, 0.02], [-0.02, 0.015, 0.01]])
    return mask, table, rng


@pytest.mark.parametrize("q,shape", [(9, (1, 18, 22)), (19, (8, 10, 12))])
@pytest.mark.parametrize("interpolated", [False, True])
def test_link_velocities_equal_to_the_table_give_the_table_step(q, shape, interpolated):
    d = 2 if q == 9 else 3
    mask, table, rng = _walls(q, shape, 3)
    _, v, _, _ = oracle.lattice_info(q)
    if d == 2:
        table = table.copy()
        table[:, 2] = 0.0
    qd = rng.uniform(0.05, 1.0, (q,) + shape) if interpolated else None
    # the table's velocity of the solid node each link of each node points at
    nz, ny, nx = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    uwl = np.zeros((q, d) + shape)
    for j in range(q):
        tgt = mask[(zz + v[j][2]) % nz, (yy + v[j][1]) % ny, (xx + v[j][0]) % nx]
        uwl[j] = np.moveaxis(table[tgt][..., :d], -1, 0)
    drho, u = wl.random_state(shape, d, seed=5, du=0.03, drho=0.01)
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=1.7, mask=mask, wall_u=table,
                       rho0=1.004)
    r_a, u_a = oracle.step_q(p, 1 + drho, u, qd)
    r_b, u_b = oracle.step_q(p, 1 + drho, u, qd, uwl)
    assert np.array_equal(r_a, r_b) and np.array_equal(u_a, u_b)
    # and the input is used: other link velocities change the step
    r_c, _ = oracle.step_q(p, 1 + drho, u, qd, 1.5 * uwl)
    assert np.abs(r_c - r_a).max() > 1e-6


def _circular(eps, t_end=20.0):
    cc = wl.CircularCouette(eps)
    _, v, _, _ = oracle.lattice_info(9)
    qd, uwl = cc.links(v)
    p = oracle.Problem(q=9, nx=cc.n, ny=cc.n, omega=cc.omega, mask=cc.mask,
                       wall_u=np.zeros((3, 3)), rho0=1.0)
    rho, u = np.ones((1, cc.n, cc.n)), np.zeros((2, 1, cc.n, cc.n))
    for _ in range(cc.steps_to(t_end)):
        rho, u = oracle.step_q(p, rho, u, qd, uwl)
    _, T = oracle.wall_force(p, rho, u, 1, center=cc.center, qd=qd)
    return cc, rho, u, T


def test_geometry_of_the_links():
    """q is where the link meets the circle; the wall velocity there is
    tangential with speed eps (the outer wall's unit physical speed)."""
    cc = wl.CircularCouette(1 / 20)
    _, v, _, _ = oracle.lattice_info(9)
    qd, uwl = cc.links(v)
    hit = qd > 0
    assert hit.any() and np.all(qd[hit] <= 1.0)
    for j in range(1, 9):
        ys, xs = np.nonzero(hit[j, 0])
        assert len(xs) > 0
        px = cc.X[ys, xs] + qd[j, 0, ys, xs] * v[j][0] * cc.eps
        py = cc.Y[ys, xs] + qd[j, 0, ys, xs] * v[j][1] * cc.eps
        r = np.hypot(px, py)
        outer = cc.mask[0, ys + v[j][1], xs + v[j][0]] == 2
        assert np.allclose(r[outer], cc.r_e, atol=1e-12)
        assert np.allclose(r[~outer], cc.r_i, atol=1e-12)
        speed = np.hypot(uwl[j, 0, 0, ys, xs], uwl[j, 1, 0, ys, xs])
        assert np.allclose(speed[outer], cc.eps, atol=1e-14)
        assert np.all(speed[~outer] == 0.0)
        radial = uwl[j, 0, 0, ys, xs] * px + uwl[j, 1, 0, ys, xs] * py
        assert np.abs(radial).max() < 1e-15


def test_circular_couette_converges_to_the_exact_solution():
    errs = {}
    for k in (10, 20, 40):
        cc, rho, u, T = _circular(1 / k)
        errs[k] = l1_errors(cc, rho, u, T[2])
        f = cc.fluid
        ur = (cc.X[f] * u[0, 0][f] + cc.Y[f] * u[1, 0][f]) / cc.R[f] / cc.eps
        assert np.abs(ur).max() < 0.02 * 40 / k  # the flow is azimuthal
        assert abs(T[0]) < 1e-12 and abs(T[1]) < 1e-12  # 2D: torque along z only
    for i in range(2):  # u_theta, p: second order (1/20 -> 1/40)
        assert errs[20][i] / errs[40][i] > 2.8, (i, errs)
        assert errs[10][i] / errs[20][i] > 1.8, (i, errs)
    _, _, t_ex = exact(wl.CircularCouette(1 / 40))
    assert errs[40][2] < 1e-3 * t_ex * 1.0  # torque within 0.1 % at 1/40
    assert errs[20][2] / errs[40][2] > 1.8   # and converging


def test_errors_are_of_the_printed_size(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "circular_couette_table.json")))
    for col, k in ((0, 20), (1, 40)):
        assert Fraction(g["eps"][col]) == Fraction(1, k)
        cc, rho, u, T = _circular(1 / k)
        e = l1_errors(cc, rho, u, T[2])
        for i, name in enumerate(("u_theta", "p", "torque")):
            ratio = e[i] / g[name][col]
            assert 1 / 3 < ratio < 3, (k, name, e[i], g[name][col])
