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


# ------------------------------------------- Appendix E with omega_p != omega
def _cse_appendix_E(rho, u, v, omega, omega_p):
    """The D2Q9 update of Appendix E in its optimised form, Eqs. CSE-CSE4,
    on periodic fields: M(1) = p = rho/3, M(2) = u, M(3) = v, E = (i+1, j),
    N = (i, j+1).  Constants as the appendix lists them, with the first
    "b = 2 - 2/omega" read as a = 2 - 2/omega (a4 = a/4) and b = 2 - 2/omega_p
    (b4 = b/4); the x-momentum line prints b4 where the y-momentum line has a4,
    and the momentum is relaxed with omega, so both lines take a4.  Returns
    (rho+, u+, v+)."""
    def at(f, dx, dy):  # f at (i + dx, j + dy)
        return np.roll(np.roll(f, -dx, axis=-1), -dy, axis=-2)

    M1 = rho / 3.0
    a, b = 2.0 - 2.0 / omega, 2.0 - 2.0 / omega_p
    a4, b4, r13, r43 = a / 4.0, b / 4.0, 1.0 / 3.0, 4.0 / 3.0

    def nb(dx, dy):
        return at(M1, dx, dy), at(u, dx, dy), at(v, dx, dy)

    pE, uE, vE = nb(1, 0)
    pW, uW, vW = nb(-1, 0)
    pN, uN, vN = nb(0, 1)
    pS, uS, vS = nb(0, -1)
    pNE, uNE, vNE = nb(1, 1)
    pNW, uNW, vNW = nb(-1, 1)
    pSE, uSE, vSE = nb(1, -1)
    pSW, uSW, vSW = nb(-1, -1)
    # Eq. CSE
    puP, pvP = M1 * u, M1 * v
    phuP, phvP = 2 * puP, 2 * pvP
    pvN, pvS, puE, puW = pN * vN, pS * vS, pE * uE, pW * uW
    puNE, puNW, puSE, puSW = pNE * uNE, pNW * uNW, pSE * uSE, pSW * uSW
    pvNE, pvNW, pvSE, pvSW = pNE * vNE, pNW * vNW, pSE * vSE, pSW * vSW
    # Eq. CSE2
    f1 = puE * (-uE + 1) + pE * (vE ** 2 / 2 - r13)
    f2 = puW * (uW + 1) - pW * (vW ** 2 / 2 - r13)
    f3 = pvN * (-vN + 1) + pN * (uN ** 2 / 2 - r13)
    f4 = pvS * (vS + 1) - pS * (uS ** 2 / 2 - r13)
    f5 = puNE * (uNE + 3 * vNE - 1) + pvNE * (vNE - 1) + pNE * r13
    f6 = puNW * (uNW - 3 * vNW + 1) + pvNW * (vNW - 1) + pNW * r13
    f7 = puSE * (uSE - 3 * vSE - 1) + pvSE * (vSE + 1) + pSE * r13
    f8 = puSW * (uSW + 3 * vSW + 1) + pvSW * (vSW + 1) + pSW * r13
    # Eq. CSE3
    fPp, fPm = puP + pvP, puP - pvP
    fNEp, fSWp, fNWm, fSEm = puNE + pvNE, puSW + pvSW, puNW - pvNW, puSE - pvSE
    FNE, FSW, FNW, FSE = fNEp - fPp, fPp - fSWp, fNWm - fPm, fPm - fSEm
    FNWSE, FNESW = FNW - FSE, FNE - FSW
    # Eq. CSE4
    rp = (M1 * r43 - phuP * u - phvP * v + f2 - f1 + f4 - f3 + (f5 + f6 + f7 + f8) / 4
          - b4 * (FNW + FSE - FNE - FSW) + b * (puE - puW + pvN - pvS))
    up = (f1 + f2 + (f6 - f5 - f7 + f8) / 4 - a * (puE - phuP + puW)
          - a4 * (FNESW + FNWSE)) / rp
    vp = (f3 + f4 + (f7 + f8 - f5 - f6) / 4 - a * (pvN - phvP + pvS)
          - a4 * (FNESW - FNWSE)) / rp
    return rp, up, vp


@pytest.mark.parametrize("omega,omega_p", [(1.6, 1.1), (1.3, 1.85), (1.9, 1.02), (1.5, 1.5)])
def test_split_step_equals_appendix_E_optimised_formulas(omega, omega_p):
    """The paper's own printed omega_p != omega update (Appendix E, Eqs.
    CSE-CSE4) equals the oracle's split step to rounding on random states."""
    nx, ny = 11, 7
    rng = np.random.Generator(np.random.PCG64(7))
    rho = 1.0 + rng.uniform(-0.05, 0.05, (1, ny, nx))
    u = rng.uniform(-0.08, 0.08, (2, 1, ny, nx))
    r1, u1 = oracle.step(Problem(q=9, nx=nx, ny=ny, omega=omega, omega_p=omega_p), rho, u)
    rp, up, vp = _cse_appendix_E(rho[0], u[0, 0], u[1, 0], omega, omega_p)
    assert np.abs(r1[0] - rp).max() < 1e-14
    assert np.abs(u1[0, 0] - up).max() < 1e-15
    assert np.abs(u1[1, 0] - vp).max() < 1e-15


def test_appendix_E_x_momentum_with_b4_is_not_the_split_update():
    """Read literally (b4 in the x-momentum line), Eq. CSE4 would let omega_p
    act on the x-momentum only; that differs from the split step by O(1e-2)
    here, so the a4 reading is the consistent one."""
    nx, ny, omega, omega_p = 11, 7, 1.6, 1.1
    rng = np.random.Generator(np.random.PCG64(7))
    rho = 1.0 + rng.uniform(-0.05, 0.05, (1, ny, nx))
    u = rng.uniform(-0.08, 0.08, (2, 1, ny, nx))
    r1, u1 = oracle.step(Problem(q=9, nx=nx, ny=ny, omega=omega, omega_p=omega_p), rho, u)
    # b4 in the x line differs from a4 by (b - a)/4 times (FNESW + FNWSE) / rho+
    rp, up, _ = _cse_appendix_E(rho[0], u[0, 0], u[1, 0], omega, omega_p)
    assert np.abs(u1[0, 0] - up).max() < 1e-15
    a, b = 2 - 2 / omega, 2 - 2 / omega_p
    M1 = rho[0] / 3

    def at(f, dx, dy):
        return np.roll(np.roll(f, -dx, axis=-1), -dy, axis=-2)

    pu, pv = M1 * u[0, 0], M1 * u[1, 0]
    fNE = at(pu, 1, 1) + at(pv, 1, 1) - (pu + pv)
    fSW = (pu + pv) - (at(pu, -1, -1) + at(pv, -1, -1))
    fNW = at(pu, -1, 1) - at(pv, -1, 1) - (pu - pv)
    fSE = (pu - pv) - (at(pu, 1, -1) - at(pv, 1, -1))
    literal = up - (b - a) / 4 * ((fNE - fSW) + (fNW - fSE)) / rp
    assert np.abs(u1[0, 0] - literal).max() > 1e-4


def _fr(s):
    from fractions import Fraction
    return float(Fraction(s))


@pytest.mark.parametrize("lattice", ["d2q9", "d3q19"])
def test_moving_wall_density_term_takes_omega_p(golden_dir, lattice):
    """Hand-derived exact values (tests/golden/hand_moving_wall_split.json):
    one moving solid node on a 3-periodic grid at rest.  Each of its link
    neighbours gains 6 w_i rho0 h_p (v_i . u_w) of density (h_p = 2/omega_p -
    1) and v_i 6 w_i rho0 h (v_i . u_w) of momentum: the moving-wall term of
    the density takes omega_p, that of the momentum omega.  The terms do not
    cancel at a single node (unlike a flat wall moving in its plane)."""
    import json
    import os
    g = json.load(open(os.path.join(golden_dir, "hand_moving_wall_split.json")))
    c = g[lattice]
    q, d = (9, 2) if lattice == "d2q9" else (19, 3)
    shape = (1, 3, 3) if q == 9 else (3, 3, 3)
    mask = np.zeros(shape, dtype=np.uint8)
    sol = c["solid"] + [0] if q == 9 else c["solid"]
    mask[sol[2], sol[1], sol[0]] = 2
    wall = np.zeros((3, 3))
    wall[2, :d] = [_fr(s) for s in c["wall_u"]]
    rho = np.ones(shape)
    u = np.zeros((d,) + shape)
    for split in (True, False):
        p = Problem(q=q, nx=3, ny=3, nz=shape[0], omega=_fr(g["omega"]), mask=mask,
                    wall_u=wall, rho0=1.0, omega_p=_fr(g["omega_p"]) if split else None)
        r1, u1 = oracle.step(p, rho, u)
        for e in c["expect"]:
            x, y = e["node"][0], e["node"][1]
            z = e["node"][2] if q == 19 else 0
            want = _fr(e["rho"] if split else e["rho_single"])
            assert abs(r1[z, y, x] - want) < 1e-15, (lattice, split, e)
            if split:
                for k in range(d):
                    assert abs(u1[k, z, y, x] - _fr(e["u"][k])) < 1e-16, (lattice, e, k)
