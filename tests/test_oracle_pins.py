"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each checks it against a
second printed statement of the same update (Appendix E), the explicit
equilibrium list of Appendix A, hand-derived exact values, exact invariants,
or closed-form discrete solutions derived from the scheme.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as wl


# ---------------------------------------------------------------- lattices
@pytest.mark.parametrize("q", [9, 19])
def test_lattice_moments(q):
    """sum w = 1, sum w v = 0, sum w v v = I/3 and the 4th-order isotropy
    sum w v_a v_b v_c v_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9 (Appendix A
    lattices; the identities Section 2.1 needs to recover Euler/NS)."""
    d, v, w, opp = oracle.lattice_info(q)
    v = v[:, :d].astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs((w[:, None] * v).sum(0)).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib->ab", w, v, v) - np.eye(d) / 3).max() < 1e-15
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, v, v, v, v)
    I = np.eye(d)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9
    assert np.abs(m4 - iso).max() < 1e-15
    for i in range(q):
        assert np.all(v[opp[i]] == -v[i])
    # all links distinct, |v|_inf = 1
    assert len({tuple(r) for r in v}) == q
    assert np.abs(v).max() == 1


def test_d2q9_order_is_appendix_A():
    """1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
    with w = 4/9, 1/9 x4, 1/36 x4 (Appendix A, Eqs. weight_factors and
    d2q9_equilibrium)."""
    _, v, w, _ = oracle.lattice_info(9)
    expect = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    assert [tuple(r[:2]) for r in v] == expect
    assert np.allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-16)


@pytest.mark.parametrize("rho_c,uc", [(1.0, (0.03, -0.02)), (1.2, (-0.07, 0.05))])
def test_equilibrium_matches_appendix_A_list(rho_c, uc):
    """With omega = 1 the update reduces to f_i(x) = f^(e)_i(x - v_i) (the
    LKS special case named in Section 2.2).  On a 3-periodic lattice with a
    single non-rest centre, node c+v_i receives exactly f^(e)_i(c), so
    rho+(c+v_i) = 1 - w_i + f^(e)_i(c).  Compare every link with the explicit
    D2Q9 equilibrium list printed in Appendix A (Eq. d2q9_equilibrium)."""
    p = oracle.Problem(q=9, nx=3, ny=3, omega=1.0)
    rho = np.ones((1, 3, 3))
    u = np.zeros((2, 1, 3, 3))
    rho[0, 1, 1] = rho_c
    u[:, 0, 1, 1] = uc
    r1, _ = oracle.step(p, rho, u)
    _, v, w, _ = oracle.lattice_info(9)
    R, U, V = rho_c, uc[0], uc[1]
    listed = [
        4 / 9 * R - 2 / 3 * R * U ** 2 - 2 / 3 * R * V ** 2,
        1 / 9 * R + 1 / 3 * R * U + 1 / 3 * R * U ** 2 - 1 / 6 * R * V ** 2,
        1 / 9 * R + 1 / 3 * R * V + 1 / 3 * R * V ** 2 - 1 / 6 * R * U ** 2,
        1 / 9 * R - 1 / 3 * R * U + 1 / 3 * R * U ** 2 - 1 / 6 * R * V ** 2,
        1 / 9 * R - 1 / 3 * R * V + 1 / 3 * R * V ** 2 - 1 / 6 * R * U ** 2,
        1 / 36 * R + 1 / 12 * R * (U + V) + 1 / 8 * R * (U + V) ** 2 - 1 / 24 * R * (U ** 2 + V ** 2),
        1 / 36 * R - 1 / 12 * R * (U - V) + 1 / 8 * R * (-U + V) ** 2 - 1 / 24 * R * (U ** 2 + V ** 2),
        1 / 36 * R - 1 / 12 * R * (U + V) + 1 / 8 * R * (-U - V) ** 2 - 1 / 24 * R * (U ** 2 + V ** 2),
        1 / 36 * R + 1 / 12 * R * (U - V) + 1 / 8 * R * (U - V) ** 2 - 1 / 24 * R * (U ** 2 + V ** 2),
    ]
    for i in range(1, 9):
        x, y = (1 + v[i][0]) % 3, (1 + v[i][1]) % 3
        got = r1[0, y, x] - 1 + w[i]
        assert abs(got - listed[i]) < 1e-15, (i, got, listed[i])
    # the centre keeps its rest population and receives w_i on every other link
    assert abs(r1[0, 1, 1] - (5 / 9 + listed[0])) < 1e-15


# ------------------------------------------ Appendix E: second printed form
def _fd_appendix_E(p, u, v, omega):
    """Eqs. FDjx, FDjy (reading '+' before the 2/3(1/omega-1) bracket, which
    the printed FDjy lacks) and FDpressure, with E = (n+1, m), N = (n, m+1)."""
    def sh(a, dx, dy):  # value at (n+dx, m+dy)
        return np.roll(np.roll(a, -dx, axis=-1), -dy, axis=-2)

    pE, uE, vE = sh(p, 1, 0), sh(u, 1, 0), sh(v, 1, 0)
    pW, uW, vW = sh(p, -1, 0), sh(u, -1, 0), sh(v, -1, 0)
    pN, uN, vN = sh(p, 0, 1), sh(u, 0, 1), sh(v, 0, 1)
    pS, uS, vS = sh(p, 0, -1), sh(u, 0, -1), sh(v, 0, -1)
    pNE, uNE, vNE = sh(p, 1, 1), sh(u, 1, 1), sh(v, 1, 1)
    pNW, uNW, vNW = sh(p, -1, 1), sh(u, -1, 1), sh(v, -1, 1)
    pSE, uSE, vSE = sh(p, 1, -1), sh(u, 1, -1), sh(v, 1, -1)
    pSW, uSW, vSW = sh(p, -1, -1), sh(u, -1, -1), sh(v, -1, -1)
    pP, uP, vP = p, u, v
    c = 2.0 / 3.0 * (1.0 / omega - 1.0)
    NE = pNE * (3 * uNE ** 2 + 9 * uNE * vNE - 3 * uNE + 3 * vNE ** 2 - 3 * vNE + 1) / 36
    NW = pNW * (3 * uNW ** 2 - 9 * uNW * vNW + 3 * uNW + 3 * vNW ** 2 - 3 * vNW + 1) / 36
    SE = pSE * (3 * uSE ** 2 - 9 * uSE * vSE - 3 * uSE + 3 * vSE ** 2 + 3 * vSE + 1) / 36
    SW = pSW * (3 * uSW ** 2 + 9 * uSW * vSW + 3 * uSW + 3 * vSW ** 2 + 3 * vSW + 1) / 36
    Ex = pE * (-6 * uE ** 2 + 6 * uE + 3 * vE ** 2 - 2) / 18
    Wx = pW * (6 * uW ** 2 + 6 * uW - 3 * vW ** 2 + 2) / 18
    Ny = pN * (3 * uN ** 2 - 6 * vN ** 2 + 6 * vN - 2) / 18
    Sy = pS * (-3 * uS ** 2 + 6 * vS ** 2 + 6 * vS + 2) / 18
    pu = (Ex + Wx - NE + NW - SE + SW
          + c * (pE * uE - 3 * pP * uP + pW * uW
                 + (pNE * uNE + pNW * uNW + pSE * uSE + pSW * uSW) / 4
                 + (pNE * vNE - pNW * vNW - pSE * vSE + pSW * vSW) / 4))
    pv = (Ny + Sy - NE - NW + SE + SW
          + c * (pN * vN - 3 * pP * vP + pS * vS
                 + (pNE * uNE - pNW * uNW - pSE * uSE + pSW * uSW) / 4
                 + (pNE * vNE + pNW * vNW + pSE * vSE + pSW * vSW) / 4))
    pp = (-2 * pP * (3 * uP ** 2 + 3 * vP ** 2 - 2) / 9
          - Ex + Wx - Ny + Sy + NE + NW + SE + SW
          + c * (-pE * uE + pS * vS + pW * uW - pN * vN
                 + (pSW * uSW + pNW * uNW - pNE * uNE - pSE * uSE) / 4
                 + (pSW * vSW - pNW * vNW - pNE * vNE + pSE * vSE) / 4))
    return pp, pu, pv


@pytest.mark.parametrize("omega", [1.0, 1.37, 1.6, 1.95])
def test_oracle_equals_appendix_E_formulas(omega):
    """The equivalent finite-difference formulas of Appendix E restate the
    D2Q9 update in moment form; they must match Eq. ACM2.0 to rounding."""
    nx, ny = 11, 7
    drho, u = wl.random_state((1, ny, nx), 2, seed=3, du=0.08, drho=0.05)
    rho = 1 + drho
    p = oracle.Problem(q=9, nx=nx, ny=ny, omega=omega)
    r1, u1 = oracle.step(p, rho, u)
    pp, pu, pv = _fd_appendix_E(rho[0] / 3, u[0, 0], u[1, 0], omega)
    assert np.abs(r1[0] / 3 - pp).max() < 1e-15
    assert np.abs(r1[0] * u1[0, 0] / 3 - pu).max() < 1e-15
    assert np.abs(r1[0] * u1[1, 0] / 3 - pv).max() < 1e-15


def test_appendix_E_without_plus_is_not_the_update():
    """Reading FDjy literally (no operator before the bracket, i.e. dropping
    that term) does not reproduce the update: the '+' reading is forced."""
    nx, ny, omega = 9, 8, 1.6
    drho, u = wl.random_state((1, ny, nx), 2, seed=4)
    rho = 1 + drho
    r1, u1 = oracle.step(oracle.Problem(q=9, nx=nx, ny=ny, omega=omega), rho, u)
    _, _, pv = _fd_appendix_E(rho[0] / 3, u[0, 0], u[1, 0], omega)
    _, _, pv_no_bracket = _fd_appendix_E(rho[0] / 3, u[0, 0], u[1, 0], 1.0)
    assert np.abs(r1[0] * u1[1, 0] / 3 - pv).max() < 1e-15
    assert np.abs(r1[0] * u1[1, 0] / 3 - pv_no_bracket).max() > 1e-5


# ---------------------------------------------- hand-derived exact values
def _frac(s):
    return float(Fraction(s)) if "/" in s or s.lstrip("-").isdigit() else float(s)


def test_hand_3x3_d2q9(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "hand_3x3.json")))["d2q9"]
    omega = _frac(g["omega"])
    for case in g["cases"]:
        rho = np.ones((1, 3, 3))
        u = np.zeros((2, 1, 3, 3))
        rho[0, 1, 1] = _frac(case["centre_rho"])
        u[:, 0, 1, 1] = [_frac(s) for s in case["centre_u"]]
        r1, u1 = oracle.step(oracle.Problem(q=9, nx=3, ny=3, omega=omega), rho, u)
        for e in case["expect"]:
            x, y = e["node"]
            assert abs(r1[0, y, x] - _frac(e["rho"])) < 1e-15, (case["name"], e)
            for k in range(2):
                assert abs(u1[k, 0, y, x] - _frac(e["u"][k])) < 2e-16, (case["name"], e, k)
        assert abs(r1.sum() - _frac(case["total_mass"])) < 1e-14
        mom = [(r1 * u1[k]).sum() for k in range(2)]
        assert np.allclose(mom, [_frac(s) for s in case["total_momentum"]], rtol=0, atol=1e-16)


def test_hand_3x3x3_d3q19(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "hand_3x3.json")))["d3q19"]
    rho = np.ones((3, 3, 3))
    u = np.zeros((3, 3, 3, 3))
    rho[1, 1, 1] = _frac(g["centre_rho"])
    u[:, 1, 1, 1] = [_frac(s) for s in g["centre_u"]]
    r1, u1 = oracle.step(oracle.Problem(q=19, nx=3, ny=3, nz=3, omega=_frac(g["omega"])), rho, u)
    for e in g["expect"]:
        x, y, z = e["node"]
        assert abs(r1[z, y, x] - _frac(e["rho"])) < 1e-15, e
        for k in range(3):
            assert abs(u1[k, z, y, x] - _frac(e["u"][k])) < 2e-16, (e, k)
    assert abs(r1.sum() - 27) < 1e-13
    mom = [(r1 * u1[k]).sum() for k in range(3)]
    assert np.allclose(mom, [_frac(s) for s in g["total_momentum"]], rtol=0, atol=1e-16)


# -------------------------------------------------------------- invariants
@pytest.mark.parametrize("q,shape", [(9, (1, 9, 13)), (19, (6, 5, 7))])
@pytest.mark.parametrize("force", [False, True])
def test_mass_and_momentum_periodic(q, shape, force):
    """Periodic domains: sum rho is conserved exactly; sum rho u is conserved
    without force and grows by exactly (sum rho) g per step with the forcing
    of Eq. force."""
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=11)
    rho = 1 + drho
    g = (2e-4, -1e-4, 3e-4)[:d] if force else None
    nz, ny, nx = shape
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=1.7, g=g)
    r, uu = rho, u
    for _ in range(5):
        m0 = r.sum()
        mom0 = np.array([(r * uu[k]).sum() for k in range(d)])
        r2, u2 = oracle.step(p, r, uu)
        assert abs(r2.sum() - m0) < 1e-12 * m0
        mom1 = np.array([(r2 * u2[k]).sum() for k in range(d)])
        expect = mom0 + (m0 * np.array(g) if force else 0)
        assert np.abs(mom1 - expect).max() < 1e-13
        r, uu = r2, u2


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("omega", [1.0, 1.5, 1.99])
def test_uniform_state_is_fixed_point(q, omega):
    d = 2 if q == 9 else 3
    shape = (1, 4, 5) if q == 9 else (3, 4, 5)
    rho = np.full(shape, 1.013)
    u = np.zeros((d,) + shape)
    u[0], u[1] = 0.031, -0.047
    if d == 3:
        u[2] = 0.02
    nz, ny, nx = shape
    r1, u1 = oracle.step(oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=omega), rho, u)
    assert np.abs(r1 - rho).max() < 1e-15
    assert np.abs(u1 - u).max() < 1e-16


@pytest.mark.parametrize("q", [9, 19])
def test_mirror_symmetry(q):
    """Reflecting x -> -x maps the lattice to itself, so the step commutes
    with the reflection (u_x odd, other components even)."""
    d = 2 if q == 9 else 3
    shape = (1, 6, 8) if q == 9 else (4, 5, 6)
    drho, u = wl.random_state(shape, d, seed=5)
    rho = 1 + drho
    nz, ny, nx = shape
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=1.63)

    def mirror(r, uu):
        idx = (-np.arange(nx)) % nx
        r2 = r[..., idx]
        u2 = uu[..., idx].copy()
        u2[0] = -u2[0]
        return r2, u2

    a = mirror(*oracle.step(p, rho, u))
    b = oracle.step(p, *mirror(rho, u))
    assert np.abs(a[0] - b[0]).max() < 1e-15
    assert np.abs(a[1] - b[1]).max() < 1e-16


# ------------------------------------------------ closed-form solutions
@pytest.mark.parametrize("q,shape", [(9, (1, 32, 4)), (19, (4, 32, 4))])
def test_shear_wave_decays_exactly(q, shape):
    """rho = 1, u = (U(y),0,0) evolves exactly as U+ = U + nu (U_{y+1} - 2U + U_{y-1})
    for the full nonlinear update (any amplitude), so a sine decays as
    lambda^t with lambda = 1 - 4 nu sin^2(pi m / N) and nu from Eq. viscosity2."""
    d = 2 if q == 9 else 3
    omega, m, u0 = 1.7, 2, 0.08
    nz, ny, nx = shape
    drho, u = wl.shear_wave(shape, d, u0, m)
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=omega)
    nu = (1 / omega - 0.5) / 3
    lam = 1 - 4 * nu * np.sin(np.pi * m / ny) ** 2
    r, uu = oracle.run(p, 1 + drho, u, 50)
    assert np.abs(r - 1).max() < 1e-14
    assert np.abs(uu[0] - u[0] * lam ** 50).max() < 1e-15
    assert np.abs(uu[1:]).max() < 1e-14  # zero up to FP64 rounding of O(0.1) terms


def _channel_recurrence(ny_fluid, nu, g, steps, u_wall_top=0.0, U=None):
    """Brute-force linear recurrence U+ = U + nu (U_{y+1} - 2 U + U_{y-1}) + g on
    the fluid rows, with halfway bounce-back acting as the ghost values
    U_{-1} = -U_0 and U_N = 2 U_w - U_{N-1}."""
    U = np.zeros(ny_fluid) if U is None else U.copy()
    for _ in range(steps):
        ext = np.concatenate([[-U[0]], U, [2 * u_wall_top - U[-1]]])
        U = U + nu * (ext[2:] - 2 * ext[1:-1] + ext[:-2]) + g
    return U


@pytest.mark.parametrize("omega", [1.0, 1.6])
def test_channel_transient_matches_recurrence(omega):
    """Body-forced channel with halfway bounce-back walls (the 256x64
    workload, x-invariant so nx = 4 suffices): the state stays rho = 1,
    u_y = 0 and the profile follows the exact recurrence; after many steps
    it approaches U_inf(y) = g/(2 nu) (-y^2 + (N-1) y + N/2)."""
    nx, ny, g = 4, 64, 1e-6
    steps = 3000 if omega != 1.0 else 20000
    p = oracle.Problem(q=9, nx=nx, ny=ny, omega=omega, mask=wl.channel_mask(nx, ny),
                       g=(g, 0.0))
    r, u = oracle.run(p, np.ones((1, ny, nx)), np.zeros((2, 1, ny, nx)), steps)
    nu = (1 / omega - 0.5) / 3
    N = ny - 2
    U_ref = _channel_recurrence(N, nu, g, steps)
    fluid = slice(1, ny - 1)
    # exact in exact arithmetic; FP64 rounding accumulates ~1e-16 per step
    assert np.abs(r[0, fluid] - 1).max() < steps * 1e-16
    assert np.abs(u[1, 0, fluid]).max() < steps * 1e-18
    for x in range(nx):
        assert np.abs(u[0, 0, fluid, x] - U_ref).max() < 1e-10 * U_ref.max()
    if omega == 1.0:
        y = np.arange(N)
        U_inf = g / (2 * nu) * (-y ** 2 + (N - 1) * y + N / 2)
        rel = np.abs(u[0, 0, fluid, 0] - U_inf).max() / U_inf.max()
        assert 1.5e-4 < rel < 2.5e-4   # slowest mode lambda_1^20000 still present


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("omega", [1.2, 1.8])
def test_couette_linear_profile_is_exact(q, omega):
    """Top wall moving at U_w, bottom at rest, halfway bounce-back with the
    moving-wall term (2/omega - 1) 2 f^(e,o)(rho0, u_w) (Eq. ACM2.0ccccbb):
    U(y) = U_w (y + 1/2)/N is an exact steady state for every omega, and a
    start from rest follows the recurrence with ghost U_N = 2 U_w - U_{N-1}.
    A wrong wall factor would shift the effective wall speed."""
    d = 2 if q == 9 else 3
    Uw = 0.04
    nx, ny, nz = 3, 20, (1 if q == 9 else 3)
    if q == 9:
        mask = wl.channel_mask(nx, ny, moving_top=True)
    else:
        mask = wl.slab_mask_3d(nx, ny, nz, moving_top=True)
    p = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=omega, mask=mask,
                       wall_u=wl.wall_table((Uw, 0.0, 0.0)))
    N = ny - 2
    y = np.arange(N)
    rho = np.ones((nz, ny, nx))
    u = np.zeros((d, nz, ny, nx))
    u[0][:, 1:ny - 1, :] = (Uw * (y + 0.5) / N)[None, :, None]
    r1, u1 = oracle.run(p, rho, u, 10)
    # exact in exact arithmetic: only FP64 rounding remains
    assert np.abs(r1[:, 1:ny - 1] - 1).max() < 1e-14
    assert np.abs(u1[0][:, 1:ny - 1] - u[0][:, 1:ny - 1]).max() < 1e-14 * Uw
    assert np.abs(u1[1:]).max() < 1e-14
    # transient from rest
    nu = (1 / omega - 0.5) / 3
    r2, u2 = oracle.run(p, rho, np.zeros_like(u), 200)
    U_ref = _channel_recurrence(N, nu, 0.0, 200, u_wall_top=Uw)
    assert np.abs(u2[0][:, 1:ny - 1, :] - U_ref[None, :, None]).max() < 1e-12 * Uw
    assert np.abs(r2[:, 1:ny - 1] - 1).max() < 1e-13


def test_taylor_green_2d_decay_factor():
    """64x64 Taylor-Green vortex, u0 = 0.01, omega = 1.6, 1000 steps in FP64:
    the projected amplitude follows lambda^t with the discrete linear factor
    lambda = 1 - 8 nu sin^2(k/2) of the diagonal modes (k, k) to O(u0^2),
    mass is conserved exactly, and the deviation shrinks ~4x when u0 halves."""
    n, omega = 64, 1.6
    nu = (1 / omega - 0.5) / 3
    k = 2 * np.pi / n
    lam = 1 - 8 * nu * np.sin(k / 2) ** 2
    assert abs(lam - 0.999197454445) < 1e-12
    devs = []
    for u0 in (0.01, 0.005):
        drho, u = wl.taylor_green_2d(n, u0)
        p = oracle.Problem(q=9, nx=n, ny=n, omega=omega)
        m0 = (1 + drho).sum()
        r, uu = oracle.run(p, 1 + drho, u, 1000)
        amp = (uu * u).sum() / (u * u).sum()
        devs.append(abs(amp - lam ** 1000) / lam ** 1000)
        assert abs(r.sum() - m0) < 1e-12 * m0
        # continuum exp(-2 nu k^2 t) differs from the discrete factor by 3.2e-4
        assert abs(amp - np.exp(-2 * nu * k * k * 1000)) / amp < 1e-3
    assert devs[0] < 1e-4
    assert 3.0 < devs[0] / devs[1] < 5.0


def test_taylor_green_3d_linear_decay_factor():
    """D3Q19 Taylor-Green vortex (modes (+-k,+-k,+-k)) in the linear limit
    (u0 = 1e-5): amplitude follows lambda3^t with
    lambda3 = (9 omega + (2 - omega) cos 2k + (4 - 2 omega) cos k - 6)/(6 omega)."""
    n, omega, steps = 16, 1.7, 100
    k = 2 * np.pi / n
    lam3 = (9 * omega + (2 - omega) * np.cos(2 * k) + (4 - 2 * omega) * np.cos(k) - 6) / (6 * omega)
    drho, u = wl.taylor_green_3d(n, 1e-5)
    p = oracle.Problem(q=19, nx=n, ny=n, nz=n, omega=omega)
    r, uu = oracle.run(p, 1 + drho, u, steps)
    amp = (uu * u).sum() / (u * u).sum()
    assert abs(amp - lam3 ** steps) / lam3 ** steps < 1e-8


# ------------------------------------------------------- reverse mode
def _dot(a, b):
    return float((np.asarray(a) * np.asarray(b)).sum())


@pytest.mark.parametrize("case", ["d2q9_periodic", "d2q9_walls_force", "d3q19_periodic",
                                  "d3q19_walls"])
def test_vjp_matches_central_differences(case):
    """<lam, dF(s; ds)> from central differences equals <VJP(lam), ds>, for
    the state and for omega (the definition of the reverse mode)."""
    rng = np.random.Generator(np.random.PCG64(7))
    if case.startswith("d2q9"):
        q, d, shape = 9, 2, (1, 6, 5)
    else:
        q, d, shape = 19, 3, (4, 6, 5)
    nz, ny, nx = shape
    mask = wall_u = g = None
    if "walls" in case:
        mask = (wl.channel_mask(nx, ny, moving_top=True) if q == 9
                else wl.slab_mask_3d(nx, ny, nz, moving_top=True))
        wall_u = wl.wall_table((0.05, 0.0, 0.02))
    if "force" in case:
        g = (3e-3, -2e-3)
    omega = 1.37
    drho, u = wl.random_state(shape, d, seed=9, du=0.06, drho=0.03)
    rho = 1 + drho
    lam_r = rng.standard_normal(shape)
    lam_u = rng.standard_normal((d,) + shape)
    if mask is not None:
        lam_r[mask != 0] = 0
        lam_u[:, mask != 0] = 0

    def F(om, r, uu):
        return oracle.step(oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=om, mask=mask,
                                          wall_u=wall_u, g=g), r, uu)

    pr = oracle.Problem(q=q, nx=nx, ny=ny, nz=nz, omega=omega, mask=mask, wall_u=wall_u, g=g)
    gr, gu, gw = oracle.vjp(pr, rho, u, lam_r, lam_u)
    dr = rng.standard_normal(shape)
    du = rng.standard_normal((d,) + shape)
    h = 1e-6
    fp = F(omega, rho + h * dr, u + h * du)
    fm = F(omega, rho - h * dr, u - h * du)
    fd = (_dot(lam_r, fp[0] - fm[0]) + _dot(lam_u, fp[1] - fm[1])) / (2 * h)
    an = _dot(gr, dr) + _dot(gu, du)
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (fd, an)
    fp = F(omega + h, rho, u)
    fm = F(omega - h, rho, u)
    fdw = (_dot(lam_r, fp[0] - fm[0]) + _dot(lam_u, fp[1] - fm[1])) / (2 * h)
    assert abs(fdw - gw) < 1e-7 * max(1.0, abs(gw)), (fdw, gw)
    if mask is not None:
        assert np.all(gr[mask != 0] == 0)


def test_gradient_through_many_steps_matches_central_differences():
    """Final-state loss L = sum |u_T - u*|^2 after 200 steps on 32x32 (seeded
    divergence-free fields, k <= 2) with a checkpoint every 10 steps: the
    reverse sweep's dL/du0 and dL/domega equal central differences."""
    n, kmax, steps, K, omega = 32, 2, 200, 10, 1.6
    drho, u0 = wl.divergence_free_field(n, kmax, 0.01, seed=0)
    _, u_tgt = wl.divergence_free_field(n, kmax, 0.01, seed=1)
    p = oracle.Problem(q=9, nx=n, ny=n, omega=omega)

    def loss(om, uu0):
        _, uT = oracle.run(oracle.Problem(q=9, nx=n, ny=n, omega=om), 1 + drho, uu0, steps)
        return float(((uT - u_tgt) ** 2).sum())

    gr, gu, gw, _ = oracle.gradient(
        p, 1 + drho, u0, steps, lambda r, uu: (np.zeros_like(r), 2 * (uu - u_tgt)), K=K)
    rng = np.random.Generator(np.random.PCG64(2))
    for _ in range(2):
        du = rng.standard_normal(u0.shape)
        h = 1e-5
        fd = (loss(omega, u0 + h * du) - loss(omega, u0 - h * du)) / (2 * h)
        an = _dot(gu, du)
        assert abs(fd - an) < 1e-6 * abs(an), (fd, an)
    h = 1e-6
    fdw = (loss(omega + h, u0) - loss(omega - h, u0)) / (2 * h)
    assert abs(fdw - gw) < 1e-6 * abs(gw), (fdw, gw)


def test_oracle_rejects_unknown_lattice():
    with pytest.raises(ValueError):
        oracle.lattice_info(15)


# ------------------------------------- FP16 storage: stochastic rounding
def _half_neighbours(y):
    """The FP16 magnitudes lo <= |y| <= hi next to |y| (numpy's float16)."""
    a = abs(y)
    h = np.float16(a)                     # nearest, from numpy
    if float(h) > a:
        return float(np.nextafter(h, np.float16(0))), float(h)
    if float(h) < a:
        return float(h), float(np.nextafter(h, np.float16(np.inf)))
    return float(h), float(h)


def test_round_fp16_sr_threshold_convention():
    """|y| goes up when F + (r >> 19) >= 2^13, F the first 13 bits of its
    position between the two neighbouring halves, in the normal and the
    subnormal range alike."""
    y = 1.0 + 2.0 ** -10 * 3 / 8            # spacing 2^-10 at 1, position 3/8
    lo, hi = 1.0, 1.0 + 2.0 ** -10
    assert oracle.round_fp16_sr(y, (5119 << 19) | 0x7FFFF) == lo
    assert oracle.round_fp16_sr(y, 5120 << 19) == hi
    assert oracle.round_fp16_sr(-y, 5120 << 19) == -hi
    s = 2.0 ** -24                          # subnormal spacing, position 1/4
    assert oracle.round_fp16_sr(s / 4, ((3 << 22) - 1) << 8) == 0.0
    assert oracle.round_fp16_sr(s / 4, (3 << 22) << 8) == s
    # a position past 13 bits is cut: 1/4 + 2^-20 still needs r >> 19 >= 6144
    assert oracle.round_fp16_sr(s * (0.25 + 2.0 ** -20), (6143 << 19) | 0x7FFFF) == 0.0
    assert oracle.round_fp16_sr(s * (0.25 + 2.0 ** -20), 6144 << 19) == s
    # below the smallest subnormal: position m / 2^-24, cut to 13 bits
    assert oracle.round_fp16_sr(s * 2.0 ** -14, 0xFFFFFFFF) == 0.0
    assert oracle.round_fp16_sr(s * 2.0 ** -13, 0xFFFFFFFF) == s
    # the largest half is 65504, the next magnitude (65536) overflows
    assert oracle.round_fp16_sr(65510.0, 0) == 65504.0
    assert oracle.round_fp16_sr(65510.0, 0xFFFFFFFF) == np.inf
    # just under 2^-14 the rounding can step up into the normal range
    assert oracle.round_fp16_sr(2.0 ** -14 - s / 2, 0xFFFFFFFF) == 2.0 ** -14


def test_round_fp16_sr_lands_on_a_neighbour_and_keeps_halves():
    rng = np.random.Generator(np.random.PCG64(11))
    ys = np.concatenate([rng.uniform(-2, 2, 300) * 10.0 ** rng.integers(-9, 4, 300),
                         rng.uniform(-1, 1, 50) * 2.0 ** -14])
    for y in ys:
        lo, hi = _half_neighbours(y)
        for r in rng.integers(0, 2 ** 32, 4):
            got = oracle.round_fp16_sr(y, int(r))
            assert abs(got) in (lo, hi), (y, r, got)
            assert np.sign(got) in (0.0, np.sign(y))
    halves = rng.integers(0, 0x7C00, 400).astype(np.uint16).view(np.float16).astype(np.float64)
    for h in halves:
        for r in (0, 0xFFFFFFFF, int(rng.integers(0, 2 ** 32))):
            assert oracle.round_fp16_sr(h, r) == h
            assert oracle.round_fp16_sr(-h, r) == -h


def test_round_fp16_sr_is_unbiased():
    """Mean over uniform random words equals y (5 sigma), normal and subnormal."""
    rng = np.random.Generator(np.random.PCG64(12))
    words = rng.integers(0, 2 ** 32, 8192)
    for y in (0.3141592653589793, -1.0e-3 - 1e-9, 327.68 + 1.0 / 3, 3.0e-6, -7.1e-8, 2.0e-8):
        lo, hi = _half_neighbours(y)
        got = np.array([oracle.round_fp16_sr(y, int(r)) for r in words])
        f = (abs(y) - lo) / (hi - lo)
        sigma = (hi - lo) * np.sqrt(f * (1 - f) / len(words)) + 1e-300
        assert abs(got.mean() - y) < 5 * sigma + (hi - lo) * 2.0 ** -13, y


def test_sr_words_are_uniform_and_balanced():
    """The four field words of the nodes of a grid at three steps: the top 13
    bits of each (the bits the rounding reads) fill 64 bins evenly
    (chi-square), each of those bits is set half of the time, and the four
    fields of a node are uncorrelated."""
    m = 3 * 4096
    w = np.zeros((m, 4), dtype=np.uint32)
    k = 0
    for t in (1, 2, 1000):
        for idx in range(4096):
            w[k] = oracle.sr_words(idx, t)
            k += 1
    top = (w >> 19).astype(np.int64)        # 13-bit variates
    counts = np.stack([np.bincount(top[:, f] >> 7, minlength=64) for f in range(4)])
    expect = m / 64
    chi2 = ((counts - expect) ** 2 / expect).sum(axis=1)
    assert np.all(chi2 < 120), chi2        # 63 degrees of freedom: mean 63, sd 11
    ones = ((top[:, :, None] >> np.arange(13)) & 1).sum(axis=0)
    assert np.all(np.abs(ones - m / 2) < 5 * np.sqrt(m / 4)), ones
    c = np.corrcoef(top.T.astype(np.float64))
    assert np.all(np.abs(c[np.triu_indices(4, 1)]) < 5 / np.sqrt(m)), c


def test_fp16_storage_rounding_preserves_slow_decay():
    """A 128^2 Taylor-Green vortex at omega = 1.7 changes u by ~1e-6 per step,
    below one FP16 spacing (~1e-5 at u = 0.02).  Stored with round-to-nearest
    its kinetic energy stalls; stored with stochastic rounding (the oracle's
    own rounding) it decays as in FP64."""
    n, omega, steps = 128, 1.7, 1000
    drho, u = wl.taylor_green_2d(n, 0.02)
    p = oracle.Problem(q=9, nx=n, ny=n, omega=omega)
    rr, ru = oracle.run(p, 1 + drho, u, steps)
    e_ref = oracle.diagnostics(p, rr, ru)[1]

    def rne(a):
        return (a * 2.0 ** 14).astype(np.float16).astype(np.float64) / 2.0 ** 14

    r1, u1 = 1 + rne(drho), rne(u)
    r2, u2 = r1.copy(), u1.copy()
    for t in range(1, steps + 1):
        r1, u1 = oracle.step(p, r1, u1)
        r1, u1 = 1 + rne(r1 - 1), rne(u1)
        r2, u2 = oracle.step(p, r2, u2)
        r2, u2 = oracle.store_fp16_sr(p, t, r2, u2)
    e_rne = oracle.diagnostics(p, r1, u1)[1]
    e_sr = oracle.diagnostics(p, r2, u2)[1]
    e0 = oracle.diagnostics(p, 1 + drho, u)[1]
    assert e_ref < 0.9 * e0                          # the flow does decay
    assert abs(e_rne / e_ref - 1) > 1e-2             # nearest: stalls
    assert abs(e_sr / e_ref - 1) < 1e-3              # stochastic: tracks FP64
    assert np.linalg.norm(u2 - ru) / np.linalg.norm(ru) < 2e-3
