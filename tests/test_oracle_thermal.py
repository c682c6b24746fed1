"""Pins of the oracle's thermal LW-ACM (Appendix "Asymptotic analysis for
energy equation", Eqs. ACM2.0t, feqe, AAT2 and diffusivity2).

- The equilibrium has the moments the appendix requires (T, T u and
  u u + T/3 I); its even part is even in u and keeps the even moments.
- A Fourier mode in a uniform flow on a periodic grid is multiplied every step
  by the amplification factor obtained by inserting e^{i k.x} into Eq.
  ACM2.0t by hand:  lambda(k) = kap + sum_i w_i (1 + 3 v_i.u - kap) e^{-i k.v_i},
  kap = 2 - 2/omega_t (the u-only terms of g^(e) and g^(e,e) cancel for a
  uniform u).  Exact to rounding.
- Long waves diffuse with the paper's alpha = (1/3)(1/omega_t - 1/2)
  (Eq. diffusivity2) and travel with the flow velocity (Eq. AAT2).
- The sum of T over the fluid nodes is conserved on a periodic grid and with
  adiabatic walls, for any flow field.
- Between two walls held at fixed temperatures (the halfway reading: the wall
  sits halfway between the last fluid and the first solid layer) the steady
  state is the exact linear profile, at rest and in plane Couette flow (the
  thermal Couette problem without viscous heating, Br = 0); a uniform
  initial state converges to it.
- A temperature lattice smaller than the flow's (Q_t != Q, which the
  appendix allows): D2Q5 under D2Q9, D3Q7 under D3Q19.  The lattice is the
  rest link and the axis links with weights fixed by the required moments
  (axis 1/6 from T/3 I, the rest the remainder: 1/3 and 0); its equilibrium
  has the moments T, T u and T/3 I exactly and no u u part (those lattices
  cannot carry it; it is O(eps^2) under the diffusive scaling).  The same
  Fourier amplification factor with these weights, the paper's alpha, the
  conservation and the linear-profile pins hold on them.
- The reverse mode of the temperature step (not in the paper: its exact
  derivative) against central differences of the step, on every input
  component of small grids, with and without walls, on all four lattices.
"""
import numpy as np
import pytest

import oracle
from oracle import Problem


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    d, v, w, _ = oracle.lattice_info(q)
    rng = _rng(1)
    for _ in range(5):
        T = rng.uniform(0.2, 1.0)
        u = rng.uniform(-0.1, 0.1, d)
        u3 = np.zeros(3)
        u3[:d] = u
        g, ge = oracle.thermal_equilibrium(q, T, u)
        vv = np.einsum("ia,ib->iab", v, v)
        pi = np.outer(u3, u3) + T / 3.0 * np.diag([1.0] * d + [0.0] * (3 - d))
        assert abs(g.sum() - T) < 1e-15
        assert np.abs(v.T @ g - T * u3).max() < 1e-15
        assert np.abs(np.einsum("iab,i->ab", vv, g) - pi).max() < 1e-15
        assert abs(ge.sum() - T) < 1e-15
        assert np.abs(v.T @ ge).max() < 1e-15
        assert np.abs(np.einsum("iab,i->ab", vv, ge) - pi).max() < 1e-15
        assert np.array_equal(ge, oracle.thermal_equilibrium(q, T, -u)[1])
        assert np.abs(ge - 0.5 * (g + oracle.thermal_equilibrium(q, T, -u)[0])).max() < 1e-16


def _mode_run(q, shape, kvec, u, omega_t, steps, T0=0.5, A=0.1):
    d, v, w, _ = oracle.lattice_info(q)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = kvec[0] * x + kvec[1] * y + kvec[2] * z
    T = T0 + A * np.cos(phase)
    uf = np.zeros((d,) + shape)
    for a in range(d):
        uf[a] = u[a]
    p = Problem(q, nx, ny, nz)
    for _ in range(steps):
        T = oracle.thermal_step(p, T, uf, omega_t)
    return T, phase, T0, A


@pytest.mark.parametrize("q,shape,kvec,u,omega_t", [
    (9, (1, 16, 24), (2 * np.pi * 3 / 24, 2 * np.pi / 16, 0.0), (0.04, -0.03), 1.3),
    (9, (1, 12, 12), (2 * np.pi * 2 / 12, 2 * np.pi * 5 / 12, 0.0), (0.0, 0.1), 0.7),
    (19, (8, 12, 10), (2 * np.pi / 10, 2 * np.pi * 2 / 12, 2 * np.pi * 3 / 8), (0.03, 0.02, -0.05),
     1.6),
])
def test_fourier_mode_in_uniform_flow(q, shape, kvec, u, omega_t):
    d, v, w, _ = oracle.lattice_info(q)
    kap = 2.0 - 2.0 / omega_t
    k3 = np.array(kvec)
    u3 = np.zeros(3)
    u3[:d] = u
    lam = kap + sum(w[i] * (1.0 + 3.0 * (v[i] @ u3) - kap) * np.exp(-1j * (k3 @ v[i]))
                    for i in range(q))
    steps = 15
    T, phase, T0, A = _mode_run(q, shape, kvec, u, omega_t, steps)
    exact = T0 + A * np.real(lam ** steps * np.exp(1j * phase))
    assert np.abs(T - exact).max() < 1e-13


def test_long_wave_diffuses_with_alpha_and_moves_with_u():
    """D2Q9, a wave of length 128: at rest its decay rate / k^2 is alpha of
    Eq. diffusivity2 to O(k^2); in a flow along it the phase speed is u, and
    the decay rate departs from alpha by O(u^2) only (the O(eps^2) of Eq.
    AAT2 under diffusive scaling, u = O(eps))."""
    n, steps = 128, 400
    kx = 2 * np.pi / n
    for omega_t, ux in [(1.2, 0.0), (1.8, 0.0), (0.8, 0.0), (1.2, 0.02), (1.8, 0.05)]:
        T, phase, T0, A = _mode_run(9, (1, 2, n), (kx, 0.0, 0.0), (ux, 0.0), omega_t, steps)
        amp = 2.0 / T[0, 0].size * np.sum((T[0, 0] - T0) * np.exp(-1j * phase[0, 0])) / A
        alpha = (1.0 / omega_t - 0.5) / 3.0
        alpha_meas = -np.log(abs(amp)) / (kx * kx * steps)
        if ux == 0.0:
            assert abs(alpha_meas / alpha - 1.0) < 5e-3, (omega_t, alpha_meas, alpha)
            assert abs(np.angle(amp)) < 1e-12
        else:
            assert abs(alpha_meas - alpha) < ux * ux, (omega_t, alpha_meas, alpha)
            speed = -np.angle(amp) / (kx * steps)
            assert abs(speed / ux - 1.0) < 5e-3, (omega_t, speed, ux)


@pytest.mark.parametrize("q,shape", [(9, (1, 18, 20)), (19, (8, 10, 12))])
def test_total_temperature_is_conserved(q, shape):
    d = 2 if q == 9 else 3
    nz, ny, nx = shape
    rng = _rng(2)
    T = rng.uniform(0.3, 1.0, shape)
    u = 0.05 * rng.standard_normal((d,) + shape)
    mask = (rng.random(shape) < 0.12).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 4, int(mask.sum())).astype(np.uint8)
    for m in (None, mask):
        p = Problem(q, nx, ny, nz, mask=m)
        fl = np.ones(shape, bool) if m is None else (m == 0)
        total0 = T[fl].sum()
        t = T
        for _ in range(20):
            t = oracle.thermal_step(p, t, u, 1.4)  # all walls adiabatic
        assert abs(t[fl].sum() / total0 - 1.0) < 1e-13
        if m is not None:
            assert np.array_equal(t[~fl], T[~fl])


def _channel(q, h, Tb, Tt, U, omega_t, steps, start_exact):
    d, v, w, _ = oracle.lattice_info(q)
    ax = 1 if q == 9 else 2
    shape = (1, h, 4) if q == 9 else (h, 4, 4)
    nz, ny, nx = shape
    mask = np.zeros(shape, np.uint8)
    sl = [slice(None)] * 3
    sl[2 - ax] = 0
    mask[tuple(sl)] = 1
    sl[2 - ax] = h - 1
    mask[tuple(sl)] = 2
    coord = np.arange(h, dtype=float)
    # walls halfway between the last fluid and the first solid layer
    exact = Tb + (Tt - Tb) * (coord - 0.5) / (h - 2.0)
    bshape = [1, 1, 1]
    bshape[2 - ax] = h
    prof = exact.reshape(bshape) * np.ones(shape)
    u = np.zeros((d,) + shape)
    u[0] = (U * (coord - 0.5) / (h - 2.0)).reshape(bshape)
    T = prof.copy() if start_exact else np.full(shape, 0.5 * (Tb + Tt))
    p = Problem(q, nx, ny, nz, mask=mask)
    for _ in range(steps):
        T = oracle.thermal_step(p, T, u, omega_t, wall_T=[np.nan, Tb, Tt])
    fl = mask == 0
    return float(np.abs(T[fl] - prof[fl]).max() / abs(Tt - Tb))


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("U", [0.0, 0.05])
@pytest.mark.parametrize("omega_t", [0.9, 1.5])
def test_linear_profile_between_fixed_temperature_walls_is_steady(q, U, omega_t):
    assert _channel(q, 10, 1.0, 0.2, U, omega_t, 40, True) < 1e-13


@pytest.mark.parametrize("q", [9, 19])
def test_thermal_couette_without_heating_converges_to_linear_profile(q):
    assert _channel(q, 10, 1.0, 0.2, 0.05, 1.5, 1500, False) < 1e-9


# ---- temperature lattices smaller than the flow's (Q_t != Q)

# The rest link and the axis links; axis weight 1/6 (second moment T/3 I),
# rest weight 1 - 2 D / 6.
def _axis_lattice(qt):
    d = 2 if qt == 5 else 3
    v = [np.zeros(3, int)]
    for a in range(d):
        for sgn in (1, -1):
            e = np.zeros(3, int)
            e[a] = sgn
            v.append(e)
    w = [1.0 - 2 * d / 6.0] + [1.0 / 6.0] * (2 * d)
    return d, np.array(v), np.array(w)


def _flow_q(qt):
    return 9 if qt == 5 else 19


@pytest.mark.parametrize("qt", [5, 7])
def test_axis_lattice_is_rest_and_axis_links_with_moment_weights(qt):
    d, v, w = _axis_lattice(qt)
    do, vo, wo, opp = oracle.lattice_info(qt)
    assert do == d
    assert sorted(map(tuple, vo)) == sorted(map(tuple, v))
    for i in range(qt):
        j = [k for k in range(qt) if tuple(v[k]) == tuple(vo[i])][0]
        assert abs(wo[i] - w[j]) < 1e-15
        assert tuple(vo[opp[i]]) == tuple(-vo[i])


@pytest.mark.parametrize("qt", [5, 7])
def test_axis_lattice_equilibrium_moments(qt):
    d, v, w, _ = oracle.lattice_info(qt)
    rng = _rng(3)
    eye = np.diag([1.0] * d + [0.0] * (3 - d))
    vv = np.einsum("ia,ib->iab", v, v)
    for _ in range(5):
        T = rng.uniform(0.2, 1.0)
        u = rng.uniform(-0.1, 0.1, d)
        u3 = np.zeros(3)
        u3[:d] = u
        g, ge = oracle.thermal_equilibrium(qt, T, u)
        assert abs(g.sum() - T) < 1e-15
        assert np.abs(v.T @ g - T * u3).max() < 1e-15
        assert np.abs(np.einsum("iab,i->ab", vv, g) - T / 3.0 * eye).max() < 1e-15
        assert abs(ge.sum() - T) < 1e-15
        assert np.abs(v.T @ ge).max() < 1e-15
        assert np.abs(np.einsum("iab,i->ab", vv, ge) - T / 3.0 * eye).max() < 1e-15
        assert np.abs(ge - 0.5 * (g + oracle.thermal_equilibrium(qt, T, -u)[0])).max() < 1e-16


@pytest.mark.parametrize("qt,shape,kvec,u,omega_t", [
    (5, (1, 16, 24), (2 * np.pi * 3 / 24, 2 * np.pi / 16, 0.0), (0.04, -0.03), 1.3),
    (5, (1, 12, 12), (2 * np.pi * 2 / 12, 2 * np.pi * 5 / 12, 0.0), (0.0, 0.1), 0.7),
    (7, (8, 12, 10), (2 * np.pi / 10, 2 * np.pi * 2 / 12, 2 * np.pi * 3 / 8), (0.03, 0.02, -0.05),
     1.6),
])
def test_axis_lattice_fourier_mode_in_uniform_flow(qt, shape, kvec, u, omega_t):
    d, v, w = _axis_lattice(qt)
    kap = 2.0 - 2.0 / omega_t
    k3 = np.array(kvec)
    u3 = np.zeros(3)
    u3[:d] = u
    lam = kap + sum(w[i] * (1.0 + 3.0 * (v[i] @ u3) - kap) * np.exp(-1j * (k3 @ v[i]))
                    for i in range(qt))
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = k3[0] * x + k3[1] * y + k3[2] * z
    T = 0.5 + 0.1 * np.cos(phase)
    uf = np.zeros((d,) + shape)
    for a in range(d):
        uf[a] = u[a]
    p = Problem(_flow_q(qt), nx, ny, nz)
    steps = 15
    for _ in range(steps):
        T = oracle.thermal_step(p, T, uf, omega_t, qt=qt)
    exact = 0.5 + 0.1 * np.real(lam ** steps * np.exp(1j * phase))
    assert np.abs(T - exact).max() < 1e-13


@pytest.mark.parametrize("qt,shape", [(5, (1, 2, 128)), (7, (2, 2, 128))])
def test_axis_lattice_long_wave_diffuses_with_alpha(qt, shape):
    n, steps = shape[2], 400
    kx = 2 * np.pi / n
    x = np.arange(n)
    for omega_t in (1.2, 1.8, 0.8):
        T = 0.5 + 0.1 * np.cos(kx * x) * np.ones(shape)
        u = np.zeros((2 if qt == 5 else 3,) + shape)
        p = Problem(_flow_q(qt), shape[2], shape[1], shape[0])
        for _ in range(steps):
            T = oracle.thermal_step(p, T, u, omega_t, qt=qt)
        amp = 2.0 / n * np.sum((T[0, 0] - 0.5) * np.exp(-1j * kx * x)) / 0.1
        alpha = (1.0 / omega_t - 0.5) / 3.0
        alpha_meas = -np.log(abs(amp)) / (kx * kx * steps)
        assert abs(alpha_meas / alpha - 1.0) < 5e-3, (omega_t, alpha_meas, alpha)


@pytest.mark.parametrize("qt,shape", [(5, (1, 18, 20)), (7, (8, 10, 12))])
def test_axis_lattice_total_temperature_is_conserved(qt, shape):
    d = 2 if qt == 5 else 3
    nz, ny, nx = shape
    rng = _rng(4)
    T = rng.uniform(0.3, 1.0, shape)
    u = 0.05 * rng.standard_normal((d,) + shape)
    mask = (rng.random(shape) < 0.12).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 4, int(mask.sum())).astype(np.uint8)
    for m in (None, mask):
        p = Problem(_flow_q(qt), nx, ny, nz, mask=m)
        fl = np.ones(shape, bool) if m is None else (m == 0)
        total0 = T[fl].sum()
        t = T
        for _ in range(20):
            t = oracle.thermal_step(p, t, u, 1.4, qt=qt)
        assert abs(t[fl].sum() / total0 - 1.0) < 1e-13
        if m is not None:
            assert np.array_equal(t[~fl], T[~fl])


def _channel_qt(qt, h, Tb, Tt, U, omega_t, steps, start_exact):
    q = _flow_q(qt)
    d = 2 if q == 9 else 3
    ax = 1 if q == 9 else 2
    shape = (1, h, 4) if q == 9 else (h, 4, 4)
    nz, ny, nx = shape
    mask = np.zeros(shape, np.uint8)
    sl = [slice(None)] * 3
    sl[2 - ax] = 0
    mask[tuple(sl)] = 1
    sl[2 - ax] = h - 1
    mask[tuple(sl)] = 2
    coord = np.arange(h, dtype=float)
    exact = Tb + (Tt - Tb) * (coord - 0.5) / (h - 2.0)
    bshape = [1, 1, 1]
    bshape[2 - ax] = h
    prof = exact.reshape(bshape) * np.ones(shape)
    u = np.zeros((d,) + shape)
    u[0] = (U * (coord - 0.5) / (h - 2.0)).reshape(bshape)
    T = prof.copy() if start_exact else np.full(shape, 0.5 * (Tb + Tt))
    p = Problem(q, nx, ny, nz, mask=mask)
    for _ in range(steps):
        T = oracle.thermal_step(p, T, u, omega_t, wall_T=[np.nan, Tb, Tt], qt=qt)
    fl = mask == 0
    return float(np.abs(T[fl] - prof[fl]).max() / abs(Tt - Tb))


@pytest.mark.parametrize("qt", [5, 7])
@pytest.mark.parametrize("U", [0.0, 0.05])
@pytest.mark.parametrize("omega_t", [0.9, 1.5])
def test_axis_lattice_linear_profile_is_steady(qt, U, omega_t):
    assert _channel_qt(qt, 10, 1.0, 0.2, U, omega_t, 40, True) < 1e-13


@pytest.mark.parametrize("qt", [5, 7])
def test_axis_lattice_converges_to_linear_profile(qt):
    assert _channel_qt(qt, 10, 1.0, 0.2, 0.05, 1.5, 1500, False) < 1e-9


def test_temperature_lattice_must_fit_the_flow():
    p = Problem(9, 8, 8, 1)
    T = np.ones((1, 8, 8))
    u = np.zeros((2, 1, 8, 8))
    for qt in (7, 19, 6):
        with pytest.raises(ValueError):
            oracle.thermal_step(p, T, u, 1.3, qt=qt)


# ---- reverse mode of the temperature step (not in the paper: the exact
# derivative of thermal_step), pinned by central differences of the step
# itself.  The step is linear in T and a polynomial of degree two in u for
# fixed T, so central differences are exact up to rounding.

@pytest.mark.parametrize("q,qt,shape", [(9, None, (1, 5, 6)), (9, 5, (1, 5, 6)),
                                        (19, None, (3, 4, 5)), (19, 7, (3, 4, 5))])
@pytest.mark.parametrize("walls", [False, True])
def test_thermal_vjp_matches_central_differences(q, qt, shape, walls):
    d = 2 if q == 9 else 3
    nz, ny, nx = shape
    rng = _rng(11)
    T = rng.uniform(0.3, 1.0, shape)
    u = 0.08 * rng.standard_normal((d,) + shape)
    lam = rng.standard_normal(shape)
    mask = None
    if walls:
        mask = (rng.random(shape) < 0.2).astype(np.uint8)
        mask[mask == 1] = rng.integers(1, 4, int(mask.sum())).astype(np.uint8)
    wall_T = [np.nan, 0.25, np.nan, 0.8]
    p = Problem(q, nx, ny, nz, mask=mask)
    omega_t = 1.35

    def loss(Tv, uv):
        return float(np.sum(lam * oracle.thermal_step(p, Tv, uv, omega_t, wall_T=wall_T, qt=qt)))

    lt, lu = oracle.thermal_vjp(p, T, u, lam, omega_t, wall_T=wall_T, qt=qt)
    eps = 1e-3
    fd_T = np.zeros(shape)
    fd_u = np.zeros((d,) + shape)
    for j in np.ndindex(shape):
        Tp, Tm = T.copy(), T.copy()
        Tp[j] += eps
        Tm[j] -= eps
        fd_T[j] = (loss(Tp, u) - loss(Tm, u)) / (2 * eps)
        for c in range(d):
            up, um = u.copy(), u.copy()
            up[(c,) + j] += eps
            um[(c,) + j] -= eps
            fd_u[(c,) + j] = (loss(T, up) - loss(T, um)) / (2 * eps)
    scale = np.abs(lam).max()
    assert np.abs(lt - fd_T).max() < 1e-11 * scale
    assert np.abs(lu - fd_u).max() < 1e-11 * scale
    if mask is not None:
        assert np.array_equal(lt[mask != 0], lam[mask != 0])
        assert not lu[:, mask != 0].any()
