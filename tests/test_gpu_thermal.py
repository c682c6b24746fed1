"""The temperature lattice of the thermal LW-ACM (lwacm_set_thermal;
Eq. ACM2.0t with the even part of Eq. feqe) against the oracle's
thermal_step, run in lockstep with the flow.

- Random flow states, random T and walls of three kinds (two held at fixed
  temperatures, one adiabatic), D2Q9 and D3Q19, several steps: T on the fluid
  nodes to the FP32 bar; the flow is the oracle's as well.
- The 256^3 Taylor-Green flow with a random T field, one step on the full
  grid against the oracle at every node; the total of T over 20 steps
  conserved to FP32 rounding (periodic grid).
- Thermal Couette flow without heating: the exact linear profile between the
  two fixed-temperature walls stays steady.
- The temperature does not change the flow (bitwise equal to the same steps
  without it); scope: the two-step kernel declines it; with FP16 flow
  storage (T in FP32) each step against the oracle from the same inputs;
  switching it off is allowed.
- D3Q19 tile shapes run the temperature step inside the flow's single-step
  kernel, with and without walls: against the temperature kernel of its own
  (generic variant) and the oracle.
- A temperature lattice smaller than the flow's (D2Q5 under D2Q9, D3Q7 under
  D3Q19) against the oracle's, with and without walls; the lattice switched
  back to the flow's mid-run; scope of lwacm_set_thermal_lattice.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from gpu_helpers import banner, fluid_of, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu

MARCH, MARCH2 = 2, 3
WALL_T = [np.nan, 0.2, np.nan, 0.9]  # ids 1 and 3 fixed, id 2 adiabatic


def _walls(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 4, int(mask.sum())).astype(np.uint8)
    return mask


@pytest.mark.parametrize("q,masked,shape", [(9, False, (1, 40, 48)), (9, True, (1, 40, 48)),
                                             (19, False, (12, 32, 32)), (19, True, (40, 32, 64)),
                                             (19, True, (10, 20, 24))])
def test_random_fields_match_oracle(q, masked, shape):
    """D3Q19 shapes with nx % 32 == 0 and ny % 16 == 0 run the tile kernel
    (one z chunk, and two chunks with a tail); (10, 20, 24) the gather kernel."""
    L = need_gpu()
    banner(f"thermal random q={q} masked={masked} shape={shape}")
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=51, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(52))
    T = rng.uniform(0.2, 1.0, shape).astype(np.float32).astype(np.float64)
    mask = _walls(shape, 53) if masked else None
    table = np.zeros((4, 3))
    s = L.Solver(q, nx, ny, nz, 1.6, mask=None if mask is None else to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table])
    s.set_state(to_dev(drho), to_dev(u))
    s.set_thermal(1.3, to_dev(T), wall_T=WALL_T)
    steps = 6
    s.step(steps)
    Tg = s.temperature().double().cpu().numpy()
    dr, uu = s.moments()
    uu = uu.double().cpu().numpy()
    s.close()
    rho0 = 1.0 + (drho if mask is None else drho[mask == 0]).astype(np.float32).mean()
    p = oracle.Problem(q, nx, ny, nz, omega=1.6, mask=mask, wall_u=table, rho0=rho0)
    r, ru, rT = 1.0 + drho, u, T
    for _ in range(steps):
        rT = oracle.thermal_step(p, rT, ru, 1.3, wall_T=WALL_T)
        r, ru = oracle.step(p, r, ru)
    fl = fluid_of(mask, shape)
    err_T = rel_l2(Tg[fl], rT[fl])
    err_max = float(np.abs(Tg[fl] - rT[fl]).max())
    banner(f"thermal random: rel-L2 T {err_T:.3e}, max |dT| {err_max:.3e}, "
           f"rel-L2 u {rel_l2(uu[:, fl], ru[:, fl]):.3e}")
    assert err_T < 1e-6 and err_max < 1e-5
    assert rel_l2(uu[:, fl], ru[:, fl]) < 1e-5
    if mask is not None:
        assert np.array_equal(Tg[~fl], T[~fl])


@pytest.mark.parametrize("shape", [(40, 32, 64), (8, 16, 32)])
def test_fused_temperature_step_matches_the_separate_kernel(shape):
    """Unmasked D3Q19 tile shapes carry the temperature step inside the
    single-step flow kernel; the generic variant runs the temperature kernel
    of its own and the gather flow kernel.  Ten steps: T and u agree to FP32
    rounding (the sums run in another order), and T matches the oracle."""
    L = need_gpu()
    banner(f"thermal fused vs separate {shape}")
    nz, ny, nx = shape
    drho, u = wl.random_state(shape, 3, seed=61, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(62))
    T = rng.uniform(0.2, 1.0, shape).astype(np.float32).astype(np.float64)
    out = []
    for variant in (MARCH, 1):
        s = L.Solver(19, nx, ny, nz, 1.6, variant=variant)
        s.set_state(to_dev(drho), to_dev(u))
        s.set_thermal(1.3, to_dev(T))
        s.step(10)
        out.append((s.temperature().double().cpu().numpy(), s.moments()[1].double().cpu().numpy()))
        s.close()
    (Tf, uf), (Ts, us) = out
    e_T, e_u = rel_l2(Tf, Ts), rel_l2(uf, us)
    p = oracle.Problem(19, nx, ny, nz, omega=1.6)
    r, ru, rT = 1.0 + drho, u, T
    for _ in range(10):
        rT = oracle.thermal_step(p, rT, ru, 1.3)
        r, ru = oracle.step(p, r, ru)
    e_o = rel_l2(Tf, rT)
    banner(f"thermal fused vs separate: rel-L2 T {e_T:.3e}, u {e_u:.3e}; vs oracle T {e_o:.3e}")
    assert e_T < 1e-6 and e_u < 1e-6 and e_o < 1e-6


@pytest.mark.parametrize("shape", [(40, 32, 64), (16, 32, 64)])
def test_fused_temperature_with_walls_matches_the_separate_kernel(shape):
    """D3Q19 tile shapes with walls of three kinds (two fixed temperatures,
    one adiabatic) and a moving wall id: the temperature fused into the flow's
    single-step kernel (bounced temperature terms summed at push time, the
    fixed-temperature links from the table lwacm_set_thermal builds) against
    the generic variant's separate kernels and the oracle, 10 steps."""
    L = need_gpu()
    banner(f"thermal fused with walls {shape}")
    nz, ny, nx = shape
    drho, u = wl.random_state(shape, 3, seed=63, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(64))
    T = rng.uniform(0.2, 1.0, shape).astype(np.float32).astype(np.float64)
    mask = _walls(shape, 65)
    u[:, mask != 0] = 0.0
    table = np.zeros((4, 3))
    table[2] = (0.02, 0.0, -0.01)  # the adiabatic id moves
    out = []
    for variant in (0, 1):
        s = L.Solver(19, nx, ny, nz, 1.6, mask=to_dev(mask, torch.uint8),
                     wall_u=[list(r) for r in table], variant=variant)
        s.set_state(to_dev(drho), to_dev(u))
        s.set_thermal(1.3, to_dev(T), wall_T=WALL_T)
        s.step(10)
        out.append((s.temperature().double().cpu().numpy(), s.moments()[1].double().cpu().numpy()))
        s.close()
    (Tf, uf), (Ts, us) = out
    fl = mask == 0
    e_T, e_u = rel_l2(Tf[fl], Ts[fl]), rel_l2(uf[:, fl], us[:, fl])
    rho0 = 1.0 + drho[fl].astype(np.float32).mean()
    p = oracle.Problem(19, nx, ny, nz, omega=1.6, mask=mask, wall_u=table, rho0=rho0)
    r, ru, rT = 1.0 + drho, u, T
    for _ in range(10):
        rT = oracle.thermal_step(p, rT, ru, 1.3, wall_T=WALL_T)
        r, ru = oracle.step(p, r, ru)
    e_o = rel_l2(Tf[fl], rT[fl])
    banner(f"thermal fused with walls: rel-L2 T {e_T:.3e}, u {e_u:.3e}; vs oracle T {e_o:.3e}")
    assert e_T < 1e-6 and e_u < 1e-6 and e_o < 1e-6
    assert np.abs(Tf[fl] - rT[fl]).max() < 1e-5
    assert np.array_equal(Tf[~fl], T[~fl])


def test_full_size_step_matches_oracle_and_conserves_total():
    L = need_gpu()
    cfg = wl.TGV3D_256
    n = cfg.nx
    banner(f"thermal 256^3 one step vs oracle, then 20 steps total")
    drho, u = wl.taylor_green_3d(n, cfg.u0)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(54))
    T = rng.uniform(0.2, 1.0, (n, n, n)).astype(np.float32)
    s = L.Solver(19, n, n, n, cfg.omega)
    s.set_state(to_dev(drho), to_dev(u))
    s.set_thermal(1.4, to_dev(T))
    s.step(1)
    Tg = s.temperature().double().cpu().numpy()
    p = oracle.Problem(19, n, n, n, omega=cfg.omega)
    rT = oracle.thermal_step(p, T.astype(np.float64), u, 1.4)
    err_max = float(np.abs(Tg - rT).max())
    banner(f"thermal 256^3: max |dT| {err_max:.3e}")
    assert err_max < 1e-6
    total0 = float(T.astype(np.float64).sum())
    s.step(19)
    total = float(s.temperature().double().sum().item())
    s.close()
    banner(f"thermal 256^3: total T drift over 20 steps {abs(total / total0 - 1):.3e}")
    assert abs(total / total0 - 1.0) < 1e-6


@pytest.mark.parametrize("q", [9, 19])
def test_linear_profile_between_fixed_temperature_walls_stays(q):
    L = need_gpu()
    banner(f"thermal Couette q={q}")
    h, U, Tb, Tt = 18, 0.02, 1.0, 0.2
    ax = 1 if q == 9 else 2
    shape = (1, h, 64) if q == 9 else (h, 16, 64)
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    mask = np.zeros(shape, np.uint8)
    sl = [slice(None)] * 3
    sl[2 - ax] = 0
    mask[tuple(sl)] = 1
    sl[2 - ax] = h - 1
    mask[tuple(sl)] = 2
    coord = np.arange(h, dtype=float)
    bshape = [1, 1, 1]
    bshape[2 - ax] = h
    prof = (Tb + (Tt - Tb) * (coord - 0.5) / (h - 2.0)).reshape(bshape) * np.ones(shape)
    u = np.zeros((d,) + shape)
    u[0] = (U * (coord - 0.5) / (h - 2.0)).reshape(bshape)
    s = L.Solver(q, nx, ny, nz, 1.5, mask=to_dev(mask, torch.uint8),
                 wall_u=[[0, 0, 0], [0, 0, 0], [U, 0, 0]])
    s.set_state(to_dev(np.zeros(shape)), to_dev(u))
    s.set_thermal(1.5, to_dev(prof), wall_T=[np.nan, Tb, Tt])
    s.step(300)
    Tg = s.temperature().double().cpu().numpy()
    s.close()
    fl = mask == 0
    err = float(np.abs(Tg[fl] - prof[fl]).max() / abs(Tt - Tb))
    banner(f"thermal Couette: max error / dT {err:.3e}")
    assert err < 2e-5


def test_temperature_leaves_the_flow_alone_and_scope():
    L = need_gpu()
    banner("thermal scope")
    shape = (16, 32, 64)
    nz, ny, nx = shape
    drho, u = wl.random_state(shape, 3, seed=55, du=0.02, drho=0.01)
    ref = L.Solver(19, nx, ny, nz, 1.7, variant=MARCH)
    ref.set_state(to_dev(drho), to_dev(u))
    ref.step(5)
    r_ref = [t.cpu().numpy() for t in ref.moments()]
    ref.close()
    s = L.Solver(19, nx, ny, nz, 1.7)
    T0 = torch.rand(shape, device="cuda")
    s.set_thermal(1.2, T0)
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_set_variant(s.ctx, MARCH2)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    s.set_state(to_dev(drho), to_dev(u))
    s.step(5)
    r = [t.cpu().numpy() for t in s.moments()]
    assert all(np.array_equal(a, b) for a, b in zip(r, r_ref))
    s.set_thermal(1.0, None)
    with pytest.raises(L.LWACMError):
        s.temperature()
    L.lwacm_set_variant(s.ctx, MARCH2)
    s.close()


@pytest.mark.parametrize("q,qt,masked,shape", [(9, None, True, (1, 40, 48)),
                                                (19, None, False, (16, 32, 64)),
                                                (19, None, True, (16, 32, 64)),
                                                (19, 7, True, (10, 20, 24))])
def test_fp16_flow_storage_temperature_matches_oracle(q, qt, masked, shape):
    """FP16 flow storage with the temperature (T stays FP32): each of four
    steps against the oracle's temperature step from the same T and the
    flow velocity the GPU state holds (dequantized, as the kernels read it);
    the D3Q19 tile shapes run it fused into the FP16 flow kernel (stochastic
    rounding of the state), with and without walls."""
    L = need_gpu()
    banner(f"thermal with FP16 flow storage q={q} qt={qt} masked={masked} shape={shape}")
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=57, du=0.03, drho=0.01)
    rng = np.random.Generator(np.random.PCG64(58))
    T = rng.uniform(0.2, 1.0, shape).astype(np.float32)
    mask = _walls(shape, 59) if masked else None
    table = np.zeros((4, 3))
    s = L.Solver(q, nx, ny, nz, 1.6, storage=1,
                 mask=None if mask is None else to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table])
    s.set_state(to_dev(drho), to_dev(u))
    s.set_thermal(1.3, to_dev(T), wall_T=WALL_T, q_t=qt or 0)
    p = oracle.Problem(q, nx, ny, nz, omega=1.6, mask=mask, wall_u=table)
    worst = 0.0
    for _ in range(4):
        Tt = s.temperature().double().cpu().numpy()
        ut = s.moments()[1].double().cpu().numpy()
        s.step(1)
        got = s.temperature().double().cpu().numpy()
        ref = oracle.thermal_step(p, Tt, ut, 1.3, wall_T=WALL_T, qt=qt)
        worst = max(worst, rel_l2(got, ref))
        assert np.abs(got - ref).max() < 1e-5
    s.close()
    banner(f"thermal with FP16 flow storage: worst rel-L2 T {worst:.3e}")
    assert worst < 1e-6


@pytest.mark.parametrize("q,qt,masked,shape", [(9, 5, False, (1, 40, 48)), (9, 5, True, (1, 40, 48)),
                                                (19, 7, False, (12, 32, 32)),
                                                (19, 7, True, (40, 32, 64)),
                                                (19, 7, True, (10, 20, 24))])
def test_axis_temperature_lattice_matches_oracle(q, qt, masked, shape):
    """A temperature lattice smaller than the flow's (lwacm_set_thermal_lattice:
    D2Q5 under D2Q9, D3Q7 under D3Q19) on tile and other shapes, random flow,
    T and walls of three kinds, 6 steps in lockstep with the flow: T on the
    fluid nodes to the FP32 bar; solid nodes keep their T."""
    L = need_gpu()
    banner(f"thermal axis lattice q={q} qt={qt} masked={masked} shape={shape}")
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=71, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(72))
    T = rng.uniform(0.2, 1.0, shape).astype(np.float32).astype(np.float64)
    mask = _walls(shape, 73) if masked else None
    table = np.zeros((4, 3))
    s = L.Solver(q, nx, ny, nz, 1.6, mask=None if mask is None else to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table])
    s.set_state(to_dev(drho), to_dev(u))
    s.set_thermal(1.3, to_dev(T), wall_T=WALL_T, q_t=qt)
    steps = 6
    s.step(steps)
    Tg = s.temperature().double().cpu().numpy()
    s.close()
    rho0 = 1.0 + (drho if mask is None else drho[mask == 0]).astype(np.float32).mean()
    p = oracle.Problem(q, nx, ny, nz, omega=1.6, mask=mask, wall_u=table, rho0=rho0)
    r, ru, rT, rT_full = 1.0 + drho, u, T, T
    for _ in range(steps):
        rT = oracle.thermal_step(p, rT, ru, 1.3, wall_T=WALL_T, qt=qt)
        rT_full = oracle.thermal_step(p, rT_full, ru, 1.3, wall_T=WALL_T)
        r, ru = oracle.step(p, r, ru)
    fl = fluid_of(mask, shape)
    err_T = rel_l2(Tg[fl], rT[fl])
    err_max = float(np.abs(Tg[fl] - rT[fl]).max())
    diff_full = rel_l2(rT_full[fl], rT[fl])
    banner(f"thermal axis lattice: rel-L2 T {err_T:.3e}, max |dT| {err_max:.3e} "
           f"(the flow's lattice differs by {diff_full:.3e})")
    assert err_T < 1e-6 and err_max < 1e-5
    assert diff_full > 100 * err_T  # the test tells the two lattices apart
    if mask is not None:
        assert np.array_equal(Tg[~fl], T[~fl])


def test_thermal_lattice_scope():
    L = need_gpu()
    for q, bad in ((9, (7, 19, 3, 6)), (19, (5, 9, 3, 8))):
        shape = (1, 16, 32) if q == 9 else (8, 16, 32)
        s = L.Solver(q, shape[2], shape[1], shape[0], 1.6)
        for qt in bad:
            with pytest.raises(L.LWACMError):
                L.lwacm_set_thermal_lattice(s.ctx, qt)
        for qt in (0, q, 5 if q == 9 else 7):
            L.lwacm_set_thermal_lattice(s.ctx, qt)
        s.close()


def test_switching_the_temperature_lattice_back():
    """D3Q7 for three steps, then the flow's D3Q19 (fused into the flow's
    tile kernel) for three: the oracle run the same way."""
    L = need_gpu()
    shape = (16, 32, 64)
    nz, ny, nx = shape
    drho, u = wl.random_state(shape, 3, seed=75, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    T = np.random.Generator(np.random.PCG64(76)).uniform(0.2, 1.0, shape)
    T = T.astype(np.float32).astype(np.float64)
    s = L.Solver(19, nx, ny, nz, 1.6)
    s.set_state(to_dev(drho), to_dev(u))
    s.set_thermal(1.3, to_dev(T), q_t=7)
    s.step(3)
    L.lwacm_set_thermal_lattice(s.ctx, 0)
    s.step(3)
    Tg = s.temperature().double().cpu().numpy()
    s.close()
    p = oracle.Problem(19, nx, ny, nz, omega=1.6)
    r, ru, rT = 1.0 + drho, u, T
    for k in range(6):
        rT = oracle.thermal_step(p, rT, ru, 1.3, qt=7 if k < 3 else None)
        r, ru = oracle.step(p, r, ru)
    err = rel_l2(Tg, rT)
    banner(f"thermal lattice switched back: rel-L2 T {err:.3e}")
    assert err < 1e-6
