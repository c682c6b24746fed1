"""Parity of the D3Q19 z-marching tile kernel: against the FP64 oracle on
sizes with partial z chunks, a single plane (the z neighbours wrap onto the
node's own plane), FP16 storage, forcing and walls, and against the generic
one-thread-per-node kernel."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import banner, fluid_of, gpu_run, need_gpu, oracle_run, rel_l2, to_dev

pytestmark = pytest.mark.gpu

MARCH, GENERIC = 2, 1


@pytest.mark.parametrize("shape", [(40, 32, 64), (1, 16, 32), (3, 16, 32), (65, 48, 96)])
@pytest.mark.parametrize("storage", [0, 1])
def test_march_matches_oracle(shape, storage):
    banner(f"march {shape} storage={storage}")
    drho, u = wl.random_state(shape, 3, seed=13, du=0.04, drho=0.01)
    if storage:
        s16 = 2.0 ** 14
        drho = (drho * s16).astype(np.float16).astype(np.float64) / s16
        u = (u * s16).astype(np.float16).astype(np.float64) / s16
    steps = 10
    dr, uu, _ = gpu_run(19, shape, 1.62, drho, u, steps, storage=storage, variant=MARCH)
    rdr, ru = oracle_run(19, shape, 1.62, drho, u, steps)
    err = rel_l2(uu, ru)
    banner(f"march {shape} storage={storage}: rel-L2 u {err:.3e}")
    assert err < (1e-5 if storage == 0 else 1e-3)
    assert rel_l2(dr, rdr) < (1e-4 if storage == 0 else 2e-2)


@pytest.mark.parametrize("masked", [False, True])
def test_forced_problems_on_the_tile_kernel(masked):
    """A uniform body acceleration (Eq. force) on the single-step tile kernel:
    it enters each node's post-combine term (a rho u + rho g in one FMA)
    instead of every link term as in the generic kernel, so the two agree to
    FP32 rounding; both match the oracle.  The two-step kernel declines forcing,
    and so does the tile kernel below 8 planes."""
    L = need_gpu()
    shape = (20, 16, 32)
    banner(f"forced march masked={masked}")
    g = (1e-4, -2e-4, 5e-5)
    s = L.Solver(19, 32, 16, 20, 1.3, g=g)
    L.lwacm_set_variant(s.ctx, MARCH)
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_set_variant(s.ctx, 3)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    s.close()
    t = L.Solver(19, 32, 16, 7, 1.3, g=g)
    with pytest.raises(L.LWACMError):
        L.lwacm_set_variant(t.ctx, MARCH)
    t.close()
    mask = None
    if masked:
        mask = np.zeros(shape, dtype=np.uint8)
        mask[:, 0] = 1
        mask[:, -1] = 1
    drho, u = wl.random_state(shape, 3, seed=14, du=0.03, drho=0.01)
    dr, uu, _ = gpu_run(19, shape, 1.3, drho, u, 20, g=g, mask=mask, variant=MARCH)
    dg, ug, _ = gpu_run(19, shape, 1.3, drho, u, 20, g=g, mask=mask, variant=GENERIC)
    rho0 = 1.0 if mask is None else 1.0 + drho.astype(np.float32)[mask == 0].mean()
    rdr, ru = oracle_run(19, shape, 1.3, drho.astype(np.float32).astype(np.float64),
                         u.astype(np.float32).astype(np.float64), 20, g=g, mask=mask, rho0=rho0)
    fl = fluid_of(mask, shape)
    assert rel_l2(uu[:, fl], ru[:, fl]) < 1e-5
    assert rel_l2(uu[:, fl], ug[:, fl]) < 1e-6


@pytest.mark.parametrize("n", [32, 64])
def test_march_masked_cavity_matches_oracle(n):
    """Lid-driven cube with the march kernel's bounce-back path."""
    banner(f"march cavity {n}")
    mask = wl.cavity_mask(n)
    table = wl.wall_table((0.05, 0.0, 0.0))
    shape = (n, n, n)
    drho, u = np.zeros(shape), np.zeros((3,) + shape)
    steps = 150
    dr, uu, s = gpu_run(19, shape, 1.9, drho, u, steps, mask=mask, wall_u=table, variant=MARCH)
    rdr, ru = oracle_run(19, shape, 1.9, drho, u, steps, mask=mask, wall_u=table)
    fl = fluid_of(mask, shape)
    err = rel_l2(uu[:, fl], ru[:, fl])
    banner(f"march cavity {n}: rel-L2 u {err:.3e}")
    assert err < 1e-5
    m, _ = s.diagnostics()
    nf = int(fl.sum())
    assert abs(m - nf) / nf < 1e-9
    # solid nodes keep their state
    assert np.all(uu[:, ~fl] == 0) and np.all(dr[~fl] == 0)


def test_march_random_walls_with_moving_ids():
    """Scattered solid nodes with two moving wall ids and random state."""
    shape = (12, 32, 32)
    banner("march random walls")
    rng = np.random.Generator(np.random.PCG64(8))
    mask = (rng.random(shape) < 0.08).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 4, int(mask.sum())).astype(np.uint8)
    table = np.array([[0, 0, 0], [0, 0, 0], [0.03, -0.01, 0.02], [-0.02, 0.0, 0.01]])
    drho, u = wl.random_state(shape, 3, seed=9, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    rho0 = 1.0 + drho[mask == 0].mean()
    dr, uu, _ = gpu_run(19, shape, 1.5, drho, u, 8, mask=mask, wall_u=table, variant=MARCH)
    rdr, ru = oracle_run(19, shape, 1.5, drho, u, 8, mask=mask, wall_u=table, rho0=rho0)
    fl = fluid_of(mask, shape)
    assert rel_l2(uu[:, fl], ru[:, fl]) < 1e-5
    dg, ug, _ = gpu_run(19, shape, 1.5, drho, u, 8, mask=mask, wall_u=table, variant=GENERIC)
    assert rel_l2(uu[:, fl], ug[:, fl]) < 1e-6


def test_march_close_to_generic_and_deterministic():
    shape = (64, 32, 64)
    banner("march vs generic")
    drho, u = wl.taylor_green_3d(64, 0.02)
    drho = drho[:, :32, :]
    u = u[:, :, :32, :]
    a = gpu_run(19, shape, 1.7, drho, u, 50, variant=MARCH)
    b = gpu_run(19, shape, 1.7, drho, u, 50, variant=GENERIC)
    c = gpu_run(19, shape, 1.7, drho, u, 50, variant=MARCH)
    assert rel_l2(a[1], b[1]) < 1e-6
    assert np.array_equal(a[1], c[1]) and np.array_equal(a[0], c[0])
    assert a[2].diagnostics() == c[2].diagnostics()


def test_march_rejects_unsupported_shape():
    L = need_gpu()
    banner("march unsupported")
    s = L.Solver(19, 48, 48, 48, 1.5)
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_set_variant(s.ctx, MARCH)
    assert ei.value.code == L.LWACM_EUNSUPPORTED


@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("storage", [0, 1])
def test_march_chunk_depths_agree_bitwise(masked, storage):
    """Every chunk depth of the tile kernel (32, 64, 128 planes per workgroup)
    on a grid that is ragged for all of them (150 planes) gives bitwise the
    same fields; depth 128 also matches the oracle."""
    L = need_gpu()
    shape = (150, 32, 64)
    nz, ny, nx = shape
    banner(f"march chunk depths masked={masked} storage={storage}")
    drho, u = wl.random_state(shape, 3, seed=21, du=0.03, drho=0.01)
    mask = wall = None
    if masked:
        mask = np.zeros(shape, dtype=np.uint8)
        mask[0], mask[:, 0], mask[:, :, 0] = 1, 1, 1
        mask[-1] = 2
        wall = wl.wall_table((0.04, 0.01, 0.0))
    outs = []
    for planes in (32, 64, 128):
        s = L.Solver(19, nx, ny, nz, 1.7, storage=storage, variant=MARCH,
                     mask=None if mask is None else to_dev(mask, torch.uint8),
                     wall_u=None if wall is None else [list(r) for r in wall])
        L.lwacm_set_march_chunk(s.ctx, planes)
        s.set_state(to_dev(drho), to_dev(u))
        s.step(5)
        dr, uu = s.moments()
        outs.append((dr.cpu().numpy(), uu.cpu().numpy()))
        s.close()
    for dr, uu in outs[1:]:
        assert np.array_equal(dr, outs[0][0]) and np.array_equal(uu, outs[0][1])
    if storage == 0:
        rdr, ru = oracle_run(19, shape, 1.7, drho.astype(np.float32).astype(np.float64),
                             u.astype(np.float32).astype(np.float64), 5, mask=mask, wall_u=wall,
                             rho0=1.0 if mask is None else
                             1.0 + drho[mask == 0].astype(np.float32).astype(np.float64).mean())
        fl = fluid_of(mask, shape)
        err = rel_l2(outs[2][1].astype(np.float64)[:, fl], ru[:, fl])
        banner(f"chunk 128 vs oracle: rel-L2 u {err:.3e}")
        assert err < 1e-5


def test_march_chunk_rejects_bad_depth():
    L = need_gpu()
    s = L.Solver(19, 32, 16, 8, 1.7)
    with pytest.raises(L.LWACMError):
        L.lwacm_set_march_chunk(s.ctx, 48)
    s.close()
    s = L.Solver(19, 20, 16, 8, 1.7)   # nx not a multiple of 32: no tile kernel
    with pytest.raises(L.LWACMError):
        L.lwacm_set_march_chunk(s.ctx, 64)
    s.close()


def test_march_256_cubed_repeat_runs_bitwise_equal():
    """Regression: at 256^3 every chunk depth gives bitwise the same fields
    run after run over 200 steps, and so does the reverse kernel over 40
    chained steps.  (Without wait states after the tile kernel's buffer
    stores, the last plane of a chunk picked up the next instruction's
    register values in a few lanes, intermittently.)"""
    L = need_gpu()
    n = 256
    banner("256^3 repeat-run determinism")
    drho, u = wl.taylor_green_3d(n, 0.02)
    d0, u0 = to_dev(drho), to_dev(u)

    def fwd(planes):
        s = L.Solver(19, n, n, n, 1.7, variant=MARCH)
        L.lwacm_set_march_chunk(s.ctx, planes)
        s.set_state(d0, u0)
        s.step(200)
        dr, uu = s.moments()
        s.close()
        return dr, uu

    ref = fwd(128)
    assert bool(torch.isfinite(ref[1]).all())
    for planes in (128, 64, 32):
        dr, uu = fwd(planes)
        assert torch.equal(dr, ref[0]) and torch.equal(uu, ref[1]), planes

    s = L.Solver(19, n, n, n, 1.7)
    s.set_state(d0, u0)
    s.step(2)
    st = s.save_state()
    lam = torch.zeros((4, n, n, n), device="cuda")
    lam[1:] = u0

    def rev():
        a = torch.zeros_like(lam)
        b = torch.zeros_like(lam)
        dw = torch.zeros(1, dtype=torch.float64, device="cuda")
        L.lwacm_adjoint_seed(s.ctx, st, lam, a)
        for _ in range(20):
            L.lwacm_adjoint_step(s.ctx, st, a, b, dw, False)
            L.lwacm_adjoint_step(s.ctx, st, b, a, dw, False)
        return a.clone(), float(dw.item())

    (ra, wa), (rb, wb) = rev(), rev()
    s.close()
    assert torch.equal(ra, rb) and wa == wb and bool(torch.isfinite(ra).all())
