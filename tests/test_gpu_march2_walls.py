"""Two forward steps per launch with halfway walls (LWACM_KERNEL_MARCH2 on a
masked problem): bitwise the fields of the single-step tile kernel with the
same walls, for scattered solid nodes with two moving wall ids and a random
state (solid nodes included: they must come back unchanged), for odd step
counts (one single step first) and on the 192^3 lid-driven cavity; mass and
energy to the rounding of the per-thread partials; the cavity against the
FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import banner, fluid_of, need_gpu, oracle_run, rel_l2, to_dev

pytestmark = pytest.mark.gpu

MARCH, MARCH2 = 2, 3


def _run(L, shape, omega, drho, u, steps, variant, mask, table, planes=None):
    nz, ny, nx = shape
    s = L.Solver(19, nx, ny, nz, omega, mask=to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table], variant=variant)
    if planes is not None:
        L.lwacm_set_march_chunk(s.ctx, planes)
    s.set_state(to_dev(drho), to_dev(u))
    s.step(steps)
    dr, uu = s.moments()
    out = (dr.cpu().numpy(), uu.cpu().numpy(), s.diagnostics())
    s.close()
    return out


def _close(x, y):
    return np.allclose(np.asarray(x), np.asarray(y), rtol=1e-6, atol=1e-9)


def _random_walls(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = (rng.random(shape) < 0.08).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 4, int(mask.sum())).astype(np.uint8)
    table = np.array([[0, 0, 0], [0, 0, 0], [0.03, -0.01, 0.02], [-0.02, 0.0, 0.01]])
    return mask, table


@pytest.mark.parametrize("shape", [(20, 32, 64), (9, 16, 32), (40, 48, 96)])
@pytest.mark.parametrize("steps", [1, 2, 7])
def test_masked_two_step_launch_bitwise_equals_single_steps(shape, steps):
    L = need_gpu()
    banner(f"march2 walls vs march {shape} steps={steps}")
    mask, table = _random_walls(shape, 41)
    drho, u = wl.random_state(shape, 3, seed=43, du=0.03, drho=0.01)
    a = _run(L, shape, 1.6, drho, u, steps, MARCH, mask, table)
    b = _run(L, shape, 1.6, drho, u, steps, MARCH2, mask, table)
    assert np.isfinite(a[1]).all()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert _close(a[2], b[2])
    # solid nodes keep the state they were given
    solid = mask != 0
    assert np.array_equal(b[0][solid], drho.astype(np.float32)[solid])
    assert np.array_equal(b[1][:, solid], u.astype(np.float32)[:, solid])


@pytest.mark.parametrize("planes", [32, 64, 128])
def test_masked_two_step_chunk_depths(planes):
    """150 planes (ragged for every depth), random walls."""
    L = need_gpu()
    shape = (150, 32, 64)
    banner(f"march2 walls chunk {planes}")
    mask, table = _random_walls(shape, 45)
    drho, u = wl.random_state(shape, 3, seed=47, du=0.03, drho=0.01)
    a = _run(L, shape, 1.7, drho, u, 4, MARCH, mask, table, planes=planes)
    b = _run(L, shape, 1.7, drho, u, 4, MARCH2, mask, table, planes=planes)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert _close(a[2], b[2])


def test_cavity_192_two_step_equals_single_steps_and_oracle_64():
    """The benchmark cavity (192^3, moving lid): 10 steps as five fused
    launches against 10 single steps; the 64^3 cavity against the oracle
    after 150 steps."""
    L = need_gpu()
    banner("march2 cavity 192^3")
    n = 192
    mask = wl.cavity_mask(n)
    table = wl.wall_table((0.1, 0.0, 0.0))
    drho, u = np.zeros((n, n, n)), np.zeros((3, n, n, n))
    a = _run(L, (n, n, n), 1.9, drho, u, 10, MARCH, mask, table)
    b = _run(L, (n, n, n), 1.9, drho, u, 10, MARCH2, mask, table)
    assert np.abs(a[1]).max() > 0.0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert _close(a[2], b[2])
    del a, b
    banner("march2 cavity 64^3 vs oracle")
    n = 64
    mask = wl.cavity_mask(n)
    table = wl.wall_table((0.05, 0.0, 0.0))
    shape = (n, n, n)
    drho, u = np.zeros(shape), np.zeros((3,) + shape)
    dr, uu, _ = _run(L, shape, 1.9, drho, u, 150, MARCH2, mask, table)
    rdr, ru = oracle_run(19, shape, 1.9, drho, u, 150, mask=mask, wall_u=table)
    fl = fluid_of(mask, shape)
    err = rel_l2(uu[:, fl], ru[:, fl])
    banner(f"march2 cavity 64: rel-L2 u {err:.3e}")
    assert err < 1e-5


def test_masked_two_step_scope():
    """Interpolated walls (a per-step wall correction) keep one step per
    launch: MARCH2 is refused there, AUTO falls back."""
    L = need_gpu()
    banner("march2 walls scope")
    shape = (8, 16, 32)
    mask = np.zeros(shape, dtype=np.uint8)
    mask[0] = 1
    nz, ny, nx = shape
    s = L.Solver(19, nx, ny, nz, 1.7, mask=to_dev(mask, torch.uint8), variant=MARCH2)
    s.close()
    q = torch.full((19, nz, ny, nx), 0.3, dtype=torch.float32, device="cuda")
    s = L.Solver(19, nx, ny, nz, 1.7, mask=to_dev(mask, torch.uint8), qd=q)
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_set_variant(s.ctx, MARCH2)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    s.close()
