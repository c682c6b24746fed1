"""Two forward steps per launch (LWACM_KERNEL_MARCH2): the fused kernel must
give bitwise the fields of the single-step tile kernel, on grids whose last
z chunk is ragged (the two-step kernel moves it down to end at nz and writes
the shared planes twice), on the thinnest grids it accepts (nz = 8, 9, 20:
chunk depths 8 and 16), for odd step counts (one single step first) and at
256^3; the same mass/energy diagnostics and per-step history (bitwise where
both kernels split the planes among blocks alike, else to the rounding of
the per-thread FP32 partial sums); and it must match the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import banner, need_gpu, oracle_run, rel_l2, to_dev

pytestmark = pytest.mark.gpu

MARCH, MARCH2 = 2, 3


def _run(L, shape, omega, drho, u, steps, variant, planes=None, hist_len=0):
    nz, ny, nx = shape
    s = L.Solver(19, nx, ny, nz, omega, variant=variant)
    if planes is not None:
        L.lwacm_set_march_chunk(s.ctx, planes)
    hist = None
    if hist_len:
        hist = torch.full((hist_len, 2), float("nan"), dtype=torch.float64, device="cuda")
        L.lwacm_set_diag_history(s.ctx, hist)
    s.set_state(to_dev(drho), to_dev(u))
    s.step(steps)
    dr, uu = s.moments()
    diag = s.diagnostics()
    out = (dr.cpu().numpy(), uu.cpu().numpy(), diag,
           None if hist is None else hist.cpu().numpy())
    s.close()
    return out


def _close(x, y):
    """Diagnostics of the same fields summed over a different split of planes
    among blocks: each thread adds its planes in FP32 before the FP64 block
    and grid sums, so the totals agree to FP32 rounding of those partials."""
    return np.allclose(np.asarray(x), np.asarray(y), rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("shape", [(150, 32, 64), (8, 16, 32), (9, 16, 32), (20, 16, 32),
                                   (40, 48, 96)])
@pytest.mark.parametrize("steps", [1, 2, 7])
def test_two_step_launch_bitwise_equals_single_steps(shape, steps):
    L = need_gpu()
    banner(f"march2 vs march {shape} steps={steps}")
    drho, u = wl.random_state(shape, 3, seed=31, du=0.03, drho=0.01)
    a = _run(L, shape, 1.7, drho, u, steps, MARCH, hist_len=steps + 1)
    b = _run(L, shape, 1.7, drho, u, steps, MARCH2, hist_len=steps + 1)
    assert np.isfinite(a[1]).all()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert _close(a[2], b[2])
    # history: slot t holds (mass deviation, energy) of step t; slot 0 unused
    assert _close(a[3][1:], b[3][1:])
    assert np.isnan(b[3][0]).all()
    if shape[0] >= 32:  # both kernels use 32-plane chunks: the same block sums
        assert a[2] == b[2] and np.array_equal(a[3][1:], b[3][1:])


@pytest.mark.parametrize("planes", [32, 64, 128])
def test_two_step_chunk_depths_agree_bitwise(planes):
    """150 planes: ragged for every depth; depth 128 is also compared with
    the oracle."""
    L = need_gpu()
    shape = (150, 32, 64)
    banner(f"march2 chunk {planes}")
    drho, u = wl.random_state(shape, 3, seed=33, du=0.03, drho=0.01)
    a = _run(L, shape, 1.6, drho, u, 6, MARCH, planes=planes)
    b = _run(L, shape, 1.6, drho, u, 6, MARCH2, planes=planes)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    c = _run(L, shape, 1.6, drho, u, 6, MARCH2, planes=32)
    assert np.array_equal(b[0], c[0]) and np.array_equal(b[1], c[1])
    if planes == 128:
        rdr, ru = oracle_run(19, shape, 1.6, drho.astype(np.float32).astype(np.float64),
                             u.astype(np.float32).astype(np.float64), 6)
        err = rel_l2(b[1].astype(np.float64), ru)
        banner(f"march2 vs oracle: rel-L2 u {err:.3e}")
        assert err < 1e-5


def test_two_step_variant_scope():
    """MARCH2 takes FP32 problems without force, halfway walls allowed (see
    test_gpu_march2_walls.py); AUTO uses it there and falls back elsewhere."""
    L = need_gpu()
    banner("march2 scope")
    s = L.Solver(19, 32, 16, 8, 1.7, storage=1)
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_set_variant(s.ctx, MARCH2)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    s.close()
    mask = torch.zeros((8, 16, 32), dtype=torch.uint8, device="cuda")
    mask[0] = 1
    s = L.Solver(19, 32, 16, 8, 1.7, mask=mask)
    L.lwacm_set_variant(s.ctx, MARCH2)
    s.close()
    s = L.Solver(19, 32, 16, 7, 1.7)   # fewer than 8 planes: single-step kernel only
    with pytest.raises(L.LWACMError):
        L.lwacm_set_variant(s.ctx, MARCH2)
    s.close()
    s = L.Solver(19, 32, 16, 8, 1.7, g=(1e-5, 0.0, 0.0))
    with pytest.raises(L.LWACMError):
        L.lwacm_set_variant(s.ctx, MARCH2)
    s.close()


def test_two_step_256_cubed_bitwise_equals_single_steps():
    """The benchmark grid: 100 steps (50 fused launches) against 100 single
    steps, and the same fused run twice."""
    L = need_gpu()
    n = 256
    banner("march2 256^3")
    drho, u = wl.taylor_green_3d(n, 0.02)
    d0, u0 = to_dev(drho), to_dev(u)

    def run(variant):
        s = L.Solver(19, n, n, n, 1.7, variant=variant)
        s.set_state(d0, u0)
        s.step(100)
        dr, uu = s.moments()
        diag = s.diagnostics()
        s.close()
        return dr, uu, diag

    a, b, c = run(MARCH), run(MARCH2), run(MARCH2)
    assert bool(torch.isfinite(a[1]).all())
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]
    assert torch.equal(b[0], c[0]) and torch.equal(b[1], c[1]) and b[2] == c[2]
