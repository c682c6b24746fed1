"""Several D2Q9 steps per launch (temporal blocking in LDS, variant AUTO)
against one step per launch (variant GENERIC): the fields must be bitwise
equal for every step count (launches of up to 8 steps, leftovers), on
periodic grids, with walls (one moving) and a body force, on grids that are
not multiples of the 32 x 32 tile and on grids smaller than the tile's
region (several periodic images in LDS); the mass and energy agree to FP64
rounding (the sums run in another order).  The step itself is pinned against
the oracle by tests/test_gpu_forward.py, which now runs this kernel."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu

GENERIC = 1


def _run(L, shape, omega, drho, u, steps, mask, table, g, variant):
    nz, ny, nx = shape
    s = L.Solver(9, nx, ny, 1, omega, mask=None if mask is None else to_dev(mask, torch.uint8),
                 wall_u=None if table is None else [list(r) for r in table], g=g,
                 variant=variant)
    s.set_state(to_dev(drho), to_dev(u))
    s.step(steps)
    st = s.save_state().cpu().numpy()
    m, e = s.diagnostics()
    s.close()
    return st, m, e


CASES = [("periodic 64^2", (1, 64, 64), False), ("channel 64x256", (1, 64, 256), True),
         ("ragged 40x48", (1, 40, 48), True), ("tiny 12x20", (1, 12, 20), False),
         ("512^2", (1, 512, 512), False)]


@pytest.mark.parametrize("name,shape,walls", CASES)
def test_multi_step_launches_equal_single_steps(name, shape, walls):
    L = need_gpu()
    nz, ny, nx = shape
    mask = table = g = None
    if walls:
        mask = wl.channel_mask(nx, ny, moving_top=True)
        table = wl.wall_table((0.02, 0.0, 0.0))
        g = (1e-5, -2e-6)
    drho, u = wl.random_state(shape, 2, seed=71, du=0.03, drho=0.01)
    if walls:
        u[:, mask != 0] = 0.0
    for steps in (1, 7, 8, 9, 23):
        banner(f"d2q9 multi {name} steps={steps}")
        a, ma, ea = _run(L, shape, 1.7, drho, u, steps, mask, table, g, 0)
        b, mb, eb = _run(L, shape, 1.7, drho, u, steps, mask, table, g, GENERIC)
        assert np.array_equal(a, b), (name, steps)
        assert abs(ma - mb) <= 1e-12 * abs(mb) and abs(ea - eb) <= 1e-12 * abs(eb)
    torch.cuda.synchronize()
