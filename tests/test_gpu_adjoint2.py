"""Two reverse steps per launch (lwacm_adjoint_step2): bitwise the mu (or the
final gradient) of two one-step reverse calls, on grids whose last z chunk
is ragged, on thin grids (nz = 8, 20: chunk depths 8 and 16), with FP32 and
FP16 states, for both output forms, and at 256^3 (128-plane chunks); the omega-gradient sum
bitwise where both kernels split the planes among workgroups alike, else to
the rounding of the per-thread FP32 partials.  Problems with walls are
declined, and the checkpointed gradient, which now pairs its reverse steps,
still matches the oracle (tests/test_gpu_adjoint.py)."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _states(L, shape, storage, seed, mask=None):
    """Two consecutive states (storage format) and a random mu."""
    nz, ny, nx = shape
    s = L.Solver(19, nx, ny, nz, 1.6, storage=storage,
                 mask=None if mask is None else to_dev(mask, torch.uint8))
    drho, u = wl.random_state(shape, 3, seed=seed, du=0.03, drho=0.01)
    s.set_state(to_dev(drho), to_dev(u))
    st_tm1 = s.save_state()
    s.step(1)
    st_t = s.save_state()
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    mu = to_dev(rng.standard_normal((4,) + shape) * 0.1)
    # node-interleaved mu for the reverse sweep
    mu_il = mu.permute(1, 2, 3, 0).contiguous()
    return s, st_t, st_tm1, mu_il


def _two_single(L, s, st_t, st_tm1, mu, final):
    tmp = torch.empty_like(mu)
    out = torch.zeros_like(mu)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    L.lwacm_adjoint_step(s.ctx, st_t, mu, tmp, dw, False)
    L.lwacm_adjoint_step(s.ctx, st_tm1, tmp, out, dw, final)
    torch.cuda.synchronize()
    return out, float(dw.item())


def _fused(L, s, st_t, st_tm1, mu, final):
    out = torch.zeros_like(mu)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert L.lwacm_adjoint_step2(s.ctx, st_t, st_tm1, mu, out, dw, final)
    torch.cuda.synchronize()
    return out, float(dw.item())


@pytest.mark.parametrize("shape", [(64, 32, 64), (150, 32, 64), (8, 16, 32), (20, 16, 32)])
@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("final", [False, True])
def test_adjoint_step2_bitwise_equals_two_steps(shape, storage, final):
    L = need_gpu()
    banner(f"adjoint2 {shape} storage={storage} final={final}")
    s, st_t, st_tm1, mu = _states(L, shape, storage, seed=41)
    a, wa = _two_single(L, s, st_t, st_tm1, mu, final)
    b, wb = _fused(L, s, st_t, st_tm1, mu, final)
    s.close()
    assert bool(torch.isfinite(a).all())
    assert torch.equal(a, b)
    if shape[0] % 64 == 0:  # both kernels use 64-plane chunks: the same block sums
        assert wa == wb
    else:
        assert abs(wa - wb) <= 1e-6 * abs(wa) + 1e-9


def test_adjoint_step2_declines_walls():
    L = need_gpu()
    banner("adjoint2 walls")
    shape = (16, 16, 32)
    mask = np.zeros(shape, dtype=np.uint8)
    mask[0] = 1
    s, st_t, st_tm1, mu = _states(L, shape, 0, seed=43, mask=mask)
    out = torch.zeros_like(mu)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert not L.lwacm_adjoint_step2(s.ctx, st_t, st_tm1, mu, out, dw, False)
    assert float(out.abs().sum()) == 0.0 and float(dw.item()) == 0.0
    s.close()


def test_adjoint_step2_256_cubed_bitwise():
    """The benchmark grid: ten fused launches against twenty single steps."""
    L = need_gpu()
    n = 256
    banner("adjoint2 256^3")
    s = L.Solver(19, n, n, n, 1.7)
    drho, u = wl.taylor_green_3d(n, 0.02)
    s.set_state(to_dev(drho), to_dev(u))
    s.step(2)
    st_tm1 = s.save_state()
    s.step(1)
    st_t = s.save_state()
    mu0 = torch.zeros((n, n, n, 4), device="cuda")
    mu0[..., 1:] = to_dev(u).permute(1, 2, 3, 0)

    def single():
        a, b = mu0.clone(), torch.empty_like(mu0)
        dw = torch.zeros(1, dtype=torch.float64, device="cuda")
        for _ in range(10):
            L.lwacm_adjoint_step(s.ctx, st_t, a, b, dw, False)
            L.lwacm_adjoint_step(s.ctx, st_tm1, b, a, dw, False)
        return a, float(dw.item())

    def fused():
        a, b = mu0.clone(), torch.empty_like(mu0)
        dw = torch.zeros(1, dtype=torch.float64, device="cuda")
        for _ in range(5):
            assert L.lwacm_adjoint_step2(s.ctx, st_t, st_tm1, a, b, dw, False)
            assert L.lwacm_adjoint_step2(s.ctx, st_t, st_tm1, b, a, dw, False)
        return a, float(dw.item())

    (ra, wa), (rb, wb) = single(), fused()
    s.close()
    assert bool(torch.isfinite(ra).all())
    assert torch.equal(ra, rb)
    # 128-plane chunks against the single step's 64: the block sums regroup
    assert abs(wa - wb) <= 1e-6 * abs(wa)
