"""The two halves of a checkpointed reverse sweep as single calls:
lwacm_forward_states (a segment's states recomputed from its checkpoint) must
give bitwise the states of the same steps taken one lwacm_step at a time
(D2Q9 periodic and with walls and force, D3Q19 tile grids, FP16 storage with
stochastic rounding at a nonzero step index, halfway and interpolated walls
(solid nodes included), the semi-implicit update), and lwacm_adjoint_sweep
bitwise the mu and dL/domega of separate reverse-step calls (D2Q9 with up to
8 steps per launch in LDS -- dL/domega there to FP64 rounding -- periodic,
with walls, a moving wall and force, and on a grid smaller than the LDS
region; D3Q19 with two steps per launch and an odd count, D3Q19 walls with a
moving id; t0 = 0 and t0 > 0)."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _solver(L, case):
    q, shape, kw = case["q"], case["shape"], dict(case.get("kw", {}))
    nz, ny, nx = shape
    if "mask" in kw:
        kw["mask"] = to_dev(kw["mask"], torch.uint8)
    if "qd" in kw:
        kw["qd"] = to_dev(kw["qd"])
    s = L.Solver(q, nx, ny, nz, 1.6, **kw)
    if case.get("semi_implicit"):
        L.lwacm_set_semi_implicit(s.ctx, 1)
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=81, du=0.03, drho=0.01)
    if "mask" in case.get("kw", {}):
        u[:, case["kw"]["mask"] != 0] = 0.0
    s.set_state(to_dev(drho), to_dev(u))
    return s


def _channel(nx, ny):
    m = wl.channel_mask(nx, ny, moving_top=True)
    return m, wl.wall_table((0.02, 0.0, 0.0))


def _cases():
    mask2, table2 = _channel(96, 40)
    rng = np.random.Generator(np.random.PCG64(83))
    mask3 = (rng.random((16, 32, 64)) < 0.05).astype(np.uint8)
    qd3 = rng.uniform(0.1, 0.9, (19, 16, 32, 64)).astype(np.float32)
    return [
        dict(name="d2q9 periodic 128^2", q=9, shape=(1, 128, 128)),
        dict(name="d2q9 channel walls and force", q=9, shape=(1, 40, 96),
             kw=dict(mask=mask2, wall_u=[list(r) for r in table2], g=(1e-5, 0.0))),
        dict(name="d3q19 tile 24x32x64", q=19, shape=(24, 32, 64)),
        dict(name="d3q19 fp16 stochastic", q=19, shape=(16, 32, 64), kw=dict(storage=1), t0=37),
        dict(name="d3q19 interpolated walls", q=19, shape=(16, 32, 64),
             kw=dict(mask=mask3, qd=qd3)),
        dict(name="d3q19 halfway walls, moving id", q=19, shape=(16, 32, 64),
             kw=dict(mask=mask3 * 2, wall_u=[[0, 0, 0], [0, 0, 0], [0.03, 0.0, -0.01]])),
        dict(name="d2q9 semi-implicit", q=9, shape=(1, 64, 64), semi_implicit=True),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_forward_states_equal_single_steps(case):
    L = need_gpu()
    banner(f"forward_states {case['name']}")
    nsteps, t0 = 11, case.get("t0", 0)
    s = _solver(L, case)
    if t0:
        s.load_state(s.save_state(), t0)  # the step index selects the FP16 rounding words
    st0 = s.save_state()
    ref = []
    for _ in range(nsteps):
        s.step(1)
        ref.append(s.save_state())
    sb = s.state_bytes
    out = torch.zeros(nsteps * sb, dtype=torch.uint8, device="cuda")
    L.lwacm_forward_states(s.ctx, st0, t0, nsteps, out)
    torch.cuda.synchronize()
    for k in range(nsteps):
        assert torch.equal(out[k * sb:(k + 1) * sb], ref[k]), (case["name"], k)
    # the context's own state and step count are untouched
    assert s.step_count == t0 + nsteps
    assert torch.equal(s.save_state(), ref[-1])
    s.close()


_MASK_S = (np.random.Generator(np.random.PCG64(87)).random((16, 32, 64)) < 0.05).astype(np.uint8) * 2
SWEEP_CASES = [
    dict(name="d2q9", q=9, shape=(1, 64, 96), n=9, t0=0),
    dict(name="d3q19 walls, moving id", q=19, shape=(16, 32, 64), n=5, t0=0,
         kw=dict(mask=_MASK_S, wall_u=[[0, 0, 0], [0, 0, 0], [0.03, 0.0, -0.01]])),
    dict(name="d2q9 t0 > 0", q=9, shape=(1, 64, 96), n=6, t0=20),
    dict(name="d2q9 walls and force, 19 steps", q=9, shape=(1, 40, 96), n=19, t0=0,
         kw=dict(mask=wl.channel_mask(96, 40, moving_top=True),
                 wall_u=[list(r) for r in wl.wall_table((0.02, 0.0, 0.0))], g=(1e-5, 0.0))),
    dict(name="d2q9 12^2 smaller than the region", q=9, shape=(1, 12, 20), n=10, t0=3),
    dict(name="d3q19 pairs odd count", q=19, shape=(16, 32, 64), n=7, t0=0),
    dict(name="d3q19 pairs t0 > 0", q=19, shape=(16, 32, 64), n=6, t0=5),
]


@pytest.mark.parametrize("case", SWEEP_CASES, ids=lambda c: c["name"])
def test_adjoint_sweep_equals_separate_calls(case):
    L = need_gpu()
    banner(f"adjoint_sweep {case['name']}")
    s = _solver(L, case)
    n, t0, sb = case["n"], case["t0"], s.state_bytes
    states = torch.zeros(n * sb, dtype=torch.uint8, device="cuda")
    for k in range(n):
        states[k * sb:(k + 1) * sb].copy_(s.save_state())
        s.step(1)
    d = s.D
    rng = np.random.Generator(np.random.PCG64(85))
    mu0 = torch.as_tensor(rng.standard_normal((d + 1,) + s.shape).astype(np.float32),
                          device="cuda")
    # separate calls, two per launch where the library can, as before
    mu, tmp = mu0.clone(), torch.empty_like(mu0)
    dw = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
    j = n - 1
    slot = lambda k: states[k * sb:(k + 1) * sb]
    while j >= 0:
        if j >= 1 and L.lwacm_adjoint_step2(s.ctx, slot(j), slot(j - 1), mu, tmp, dw,
                                            t0 + j - 1 == 0):
            j -= 2
        else:
            L.lwacm_adjoint_step(s.ctx, slot(j), mu, tmp, dw, t0 + j == 0)
            j -= 1
        mu, tmp = tmp, mu
    # one sweep
    mu_s, tmp_s = mu0.clone(), torch.empty_like(mu0)
    dw_s = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
    L.lwacm_adjoint_sweep(s.ctx, states, t0, n, mu_s, tmp_s, dw_s)
    torch.cuda.synchronize()
    assert torch.equal(mu_s, mu)
    if case["q"] == 9:  # 8 steps per launch: per-step sums over 32 x 32 tiles
        assert abs(dw_s.item() - dw.item()) <= 1e-12 * abs(dw.item() - 0.25)
    else:
        assert dw_s.item() == dw.item()
    assert np.isfinite(mu_s.cpu().numpy()).all() and dw_s.item() != 0.25
    s.close()


def test_segment_calls_reject_bad_arguments():
    L = need_gpu()
    s = L.Solver(9, 32, 32, 1, 1.6)
    st = s.save_state()
    with pytest.raises(L.LWACMError):
        L.lwacm_forward_states(s.ctx, st, 0, 2, st)  # overlapping slots
    mu = torch.zeros((3, 1, 32, 32), device="cuda")
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LWACMError):
        L.lwacm_adjoint_sweep(s.ctx, st, 0, 1, mu, mu, dw)  # mu and scratch alias
    s.close()
