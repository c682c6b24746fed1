"""lwacm_step_static: the forward steps for callers that cannot allocate,
with its reduction partials in the library's fixed device array, against the
context path (lwacm_init + lwacm_set_state + lwacm_step + lwacm_diagnostics)
on the same inputs: the state bytes and the FP64 mass and energy must be
bitwise equal (the same kernels in the same order).  Two calls in a row, the
second on a smaller problem, so leftovers of the first call in the shared
array cannot leak into the second."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import banner, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _context_run(L, q, shape, omega, drho, u, nsteps):
    nz, ny, nx = shape
    s = L.Solver(q, nx, ny, nz, omega)
    s.set_state(to_dev(drho), to_dev(u))
    init = s.save_state()
    s.step(nsteps)
    out = s.save_state()
    mass, energy = s.diagnostics() if nsteps > 0 else (None, None)
    s.close()
    return init, out, mass, energy


def _static_run(L, q, shape, omega, init, nsteps):
    nz, ny, nx = shape
    a = init.clone().view(torch.float32)
    b = torch.full_like(a, float("nan"))
    diag = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    out = L.lwacm_step_static(q, nx, ny, nz, omega, a, b, nsteps, diag)
    torch.cuda.synchronize()
    assert out is a or out is b
    return out, diag.cpu().numpy()


# (lattice, shape (nz, ny, nx), omega, steps): the two-step tile kernel with
# an odd count (one single step, then pairs), a smaller tile grid, the
# generic kernel (D3Q19 off the tile shape, D2Q9), a count of zero
CASES = [(19, (24, 32, 64), 1.7, 7), (19, (8, 16, 32), 1.6, 4), (19, (5, 7, 9), 1.3, 3),
         (9, (1, 40, 48), 1.8, 5), (19, (8, 16, 32), 1.7, 0)]


def test_static_step_matches_the_context_path_twice_in_a_row():
    L = need_gpu()
    for seed, (q, shape, omega, nsteps) in enumerate(CASES):
        banner(f"lwacm_step_static q={q} shape={shape} steps={nsteps}")
        d = 2 if q == 9 else 3
        drho, u = wl.random_state(shape, d, seed=10 + seed, du=0.04, drho=0.01)
        init, ref, mass, energy = _context_run(L, q, shape, omega, drho, u, nsteps)
        got, diag = _static_run(L, q, shape, omega, init, nsteps)
        assert torch.equal(got.view(torch.uint8), ref), (q, shape)
        if nsteps > 0:
            n = int(np.prod(shape))
            assert float(n) + diag[0] == mass
            assert diag[1] == energy
        else:
            assert np.isnan(diag).all()  # no step: nothing written


def test_static_step_rejects_problems_beyond_its_scratch():
    """(3072/32) x (1536/16) tiles of one 8-plane chunk need 9216 blocks,
    more than the 8192 the fixed array holds: LWACM_ESCRATCH, nothing
    launched (both buffers keep their bytes)."""
    L = need_gpu()
    banner("lwacm_step_static scratch limit")
    nx, ny, nz = 3072, 1536, 8
    nbytes = L.lwacm_state_bytes(19, nx, ny, nz, 0)
    a = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    with pytest.raises(L.LWACMError) as e:
        L.lwacm_step_static(19, nx, ny, nz, 1.7, a, b, 2)
    assert e.value.code == L.LWACM_ESCRATCH
    torch.cuda.synchronize()
    assert float(a.abs().max()) == 0.0 and float(b.min()) == 1.0
    del a, b
    torch.cuda.empty_cache()
