"""Status codes of the C ABI on the GPU: a run driven to blow-up is reported
as LWACM_ENONFINITE by lwacm_diagnostics and lwacm_moments, and a relaxation
frequency below 1 is accepted with the LWACM_WOMEGA warning (the paper finds
the method stable for 1 <= omega < 2, Section "Physical and lattice units")."""
import warnings

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import banner, gpu_run, need_gpu, oracle_run, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("q,shape", [(9, (1, 32, 32)), (19, (8, 16, 32))])
def test_blow_up_is_reported_as_nonfinite(q, shape):
    """|u| up to 0.35 at omega = 1.99 diverges (the FP64 oracle passes 1e38 by
    step ~130 on both grids), so after 400 FP32 steps mass and energy are not
    finite and both diagnostic calls say so."""
    L = need_gpu()
    banner(f"blow-up q={q} shape={shape}")
    d = 2 if q == 9 else 3
    drho, u = wl.random_state(shape, d, seed=5, du=0.35, drho=0.05)
    nz, ny, nx = shape
    s = L.Solver(q, nx, ny, nz, 1.99)
    s.set_state(to_dev(drho), to_dev(u))
    s.step(400)
    with pytest.raises(L.LWACMError) as e1:
        s.diagnostics()
    assert e1.value.code == L.LWACM_ENONFINITE
    with pytest.raises(L.LWACMError) as e2:
        s.moments(diagnostics=True)
    assert e2.value.code == L.LWACM_ENONFINITE
    # a stable run on the same context's grid reports finite values
    s.close()
    s = L.Solver(q, nx, ny, nz, 1.6)
    s.set_state(to_dev(drho), to_dev(0.1 * u))
    s.step(10)
    m, e = s.diagnostics()
    assert np.isfinite(m) and np.isfinite(e)
    s.close()


def test_omega_below_one_is_accepted_with_a_warning():
    """The step still runs as specified.  Only 3 steps: below omega = 1 the
    grid-scale modes of a random state grow (a 1e-7 perturbation reaches
    2.5e-5 after 20 steps in the FP64 oracle), so FP32 rounding would be
    amplified past the parity bar over longer runs."""
    L = need_gpu()
    banner("omega 0.9 warning")
    shape = (1, 24, 20)
    drho, u = wl.random_state(shape, 2, seed=2, du=0.02, drho=0.01)
    with pytest.warns(L.LWACMOmegaWarning):
        dr, uu, s = gpu_run(9, shape, 0.9, drho, u, 3)
    s.close()
    r_ref, u_ref = oracle_run(9, shape, 0.9, drho, u, 3)
    assert rel_l2(uu, u_ref) < 1e-5
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        s = L.Solver(9, 20, 24, 1, 1.2)  # omega >= 1: no warning
        with pytest.warns(L.LWACMOmegaWarning):
            L.lwacm_set_omega_p(s.ctx, 0.8)
        s.close()
    torch.cuda.synchronize()
