"""Interpolated bounce-back with link-wall distances (lwacm_init's d_q;
Eqs. ACM2.0cc and ACM2.0move) against the oracle's step_q.

- q = 1/2 on every link gives the halfway step of the generic kernel, bit
  for bit.
- Random walls with moving ids and random q in [0.05, 1]: D2Q9 and D3Q19,
  FP32 and FP16 storage, to the parity bars.
- Plane Couette flow between off-lattice walls (q = 0.3 and 0.7): the GPU's
  steady state is the exact linear profile to FP32 accuracy.
- Scope: the reverse steps, the two-step kernel and a separate omega_p
  decline d_q (the single-step D3Q19 tile kernels take it through the
  per-step wall correction: tests/test_gpu_wall_correction.py).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from gpu_helpers import banner, fluid_of, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu

GENERIC, MARCH = 1, 2


def _library_order(q, qd_oracle):
    """The oracle's per-link fields reordered into the library's link order
    (lwacm.LINK_VELOCITIES), matching links by their velocity vectors."""
    from paper_1111_2142_amd import lwacm as L
    _, v, _, _ = oracle.lattice_info(q)
    where = {tuple(int(c) for c in v[k]): k for k in range(q)}
    return np.stack([qd_oracle[where[vel]] for vel in L.LINK_VELOCITIES[q]])


def _walls(q, shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = (rng.random(shape) < 0.1).astype(np.uint8)
    mask[mask == 1] = rng.integers(1, 3, int(mask.sum())).astype(np.uint8)
    qd = rng.uniform(0.05, 1.0, (q,) + shape)
    table = np.array([[0, 0, 0], [0, 0, 0], [0.03, -0.01, 0.02]])
    return mask, qd, table


def _gpu(L, q, shape, omega, drho, u, steps, mask, table, qd, storage=0, variant=0):
    nz, ny, nx = shape
    s = L.Solver(q, nx, ny, nz, omega, storage=storage, mask=to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table], variant=variant,
                 qd=None if qd is None else to_dev(qd))
    s.set_state(to_dev(drho), to_dev(u))
    s.step(steps)
    dr, uu = s.moments()
    s.close()
    return dr.double().cpu().numpy(), uu.double().cpu().numpy()


@pytest.mark.parametrize("q,shape", [(9, (1, 40, 48)), (19, (12, 32, 32))])
def test_q_one_half_is_the_halfway_step(q, shape):
    """On the generic kernel q = 1/2 gives the halfway step bit for bit; on the
    D3Q19 tile kernel (halfway terms plus the per-step wall correction, whose
    interpolation part is then zero) it agrees with it to FP32 rounding."""
    L = need_gpu()
    banner(f"interpolated bb q=1/2 q={q}")
    d = 2 if q == 9 else 3
    mask, _, table = _walls(q, shape, 41)
    drho, u = wl.random_state(shape, d, seed=42, du=0.03, drho=0.01)
    a = _gpu(L, q, shape, 1.5, drho, u, 5, mask, table, None, variant=GENERIC)
    half = np.full((q,) + shape, 0.5)
    b = _gpu(L, q, shape, 1.5, drho, u, 5, mask, table, half, variant=GENERIC)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    if q == 19:
        c = _gpu(L, q, shape, 1.5, drho, u, 5, mask, table, half)
        assert np.abs(c[1] - a[1]).max() < 1e-8 and np.abs(c[0] - a[0]).max() < 1e-7


@pytest.mark.parametrize("q,storage", [(9, 0), (19, 0), (19, 1)])
def test_random_walls_and_distances_match_oracle(q, storage):
    L = need_gpu()
    banner(f"interpolated bb random q={q} storage={storage}")
    shape = (1, 40, 48) if q == 9 else (12, 32, 32)
    nz, ny, nx = shape
    d = 2 if q == 9 else 3
    mask, qd, table = _walls(q, shape, 43)
    qd = qd.astype(np.float32).astype(np.float64)
    drho, u = wl.random_state(shape, d, seed=44, du=0.03, drho=0.01)
    drho = drho.astype(np.float32).astype(np.float64)
    u = u.astype(np.float32).astype(np.float64)
    rho0 = 1.0 + drho[mask == 0].astype(np.float32).mean()
    dr, uu = _gpu(L, q, shape, 1.5, drho, u, 6, mask, table, _library_order(q, qd),
                  storage=storage)
    p = oracle.Problem(q, nx, ny, nz, omega=1.5, mask=mask, wall_u=table, rho0=rho0)
    r, ru = 1.0 + drho, u
    for _ in range(6):
        r, ru = oracle.step_q(p, r, ru, qd)
    fl = fluid_of(mask, shape)
    err_u, err_r = rel_l2(uu[:, fl], ru[:, fl]), rel_l2(dr[fl], (r - 1.0)[fl])
    banner(f"interpolated bb: rel-L2 u {err_u:.3e}, drho {err_r:.3e}")
    assert err_u < (1e-5 if storage == 0 else 1e-3)
    assert err_r < (1e-4 if storage == 0 else 2e-2)


@pytest.mark.parametrize("q", [9, 19])
def test_couette_between_off_lattice_walls(q):
    L = need_gpu()
    banner(f"interpolated bb Couette q={q}")
    h, U, qb, qt = 12, 0.01, 0.3, 0.7
    d, v, _, _ = oracle.lattice_info(q)
    ax = 1 if q == 9 else 2
    shape = (1, h, 32) if q == 9 else (h, 16, 32)
    mask = np.zeros(shape, np.uint8)
    sl = [slice(None)] * 3
    sl[2 - ax] = 0
    mask[tuple(sl)] = 1
    sl[2 - ax] = h - 1
    mask[tuple(sl)] = 2
    qd = np.full((q,) + shape, 0.5)
    for j in range(q):
        if v[j][ax] == -1:
            sl[2 - ax] = 1
            qd[(j,) + tuple(sl)] = qb
        if v[j][ax] == 1:
            sl[2 - ax] = h - 2
            qd[(j,) + tuple(sl)] = qt
    table = np.array([[0, 0, 0], [0, 0, 0], [U, 0, 0]])
    dr, uu = _gpu(L, q, shape, 1.0, np.zeros(shape), np.zeros((d,) + shape), 4000, mask,
                  table, _library_order(q, qd))
    coord = np.arange(1, h - 1)
    exact = U * (coord - (1 - qb)) / ((h - 2 + qt) - (1 - qb))
    sl[2 - ax] = slice(1, h - 1)
    ux = uu[0][tuple(sl)]
    prof = ux.reshape(h - 2, -1) if ax == 2 else np.moveaxis(ux, 1, 0).reshape(h - 2, -1)
    err = float(np.abs(prof - exact[:, None]).max() / U)
    banner(f"interpolated bb Couette: max error / U {err:.3e}")
    assert err < 1e-5


def test_interpolated_bb_scope():
    L = need_gpu()
    banner("interpolated bb scope")
    shape = (16, 32, 64)
    mask, qd, table = _walls(19, shape, 45)
    s = L.Solver(19, 64, 32, 16, 1.6, mask=to_dev(mask, torch.uint8),
                 wall_u=[list(r) for r in table], qd=to_dev(qd))
    L.lwacm_set_variant(s.ctx, MARCH)  # the tile kernels take d_q (wall correction)
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_set_variant(s.ctx, 3)  # not the two-step kernel (walls)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_set_omega_p(s.ctx, 1.1)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    drho, u = wl.random_state(shape, 3, seed=46, du=0.02, drho=0.01)
    s.set_state(to_dev(drho), to_dev(u))
    st = s.save_state()
    mu = torch.zeros(shape + (4,), device="cuda")
    out = torch.zeros_like(mu)
    dw = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LWACMError) as ei:
        L.lwacm_adjoint_step(s.ctx, st, mu, out, dw, False)
    assert ei.value.code == L.LWACM_EUNSUPPORTED
    assert not L.lwacm_adjoint_step2(s.ctx, st, st, mu, out, dw, False)
    s.close()
