"""Write the FP64 oracle's circular Couette runs (Section "Circular Couette
flow") at eps = 1/20, 1/40 and 1/80 to t = 20: the final fields at 1/20 and
1/40, and the L1 errors and inner-cylinder torque at every eps.

Geometry and inputs: ``workloads.CircularCouette(eps)`` (r_i = 0.5, r_e = 1,
nu = 0.07, link-wall distances and wall velocities from the exact circles),
fluid at rest with rho = 1 at t = 0.  Calls only ``oracle``; about 2 minutes
on 8 threads (most of it at 1/80).

    python tests/golden/make_circular_couette_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import workloads as wl  # noqa: E402
from circular_couette import l1_errors  # noqa: E402

OUT = os.path.join(HERE, "circular_couette_oracle.npz")


def run(eps, t_end=20.0):
    cc = wl.CircularCouette(eps)
    _, v, _, _ = oracle.lattice_info(9)
    qd, uwl = cc.links(v)
    p = oracle.Problem(q=9, nx=cc.n, ny=cc.n, omega=cc.omega, mask=cc.mask,
                       wall_u=np.zeros((3, 3)), rho0=1.0)
    rho, u = np.ones((1, cc.n, cc.n)), np.zeros((2, 1, cc.n, cc.n))
    for _ in range(cc.steps_to(t_end)):
        rho, u = oracle.step_q(p, rho, u, qd, uwl)
    _, T = oracle.wall_force(p, rho, u, 1, center=cc.center, qd=qd)
    return rho, u, T[2], l1_errors(cc, rho, u, T[2])


def main():
    out = {}
    for k, eps in ((20, 1 / 20), (40, 1 / 40), (80, 1 / 80)):
        t0 = time.time()
        rho, u, tz, err = run(eps)
        print(f"eps = 1/{k}: L1 u_theta {err[0]:.6e}, p {err[1]:.6e}, |T| {err[2]:.6e}, "
              f"T_z {tz:.9f} ({time.time() - t0:.0f} s)", flush=True)
        out[f"errors_{k}"] = np.array(err)
        out[f"torque_{k}"] = np.float64(tz)
        if k <= 40:
            out[f"rho_{k}"] = rho
            out[f"u_{k}"] = u
    np.savez_compressed(OUT, **out)


if __name__ == "__main__":
    main()
