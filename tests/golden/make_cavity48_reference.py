"""Write the FP64 oracle's reference for the 48^3 lid-driven cavity.

Workload: D3Q19 on a 48^3 array, boundary shell solid (46^3 fluid nodes),
the top plane z = 47 is the lid moving at (0.05, 0, 0), Re = 1000 on the
fluid width (omega = 1.972776), rho = 1 and u = 0 at rest, 50000 steps.
Stored: the full state (rho - 1, u) after 5000 and 50000 steps, and the two
centreline profiles of the steady state: u_x along z through the cavity
centre and u_z along x through it (each the mean of the 2 x 2 columns around
the centre, which lies between nodes 23 and 24).

Only the oracle is called.  Run time is about ten minutes on 8 cores:

    python tests/golden/make_cavity48_reference.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "cavity48_steps5000_50000.npz")
SNAP = 5000


def centrelines(u, n):
    """u_x(z) at the centre column and u_z(x) on the centre row, fluid nodes only."""
    c = slice(n // 2 - 1, n // 2 + 1)
    ux_z = u[0][1:n - 1, c, c].mean(axis=(1, 2))           # index z
    uz_x = u[2][c, c, 1:n - 1].mean(axis=(0, 1))           # index x
    return ux_z, uz_x


def main():
    c = wl.CAVITY_48
    n = c.nx
    mask = wl.cavity_mask(n)
    table = wl.wall_table(c.lid)
    p = oracle.Problem(q=19, nx=n, ny=n, nz=n, omega=c.omega, mask=mask, wall_u=table)
    snap = {}
    t0 = time.time()

    def cb(t, rho, uu):
        if t == SNAP:
            snap["drho"], snap["u"] = rho - 1.0, uu.copy()
        if t % 5000 == 0:
            m, e = oracle.diagnostics(p, rho, uu)
            print(f"step {t}: mass {m:.12f} energy {e:.12e} ({time.time() - t0:.0f} s)",
                  flush=True)

    rho, uu = oracle.run(p, np.ones((n, n, n)), np.zeros((3, n, n, n)), c.steps, callback=cb)
    ux_z, uz_x = centrelines(uu, n)
    np.savez_compressed(
        OUT, drho_5000=snap["drho"], u_5000=snap["u"], drho_50000=rho - 1.0, u_50000=uu,
        ux_z=ux_z, uz_x=uz_x, omega=c.omega, lid=np.array(c.lid), n=n,
        meta=json.dumps({"workload": c.name, "steps": [SNAP, c.steps],
                         "oracle_threads": oracle.num_threads(),
                         "seconds": time.time() - t0}))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
