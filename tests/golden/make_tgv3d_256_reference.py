"""Write the FP64 oracle's reference for the 256^3 D3Q19 Taylor-Green run.

Workload: D3Q19, 256^3 periodic, u = u0 sin kx cos ky cos kz,
v = -u0 cos kx sin ky cos kz, w = 0, rho = 1, u0 = 0.02, omega = 1.7,
1000 steps.  The full field at step 1000 is 512 MiB in FP64, so the fixture
keeps a regular subsample (every 8th node along each axis, 32^3 nodes) of
rho - 1 and u, plus the oracle's mass and kinetic energy every 100 steps.

Only the oracle is called.  Run time is about an hour on 8 cores:

    OMP_NUM_THREADS=8 python tests/golden/make_tgv3d_256_reference.py
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

STRIDE = 8
OUT = os.path.join(HERE, "tgv3d_256_step1000_sub8.npz")


def main():
    c = wl.TGV3D_256
    drho, u = wl.taylor_green_3d(c.nx, c.u0)
    p = oracle.Problem(q=19, nx=c.nx, ny=c.ny, nz=c.nz, omega=c.omega)
    diag = {}
    t0 = time.time()

    def cb(t, rho, uu):
        if t % 100 == 0:
            diag[t] = oracle.diagnostics(p, rho, uu)
            print(f"step {t}: mass {diag[t][0]:.12f} energy {diag[t][1]:.12e} "
                  f"({time.time() - t0:.0f} s)", flush=True)

    rho, uu = oracle.run(p, 1.0 + drho, u, c.steps, callback=cb)
    sub = (slice(None, None, STRIDE),) * 3
    np.savez_compressed(
        OUT, drho=(rho - 1.0)[sub], u=uu[(slice(None),) + sub], stride=STRIDE,
        steps=c.steps, omega=c.omega, u0=c.u0, n=c.nx,
        diag_steps=np.array(sorted(diag)), diag=np.array([diag[k] for k in sorted(diag)]),
        meta=json.dumps({"workload": c.name, "oracle_threads": oracle.num_threads(),
                         "seconds": time.time() - t0}))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
