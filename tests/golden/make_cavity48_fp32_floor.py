"""Write the FP32-storage floor of the 48^3 lid-driven cavity reference.

The oracle's FP64 step is run again from rest, with its state rounded to
FP32 after every step: the error that storing the state in FP32 causes by
itself, whatever the arithmetic.  Written: the relative L2 error of u and of
rho - 1 over fluid nodes against the FP64 run stored in
cavity48_steps5000_50000.npz, after 5000 and 50000 steps.

Only the oracle is called.  Run time is about ten minutes on 8 cores:

    python tests/golden/make_cavity48_fp32_floor.py
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

REF = os.path.join(HERE, "cavity48_steps5000_50000.npz")
OUT = os.path.join(HERE, "cavity48_fp32_floor.json")


def rel_l2(x, ref):
    return float(np.sqrt(((x - ref) ** 2).sum()) / np.sqrt((ref ** 2).sum()))


def main():
    ref = np.load(REF)
    c = wl.CAVITY_48
    n = c.nx
    mask = wl.cavity_mask(n)
    fl = mask == 0
    p = oracle.Problem(q=19, nx=n, ny=n, nz=n, omega=c.omega, mask=mask,
                       wall_u=wl.wall_table(c.lid))
    r = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    out = {"workload": c.name, "what": "FP64 oracle step, state rounded to FP32 after every step"}
    t0 = time.time()
    for t in range(1, c.steps + 1):
        r, u = oracle.step(p, r, u)
        # the stored quantities are rho - 1 and u, as in the FP32 storage
        r = 1.0 + (r - 1.0).astype(np.float32).astype(np.float64)
        u = u.astype(np.float32).astype(np.float64)
        if t in (5000, 50000):
            out[f"u_{t}"] = rel_l2(u[:, fl], ref[f"u_{t}"][:, fl])
            out[f"drho_{t}"] = rel_l2((r - 1.0)[fl], ref[f"drho_{t}"][fl])
            print(t, out, f"({time.time() - t0:.0f} s)", flush=True)
    out["seconds"] = time.time() - t0
    json.dump(out, open(OUT, "w"), indent=1)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
