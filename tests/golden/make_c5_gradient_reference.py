"""Write the FP64 oracle's gradient of the differentiable D2Q9 512x512
workload at its configured length: 2000 steps, checkpoint every 100.

Inputs (the workload recipe): seeded divergence-free fields of
``workloads.divergence_free_field`` (k <= 8, max |u| = 0.01, rho = 1; seed 0
initial, seed 1 target), omega = 1.6, loss L = sum |u_T - u*|^2.  The initial
velocity is taken after rounding to FP32, the value the GPU run starts from.
Calls only ``oracle`` (its reverse sweep with recomputation); about 2 minutes
on 8 threads.

    python tests/golden/make_c5_gradient_reference.py

writes tests/golden/c5_gradient_512_steps2000_K100.npz:
  du0, ddrho0   dL/du0 (2, 1, 512, 512) and dL/d(rho0 - 1) (1, 512, 512), float32
  domega, loss  float64 scalars
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

N, KMAX, STEPS, K, OMEGA = 512, 8, 2000, 100, 1.6
OUT = os.path.join(HERE, "c5_gradient_512_steps2000_K100.npz")


def main():
    drho, u0 = wl.divergence_free_field(N, KMAX, 0.01, seed=0)
    _, u_tgt = wl.divergence_free_field(N, KMAX, 0.01, seed=1)
    u0 = u0.astype(np.float32).astype(np.float64)
    p = oracle.Problem(q=9, nx=N, ny=N, omega=OMEGA)
    t0 = time.time()
    gr, gu, gw, (rT, uT) = oracle.gradient(
        p, 1.0 + drho, u0, STEPS, lambda r, uu: (np.zeros_like(r), 2.0 * (uu - u_tgt)), K=K)
    loss = float(((uT - u_tgt) ** 2).sum())
    print(f"{STEPS} steps, K = {K}: loss {loss:.12e}, dL/domega {gw:.12e}, "
          f"|dL/du0| {np.linalg.norm(gu):.6e} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(OUT, du0=gu.astype(np.float32), ddrho0=gr.astype(np.float32),
                        domega=np.float64(gw), loss=np.float64(loss),
                        recipe=np.array(f"n={N} kmax={KMAX} seeds=0,1 omega={OMEGA} "
                                        f"steps={STEPS} K={K} u0 rounded to FP32"))


if __name__ == "__main__":
    main()
