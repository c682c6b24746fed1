"""Error measures of the circular Couette flow (Section "Circular Couette
flow") against its exact steady solution, shared by the oracle pins and the
GPU tests.

Exact solution (Eqs. circcouttesol and circcouttesolC), inner cylinder at
rest, outer cylinder turning at angular velocity 1/r_e:
  u_theta(r) = C (r/r_i - r_i/r),  C = 1 / (r_e/r_i - r_i/r_e),
  p(r) = p_i + C^2 ln(r_i^2/r^2) - C^2/2 (r_i^2/r^2 - r^2/r_i^2),
  torque on the inner cylinder = 4 pi C nu r_i (per unit length, rho = 1).

Readings of the printed error table (the paper does not state them): the L1
error of a field is the mean absolute error over fluid nodes (as for the
generalized Taylor-Green table); the pressure is compared with the mean over
fluid nodes removed from both sides (p_i is free); the physical velocity is
u / eps and the physical pressure (rho/3 - p0) / eps^2 (Table "tab:scaling");
the physical torque equals the lattice one (same table), whose hydrostatic
part cancels over the whole cylinder.
"""
import numpy as np


def exact(cc):
    """(u_theta, p) at the nodes of the geometry cc (physical units, p up to a
    constant; values at non-fluid nodes are meaningless) and the torque."""
    r = np.where(cc.fluid, cc.R, 1.0)
    C, ri = cc.C, cc.r_i
    ut = C * (r / ri - ri / r)
    p = C ** 2 * np.log(ri ** 2 / r ** 2) - 0.5 * C ** 2 * (ri ** 2 / r ** 2 - r ** 2 / ri ** 2)
    return ut, p, 4.0 * np.pi * C * cc.NU * ri


def l1_errors(cc, rho, u, torque_z):
    """L1 errors (u_theta, p, |T|) of a lattice state (rho (1, n, n), u (2, 1,
    n, n), float64) and the lattice z-torque on the inner cylinder."""
    f = cc.fluid
    X, Y, R = cc.X[f], cc.Y[f], cc.R[f]
    ux, uy = u[0, 0][f] / cc.eps, u[1, 0][f] / cc.eps
    ut = (-Y * ux + X * uy) / R
    ut_ex, p_ex, t_ex = exact(cc)
    e_u = float(np.abs(ut - ut_ex[f]).mean())
    pn = rho[0][f] / 3.0 / cc.eps ** 2
    pn = pn - pn.mean()
    pe = p_ex[f] - p_ex[f].mean()
    e_p = float(np.abs(pn - pe).mean())
    e_t = float(abs(abs(torque_z) - t_ex))
    return e_u, e_p, e_t
