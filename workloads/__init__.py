"""Seeded synthetic inputs for LW-ACM runs: initial fields, wall masks, seeds.

Shared by the tests, the benchmark and the smoke check on both sides of every
comparison (the HIP library and the CPU oracle).  Nothing here evaluates the
method: it only builds the analytic initial fields and geometries of the
paper's kind of workload (low-Mach periodic vortices, channels and cavities on
uniform grids; Sections 3.1-3.2), in float64 numpy arrays.

Array convention: ``drho`` (= rho - 1) has shape (nz, ny, nx) (nz = 1 in 2D),
``u`` has shape (D, nz, ny, nx), x fastest.
"""
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

# Wall ids used in masks: 0 is fluid, 1 a wall at rest, 2 a moving wall.
FLUID, WALL, MOVING_WALL = 0, 1, 2


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def taylor_green_2d(n: int, u0: float, ny: Optional[int] = None):
    """2D Taylor-Green vortex u = -u0 cos kx sin ky, v = u0 sin kx cos ky, rho = 1.

    k = 2 pi / n on node coordinates x = i (the decaying vortex of the
    configs; the paper's forced variant is Eq. exactsolution without forcing).
    """
    ny = n if ny is None else ny
    x, y, _ = _grid(n, ny, 1)
    kx, ky = 2 * np.pi / n, 2 * np.pi / ny
    u = np.stack([-u0 * np.cos(kx * x) * np.sin(ky * y), u0 * np.sin(kx * x) * np.cos(ky * y)])
    return np.zeros((1, ny, n)), u


def taylor_green_3d(n: int, u0: float):
    """3D Taylor-Green vortex u = u0 sin kx cos ky cos kz, v = -u0 cos kx sin ky cos kz, w = 0."""
    x, y, z = _grid(n, n, n)
    k = 2 * np.pi / n
    u = np.stack([u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z),
                  -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z),
                  np.zeros_like(x)])
    return np.zeros((n, n, n)), u


def shear_wave(shape: Tuple[int, int, int], d: int, u0: float, m: int = 1):
    """u_x = u0 sin(2 pi m y / ny), other components zero, rho = 1."""
    nz, ny, nx = shape
    _, y, _ = _grid(nx, ny, nz)
    u = np.zeros((d,) + shape)
    u[0] = u0 * np.sin(2 * np.pi * m * y / ny)
    return np.zeros(shape), u


def channel_mask(nx: int, ny: int, moving_top: bool = False):
    """2D channel: rows y = 0 and y = ny-1 solid (walls half a link outside
    the outermost fluid rows), periodic in x.  ``moving_top`` marks the top
    row with the moving-wall id."""
    m = np.zeros((1, ny, nx), dtype=np.uint8)
    m[0, 0, :] = WALL
    m[0, ny - 1, :] = MOVING_WALL if moving_top else WALL
    return m


def slab_mask_3d(nx: int, ny: int, nz: int, moving_top: bool = False):
    """3D channel between the planes y = 0 and y = ny-1 (solid), periodic in x and z."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:, 0, :] = WALL
    m[:, ny - 1, :] = MOVING_WALL if moving_top else WALL
    return m


def cavity_mask(n: int):
    """Cubic lid-driven cavity on an n^3 array: the six boundary planes are
    solid, the whole top plane z = n-1 (edges included, the lid-corner rule)
    is the moving lid; (n-2)^3 fluid nodes."""
    m = np.full((n, n, n), WALL, dtype=np.uint8)
    m[1:n - 1, 1:n - 1, 1:n - 1] = FLUID
    m[n - 1, :, :] = MOVING_WALL
    return m


def wall_table(u_moving=(0.0, 0.0, 0.0)):
    """Wall velocities by mask id: id 0 unused (fluid), id 1 at rest, id 2 moving."""
    t = np.zeros((3, 3))
    t[MOVING_WALL, :len(u_moving)] = u_moving
    return t


def divergence_free_field(n: int, kmax: int, amplitude: float, seed: int):
    """Seeded random divergence-free 2D field on an n x n periodic grid.

    Stream function psi = sum_k a_k cos(2 pi k.x / n + phi_k) over integer
    wavevectors 0 < |k| <= kmax in a half plane, a_k ~ N(0,1) and
    phi_k ~ U[0, 2 pi) from numpy's PCG64 with the given seed; u = d psi/dy,
    v = -d psi/dx taken analytically, then scaled so max |u| = amplitude.
    rho = 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, _ = _grid(n, n, 1)
    ks = []
    for kx in range(0, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            if kx == 0 and ky <= 0:
                continue
            if kx * kx + ky * ky <= kmax * kmax:
                ks.append((kx, ky))
    u = np.zeros((2, 1, n, n))
    for kx, ky in ks:
        a = rng.standard_normal()
        phi = rng.uniform(0.0, 2 * np.pi)
        arg = 2 * np.pi * (kx * x + ky * y) / n + phi
        s = -a * np.sin(arg) * 2 * np.pi / n
        u[0] += s * ky
        u[1] -= s * kx
    speed = np.sqrt(u[0] ** 2 + u[1] ** 2).max()
    u *= amplitude / speed
    return np.zeros((1, n, n)), u


def double_shear_layer(n: int, u0: float, k: float = 80.0, delta: float = 0.05):
    """The doubly periodic shear layer the paper uses to show the separate
    omega_p (Section on the Minion & Brown test): on the unit square,
    u = tanh(k (y - 1/4)) for y <= 1/2 and tanh(k (3/4 - y)) above, v = delta
    sin(2 pi (x + 1/4)), both scaled by the lattice velocity u0; node i sits at
    i / n.  rho = 1."""
    x, y, _ = _grid(n, n, 1)
    xs, ys = x / n, y / n
    u = np.zeros((2, 1, n, n))
    u[0] = u0 * np.where(ys <= 0.5, np.tanh(k * (ys - 0.25)), np.tanh(k * (0.75 - ys)))
    u[1] = u0 * delta * np.sin(2 * np.pi * (xs + 0.25))
    return np.zeros((1, n, n)), u


class ForcedTaylorGreen:
    """The generalized Taylor-Green vortex of the paper (its section of that
    name): a time-periodic flow kept up by an external acceleration, on the
    periodic square [0, 2 pi]^2 with (u0, v0) = (0.3, 0.6) and nu = 0.1, in
    diffusive scaling (dx = eps, dt = eps^2, Table "scaling").  Node i sits at
    i eps, N = 2 pi / eps nodes per side; lattice velocity u = eps u_bar,
    pressure p_bar = (rho/3 - p0) / eps^2 with p0 the mean, acceleration
    g = eps^3 g_bar, omega from nu (Eq. viscosity2)."""

    u0, v0, nu = 0.3, 0.6, 0.1

    def __init__(self, m: int):
        self.eps = np.pi / m          # eps = pi/16, pi/32, pi/64 in the paper's table
        self.n = 2 * m
        self.omega = omega_for_viscosity(self.nu)
        idx = np.arange(self.n) * self.eps
        self.x, self.y = np.meshgrid(idx, idx, indexing="xy")  # [y, x]

    def steps_to(self, t: float) -> int:
        return int(round(t / self.eps ** 2))

    def exact(self, t: float):
        """(u_bar, v_bar, p_bar) of the analytic solution at time t."""
        a, b = self.x - self.u0 * t, self.y - self.v0 * t
        u = self.u0 + np.sin(a) * np.cos(b) * np.cos(t)
        v = self.v0 - np.cos(a) * np.sin(b) * np.cos(t)
        p = 0.25 * (np.cos(2 * a) + np.cos(2 * b)) * np.cos(t) ** 2
        return u, v, p

    def initial_state(self):
        """(drho (1, n, n), u (2, 1, n, n)) in lattice units at t = 0."""
        ub, vb, pb = self.exact(0.0)
        drho = (3.0 * self.eps ** 2 * pb)[None]
        u = np.stack([self.eps * ub, self.eps * vb])[:, None]
        return drho, u

    def acceleration(self, step: int):
        """Lattice acceleration field (2, 1, n, n) of the step that starts at
        t = step eps^2 (Eq. force takes g at the current time level)."""
        t = step * self.eps ** 2
        a, b = self.x - self.u0 * t, self.y - self.v0 * t
        f = 2.0 * self.nu * np.cos(t) - np.sin(t)
        e3 = self.eps ** 3
        return np.stack([e3 * np.sin(a) * np.cos(b) * f, -e3 * np.cos(a) * np.sin(b) * f])[:, None]

    def l1_errors(self, step: int, drho, u):
        """Mean absolute errors of (u_bar, v_bar, p_bar) over the nodes after
        `step` steps (lattice state drho (1, n, n), u (2, 1, n, n))."""
        ue, ve, pe = self.exact(step * self.eps ** 2)
        r = 1.0 + np.asarray(drho, dtype=np.float64)[0]
        p = r / 3.0
        pnum = (p - p.mean()) / self.eps ** 2
        uu = np.asarray(u, dtype=np.float64)
        return (float(np.abs(uu[0, 0] / self.eps - ue).mean()),
                float(np.abs(uu[1, 0] / self.eps - ve).mean()),
                float(np.abs(pnum - pe).mean()))


class CircularCouette:
    """Flow between two concentric cylinders on a D2Q9 grid (the paper's
    Section "Circular Couette flow"): the inner cylinder (radius r_i) at rest,
    the outer one (radius r_e) turning at angular velocity 1/r_e, so its wall
    moves at speed 1; nu = 0.07 in physical units; diffusive scaling with grid
    spacing eps = Ma (lattice velocity = eps x physical velocity, lattice time
    step eps^2).

    Geometry only: node (i, j) sits at the physical point
    X = (i + 1/2 - n/2) eps, Y = (j + 1/2 - n/2) eps, so the common axis lies
    between nodes; nodes with r <= r_i are solid with mask id 1 (at rest),
    nodes with r >= r_e solid with id 2 (turning), the rest fluid.  For every
    fluid node x and link v_j with x + v_j solid, q_j(x) is the fraction of
    the link at which it meets the circle (the root in (0, 1] of
    |x + t v_j eps| = r), and uw_j(x) the wall velocity at that point in
    lattice units: eps / r_e (-P_y, P_x) on the outer cylinder, 0 on the
    inner one.
    """

    NU = 0.07

    def __init__(self, eps: float, r_i: float = 0.5, r_e: float = 1.0):
        self.eps, self.r_i, self.r_e = float(eps), float(r_i), float(r_e)
        self.n = 2 * int(np.ceil(self.r_e / self.eps + 2.0))
        n = self.n
        c = (np.arange(n, dtype=np.float64) + 0.5 - n / 2.0) * self.eps
        self.X, self.Y = np.meshgrid(c, c, indexing="xy")  # (ny, nx)
        self.R = np.hypot(self.X, self.Y)
        mask = np.zeros((1, n, n), dtype=np.uint8)
        mask[0][self.R <= self.r_i] = 1
        mask[0][self.R >= self.r_e] = 2
        self.mask = mask
        self.fluid = mask[0] == 0
        # diffusive scaling: lattice viscosity = physical viscosity
        self.omega = 1.0 / (3.0 * self.NU + 0.5)
        self.C = 1.0 / (self.r_e / self.r_i - self.r_i / self.r_e)
        self.center = ((n - 1) / 2.0, (n - 1) / 2.0, 0.0)  # node coordinates of the axis

    def steps_to(self, t: float) -> int:
        return int(round(t / self.eps ** 2))

    def links(self, velocities):
        """(qd, uwl) for the given link velocities (sequence of (vx, vy[, vz])):
        qd (Q, 1, n, n) and uwl (Q, 2, 1, n, n); 0 where the link stays in
        the fluid."""
        n, eps = self.n, self.eps
        Q = len(velocities)
        qd = np.zeros((Q, 1, n, n))
        uwl = np.zeros((Q, 2, 1, n, n))
        fy, fx = np.nonzero(self.fluid)
        for j, v in enumerate(velocities):
            vx, vy = int(v[0]), int(v[1])
            if vx == 0 and vy == 0:
                continue
            tx, ty = fx + vx, fy + vy
            solid = self.mask[0, ty, tx]
            sel = solid != 0
            x0, y0 = self.X[fy[sel], fx[sel]], self.Y[fy[sel], fx[sel]]
            r = np.where(solid[sel] == 1, self.r_i, self.r_e)
            a = (vx * vx + vy * vy) * eps * eps
            b = 2.0 * eps * (x0 * vx + y0 * vy)
            cc = x0 * x0 + y0 * y0 - r * r
            disc = np.sqrt(b * b - 4.0 * a * cc)
            # inner cylinder: the link enters the circle (smaller root);
            # outer cylinder: it leaves the disc r < r_e (larger root)
            t = np.where(solid[sel] == 1, (-b - disc) / (2.0 * a), (-b + disc) / (2.0 * a))
            qd[j, 0, fy[sel], fx[sel]] = t
            px, py = x0 + t * vx * eps, y0 + t * vy * eps
            om = np.where(solid[sel] == 2, eps / self.r_e, 0.0)
            uwl[j, 0, 0, fy[sel], fx[sel]] = -om * py
            uwl[j, 1, 0, fy[sel], fx[sel]] = om * px
        return qd, uwl


def random_state(shape: Tuple[int, int, int], d: int, seed: int, du: float = 0.05,
                 drho: float = 0.02):
    """Uniform random (drho, u) perturbations of the rest state (for algebraic
    checks that must hold for any state)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.uniform(-drho, drho, size=shape), rng.uniform(-du, du, size=(d,) + shape))


@dataclass(frozen=True)
class Config:
    """One workload: lattice, grid, omega, walls, force, initial field, steps."""
    name: str
    q: int
    nx: int
    ny: int
    nz: int
    omega: float
    steps: int
    u0: float = 0.0
    g: Optional[Tuple[float, float, float]] = None
    lid: Optional[Tuple[float, float, float]] = None

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz


def viscosity(omega: float) -> float:
    """nu = (1/omega - 1/2)/3, Eq. viscosity2 (for setting omega from a Reynolds number)."""
    return (1.0 / omega - 0.5) / 3.0


def omega_for_viscosity(nu: float) -> float:
    """Inverse of Eq. viscosity2."""
    return 1.0 / (3.0 * nu + 0.5)


# The five workloads (sizes and parameters as stated for the runs).
TGV2D_64 = Config("d2q9_tgv_64x64", 9, 64, 64, 1, 1.6, 1000, u0=0.01)
CHANNEL_256x64 = Config("d2q9_channel_256x64", 9, 256, 64, 1, 1.0, 20000, g=(1e-6, 0.0, 0.0))
TGV3D_256 = Config("d3q19_tgv_256^3", 19, 256, 256, 256, 1.7, 1000, u0=0.02)
# Lid-driven cube: 192^3 array, 190^3 fluid, Re = u_lid L / nu = 1000 with L = 190.
CAVITY_192 = Config("d3q19_cavity_192^3", 19, 192, 192, 192,
                    omega_for_viscosity(0.05 * 190 / 1000.0), 50000, lid=(0.05, 0.0, 0.0))
CAVITY_48 = Config("d3q19_cavity_48^3", 19, 48, 48, 48,
                   omega_for_viscosity(0.05 * 46 / 1000.0), 50000, lid=(0.05, 0.0, 0.0))
ADJOINT_512 = Config("d2q9_adjoint_512x512", 9, 512, 512, 1, 1.6, 2000, u0=0.01)
