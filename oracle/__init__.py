"""Plain FP64 CPU oracle of the LW-ACM time step (arXiv:1111.2142).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; the product library never
imports, links or calls it.  It shares no code with the HIP library.

The arithmetic lives in ``lwacm_oracle.c`` (population form of Eq. ACM2.0,
odd parts from their definition Eq. feqo, forcing Eq. force, halfway
bounce-back Eqs. ACM2.0cbb-ACM2.0cccbb2 and moving walls Eq. ACM2.0ccccbb,
reverse mode by the chain rule).  This module only marshals numpy arrays and
strings the per-step calls together:

* ``run``        -- n forward steps (two arrays toggled);
* ``diagnostics``-- mass sum(rho) and energy 1/2 sum|u|^2 over fluid nodes;
* ``vjp``        -- reverse mode of one step;
* ``gradient``   -- reverse sweep over n steps with a checkpoint every K
                    steps and recomputation in between;
* ``thermal_step`` -- one step of the temperature lattice (Eq. ACM2.0t)
                    advected by a given flow velocity;
* ``thermal_vjp`` -- reverse mode of one temperature step;
* ``step_q``     -- one step with link-wall distances (interpolated
                    bounce-back) and, optionally, wall velocities per link.

Arrays: ``rho`` has shape (nz, ny, nx) (nz = 1 for D2Q9), ``u`` has shape
(D, nz, ny, nx); float64, C order (x fastest).
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Callable, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LWACM_ORACLE_LIB selects another build of the same source (the sanitizer
# build of tests/test_sanitizers.py)
_LIBPATH = os.environ.get("LWACM_ORACLE_LIB") or os.path.join(_HERE, "liblwacm_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    common = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
              _u8p, _dp, ctypes.c_int, _dp, ctypes.c_double]
    lib.oracle_step.argtypes = common + [_dp, _dp, _dp, _dp]
    lib.oracle_step.restype = ctypes.c_int
    lib.oracle_step_split.argtypes = common[:5] + [ctypes.c_double] + common[5:] + [_dp, _dp, _dp,
                                                                                     _dp]
    lib.oracle_step_split.restype = ctypes.c_int
    lib.oracle_step_field.argtypes = common[:8] + [_dp, ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.oracle_step_field.restype = ctypes.c_int
    lib.oracle_step_q.argtypes = common + [_dp, _dp, _dp, _dp, _dp]
    lib.oracle_step_q.restype = ctypes.c_int
    lib.oracle_step_qw.argtypes = common + [_dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_step_qw.restype = ctypes.c_int
    lib.oracle_step_si.argtypes = common[:9] + [_dp, ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.oracle_step_si.restype = ctypes.c_int
    lib.oracle_vjp.argtypes = common + [_dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_vjp.restype = ctypes.c_int
    lib.oracle_step_nodes.argtypes = common + [_dp, _dp, ctypes.POINTER(ctypes.c_long),
                                               ctypes.c_long, _dp, _dp]
    lib.oracle_step_nodes.restype = ctypes.c_int
    lib.oracle_thermal_step.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, _u8p, _dp,
                                                            ctypes.c_int, _dp, _dp, _dp]
    lib.oracle_thermal_step.restype = ctypes.c_int
    lib.oracle_thermal_vjp.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, _u8p, _dp,
                                                            ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_thermal_vjp.restype = ctypes.c_int
    lib.oracle_thermal_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
    lib.oracle_thermal_equilibrium.restype = ctypes.c_int
    lib.oracle_wall_force.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, _u8p, _dp, _dp, _dp,
                                                          ctypes.c_int, _dp, _dp]
    lib.oracle_wall_force.restype = ctypes.c_int
    lib.oracle_diagnostics.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       _u8p, _dp, _dp, _dp, _dp]
    lib.oracle_diagnostics.restype = ctypes.c_int
    lib.oracle_lattice_info.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), _dp,
                                        ctypes.POINTER(ctypes.c_int)]
    lib.oracle_lattice_info.restype = ctypes.c_int
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_round_fp16_sr.argtypes = [ctypes.c_double, ctypes.c_uint32]
    lib.oracle_round_fp16_sr.restype = ctypes.c_double
    lib.oracle_store_fp16_sr.argtypes = [ctypes.c_int] * 4 + [ctypes.c_uint32] * 2 + \
        [ctypes.c_int] * 2 + [_dp, _dp]
    lib.oracle_store_fp16_sr.restype = ctypes.c_int
    lib.oracle_sr_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32, u32p]
    lib.oracle_sr_words.restype = None
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray], p=_dp):
    if a is None:
        return ctypes.cast(None, p)
    return a.ctypes.data_as(p)


def num_threads() -> int:
    """Threads the oracle's parallel loops use (OMP_NUM_THREADS)."""
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's parallel loops from now on."""
    _load().oracle_set_num_threads(int(n))


def lattice_info(q: int):
    """(D, velocities (q,3) int, weights (q,), opposite (q,)) of the oracle's lattice."""
    lib = _load()
    d = ctypes.c_int()
    v = (ctypes.c_int * (3 * q))()
    w = (ctypes.c_double * q)()
    opp = (ctypes.c_int * q)()
    if lib.oracle_lattice_info(q, ctypes.byref(d), v, w, opp) != 0:
        raise ValueError(f"unknown lattice Q={q}")
    return (d.value, np.array(v[:], dtype=np.int64).reshape(q, 3), np.array(w[:]),
            np.array(opp[:], dtype=np.int64))


@dataclass
class Problem:
    """What the paper's statement of a run fixes: lattice, grid, omega, walls, force."""
    q: int                     # 9 (D2Q9) or 19 (D3Q19)
    nx: int
    ny: int
    nz: int = 1
    omega: float = 1.0
    mask: Optional[np.ndarray] = None     # uint8 (nz,ny,nx); 0 fluid, m>=1 wall id
    wall_u: Optional[np.ndarray] = None   # (n_ids, 3) wall velocities by id
    g: Optional[Tuple[float, ...]] = None  # body acceleration
    rho0: float = 1.0          # mean fluid density at t=0, used by moving walls
    omega_p: Optional[float] = None  # separate relaxation of the density (None: omega)

    @property
    def d(self) -> int:
        return 2 if self.q == 9 else 3

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def _args(self):
        mask = None
        if self.mask is not None:
            mask = np.ascontiguousarray(self.mask, dtype=np.uint8)
            assert mask.shape == self.shape
        wall = None
        n_ids = 0
        if self.wall_u is not None:
            wall = np.ascontiguousarray(self.wall_u, dtype=np.float64).reshape(-1, 3)
            n_ids = wall.shape[0]
            wall = wall.reshape(-1)
        g = None
        if self.g is not None:
            g = np.zeros(3)
            g[:len(self.g)] = self.g
        self._keep = (mask, wall, g)
        return [self.q, self.nx, self.ny, self.nz, float(self.omega), _ptr(mask, _u8p),
                _ptr(wall), n_ids, _ptr(g), float(self.rho0)]


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _step_call(lib, p: Problem, args, rho_in, u_in, rho_out, u_out):
    """oracle_step, or oracle_step_split when the problem has its own omega_p."""
    if p.omega_p is None:
        return lib.oracle_step(*args, _ptr(rho_in), _ptr(u_in), _ptr(rho_out), _ptr(u_out))
    split = args[:5] + [float(p.omega_p)] + args[5:]
    return lib.oracle_step_split(*split, _ptr(rho_in), _ptr(u_in), _ptr(rho_out), _ptr(u_out))


def step(p: Problem, rho, u):
    """One step of Eq. ACM2.0 (with forcing, walls and, if given, a separate
    omega_p for the density); returns new (rho, u)."""
    lib = _load()
    rho = _f64(rho, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    r1 = np.empty_like(rho)
    u1 = np.empty_like(u)
    rc = _step_call(lib, p, p._args(), rho, u, r1, u1)
    if rc != 0:
        raise RuntimeError(f"oracle_step failed ({rc})")
    return r1, u1


def step_field(p: Problem, rho, u, g_field):
    """One step with a node-by-node body acceleration g_field (D, nz, ny, nx)
    (the problem's uniform g and omega_p are not used); returns new (rho, u)."""
    lib = _load()
    rho = _f64(rho, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    g = _f64(g_field, (p.d,) + p.shape)
    r1 = np.empty_like(rho)
    u1 = np.empty_like(u)
    args = p._args()
    rc = lib.oracle_step_field(*args[:8], _ptr(g), args[9], _ptr(rho), _ptr(u), _ptr(r1),
                               _ptr(u1))
    if rc != 0:
        raise RuntimeError(f"oracle_step_field failed ({rc})")
    return r1, u1


def step_si(p: Problem, rho, u, g_field=None):
    """One step with the semi-implicit pressure update (Eq. FDcompact_si): the
    explicit step's velocity, then the density from the old density and the
    new velocity.  g_field (D, nz, ny, nx) replaces the problem's uniform g
    when given.  Returns new (rho, u)."""
    lib = _load()
    rho = _f64(rho, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    gf = None if g_field is None else _f64(g_field, (p.d,) + p.shape)
    r1 = np.empty_like(rho)
    u1 = np.empty_like(u)
    a = p._args()
    rc = lib.oracle_step_si(*a[:9], _ptr(gf), a[9], _ptr(rho), _ptr(u), _ptr(r1), _ptr(u1))
    if rc != 0:
        raise RuntimeError(f"oracle_step_si failed ({rc})")
    return r1, u1


def step_q(p: Problem, rho, u, qd, uwl=None):
    """One step with link-wall distances qd (Q, nz, ny, nx): qd[j] at node x is
    the fraction of the link x -> x + v_j at which the wall cuts it (read where
    x + v_j is solid; None: q = 1/2).  uwl (Q, D, nz, ny, nx), if given, is the
    velocity of the wall where that link crosses it, in place of the per-id
    table.  Returns new (rho, u)."""
    lib = _load()
    rho = _f64(rho, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    qd = None if qd is None else _f64(qd, (p.q,) + p.shape)
    uwl = None if uwl is None else _f64(uwl, (p.q, p.d) + p.shape)
    r1 = np.empty_like(rho)
    u1 = np.empty_like(u)
    rc = lib.oracle_step_qw(*p._args(), _ptr(qd), _ptr(uwl), _ptr(rho), _ptr(u), _ptr(r1),
                            _ptr(u1))
    if rc != 0:
        raise RuntimeError(f"oracle_step_q failed ({rc})")
    return r1, u1


def thermal_step(p: Problem, T, u, omega_t: float, wall_T=None, qt=None):
    """One step of the temperature lattice (Eq. ACM2.0t) on the problem's
    grid and mask, advected by the flow velocity u (D, nz, ny, nx) at the
    same time; wall_T[m] is the temperature of the walls with mask id m
    (NaN or ids past the end: adiabatic; None: all adiabatic).  qt: the
    temperature lattice, None for the problem's own, 5 (D2Q5) under D2Q9 or
    7 (D3Q7) under D3Q19.  Returns T at the next step."""
    lib = _load()
    T = _f64(T, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    mask = None if p.mask is None else np.ascontiguousarray(p.mask, dtype=np.uint8)
    wt = None if wall_T is None else np.ascontiguousarray(wall_T, dtype=np.float64).reshape(-1)
    out = np.empty_like(T)
    q = p.q if qt is None else int(qt)
    if q not in (p.q, 5 if p.q == 9 else 7):
        raise ValueError(f"temperature lattice Q={q} under a Q={p.q} flow")
    rc = lib.oracle_thermal_step(q, p.nx, p.ny, p.nz, float(omega_t), _ptr(mask, _u8p),
                                 _ptr(wt), 0 if wt is None else len(wt), _ptr(T), _ptr(u),
                                 _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_thermal_step failed ({rc})")
    return out


def thermal_vjp(p: Problem, T, u, lam, omega_t: float, wall_T=None, qt=None):
    """Reverse mode of one temperature step (thermal_step's arguments) for the
    cotangent lam = dL/dT(t+1): returns (dL/dT(t), dL/du(t)) through that
    step, u's cotangent of shape (D, nz, ny, nx)."""
    lib = _load()
    T = _f64(T, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    lam = _f64(lam, p.shape)
    mask = None if p.mask is None else np.ascontiguousarray(p.mask, dtype=np.uint8)
    wt = None if wall_T is None else np.ascontiguousarray(wall_T, dtype=np.float64).reshape(-1)
    q = p.q if qt is None else int(qt)
    if q not in (p.q, 5 if p.q == 9 else 7):
        raise ValueError(f"temperature lattice Q={q} under a Q={p.q} flow")
    lt = np.empty_like(T)
    lu = np.empty_like(u)
    rc = lib.oracle_thermal_vjp(q, p.nx, p.ny, p.nz, float(omega_t), _ptr(mask, _u8p), _ptr(wt),
                                0 if wt is None else len(wt), _ptr(T), _ptr(u), _ptr(lam),
                                _ptr(lt), _ptr(lu))
    if rc != 0:
        raise RuntimeError(f"oracle_thermal_vjp failed ({rc})")
    return lt, lu


def wall_force(p: Problem, rho, u, wall_id: int, center=(0.0, 0.0, 0.0), qd=None):
    """Force and torque on the walls with mask id ``wall_id`` by momentum
    exchange (Eqs. MEA3-MEA5) at the state (rho, u); qd as in step_q.
    Returns (F[3], T[3]) in lattice units, torque about ``center`` (node
    coordinates x, y, z)."""
    lib = _load()
    rho = _f64(rho, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    mask = np.ascontiguousarray(p.mask, dtype=np.uint8)
    q = None if qd is None else _f64(qd, (p.q,) + p.shape)
    c = np.zeros(3)
    c[:len(center)] = center
    out = np.empty(6)
    rc = lib.oracle_wall_force(p.q, p.nx, p.ny, p.nz, float(p.omega), _ptr(mask, _u8p), _ptr(q),
                               _ptr(rho), _ptr(u), int(wall_id), _ptr(c), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_wall_force failed ({rc})")
    return out[:3].copy(), out[3:].copy()


def thermal_equilibrium(q: int, T: float, u):
    """(g^(e)_i, g^(e,e)_i), i = 0..q-1, of the temperature lattice q (5, 7,
    9 or 19) at (T, u)."""
    lib = _load()
    uu = np.zeros(3)
    uu[:len(u)] = u
    g = np.empty(q)
    ge = np.empty(q)
    if lib.oracle_thermal_equilibrium(q, float(T), _ptr(uu), _ptr(g), _ptr(ge)) != 0:
        raise ValueError(f"unknown lattice Q={q}")
    return g, ge


def step_nodes(p: Problem, rho, u, idx):
    """One step evaluated only at the flat node indices ``idx``.

    Returns (rho_new[len(idx)], u_new[D, len(idx)]).
    """
    if p.omega_p is not None:
        raise NotImplementedError("step_nodes: no separate omega_p")
    lib = _load()
    rho = _f64(rho, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    r = np.empty(len(idx))
    uu = np.empty((len(idx), p.d))
    rc = lib.oracle_step_nodes(*p._args(), _ptr(rho), _ptr(u),
                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(idx),
                               _ptr(r), _ptr(uu))
    if rc != 0:
        raise RuntimeError(f"oracle_step_nodes failed ({rc})")
    return r, np.ascontiguousarray(uu.T)


def run(p: Problem, rho, u, nsteps: int, callback: Optional[Callable] = None):
    """n forward steps; ``callback(t, rho, u)`` after each step if given."""
    lib = _load()
    a_r = _f64(rho, p.shape).copy()
    a_u = _f64(u, (p.d,) + p.shape).copy()
    b_r = np.empty_like(a_r)
    b_u = np.empty_like(a_u)
    args = p._args()
    for t in range(nsteps):
        rc = _step_call(lib, p, args, a_r, a_u, b_r, b_u)
        if rc != 0:
            raise RuntimeError(f"oracle_step failed ({rc})")
        a_r, b_r = b_r, a_r
        a_u, b_u = b_u, a_u
        if callback is not None:
            callback(t + 1, a_r, a_u)
    return a_r, a_u


def sr_words(idx: int, w: int):
    """The four field words of node idx at step word w = t ^ seed: (a, b,
    a << 13, b << 13) with (a, b) the pcg2d hash of (idx, w)."""
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_sr_words(int(idx) & 0xFFFFFFFF, int(w) & 0xFFFFFFFF,
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def round_fp16_sr(y: float, r: int) -> float:
    """Stochastic rounding of the real y to an IEEE half value, random word r."""
    return float(_load().oracle_round_fp16_sr(float(y), int(r) & 0xFFFFFFFF))


def store_fp16_sr(p: Problem, t: int, rho, u, seed: int = 0, k_rho: int = 14, k_u: int = 14):
    """(rho, u) as FP16 storage with stochastic rounding holds the output of
    step t: rho - 1 and u scaled by 2^k, rounded, scaled back.  Returns copies."""
    rho = _f64(rho, p.shape).copy()
    u = _f64(u, (p.d,) + p.shape).copy()
    rc = _load().oracle_store_fp16_sr(p.q, p.nx, p.ny, p.nz, int(t) & 0xFFFFFFFF,
                                      int(seed) & 0xFFFFFFFF, k_rho, k_u, _ptr(rho), _ptr(u))
    if rc:
        raise ValueError("oracle_store_fp16_sr: bad lattice")
    return rho, u


def diagnostics(p: Problem, rho, u):
    """(mass, energy) = (sum rho, 1/2 sum |u|^2) over fluid nodes."""
    lib = _load()
    rho = _f64(rho, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    m = ctypes.c_double()
    e = ctypes.c_double()
    mask = None if p.mask is None else np.ascontiguousarray(p.mask, dtype=np.uint8)
    lib.oracle_diagnostics(p.q, p.nx, p.ny, p.nz, _ptr(mask, _u8p), _ptr(rho), _ptr(u),
                           ctypes.byref(m), ctypes.byref(e))
    return m.value, e.value


def vjp(p: Problem, rho, u, lam_rho1, lam_u1):
    """Reverse mode of one step entered with state (rho, u).

    Returns (lam_rho0, lam_u0, dL_domega) for output cotangents (lam_rho1, lam_u1).
    """
    if p.omega_p is not None:
        raise NotImplementedError("vjp: no separate omega_p")
    lib = _load()
    rho = _f64(rho, p.shape)
    u = _f64(u, (p.d,) + p.shape)
    lr1 = _f64(lam_rho1, p.shape)
    lu1 = _f64(lam_u1, (p.d,) + p.shape)
    lr0 = np.empty_like(rho)
    lu0 = np.empty_like(u)
    dw = ctypes.c_double()
    rc = lib.oracle_vjp(*p._args(), _ptr(rho), _ptr(u), _ptr(lr1), _ptr(lu1), _ptr(lr0),
                        _ptr(lu0), ctypes.byref(dw))
    if rc != 0:
        raise RuntimeError(f"oracle_vjp failed ({rc})")
    return lr0, lu0, dw.value


def gradient(p: Problem, rho0, u0, nsteps: int, final_cotangent: Callable, K: int = 100):
    """Gradient of a final-state loss through ``nsteps`` steps.

    ``final_cotangent(rho_T, u_T) -> (lam_rho_T, lam_u_T)`` gives dL/d(state_T).
    The reverse sweep keeps a checkpoint every K steps and recomputes the
    states of one segment at a time.  Returns (dL/drho0, dL/du0, dL/domega,
    (rho_T, u_T)).
    """
    rho = _f64(rho0, p.shape).copy()
    u = _f64(u0, (p.d,) + p.shape).copy()
    checkpoints = {}
    for t0 in range(0, nsteps, K):
        checkpoints[t0] = (rho.copy(), u.copy())
        rho, u = run(p, rho, u, min(K, nsteps - t0))
    lam_r, lam_u = final_cotangent(rho, u)
    lam_r = _f64(lam_r, p.shape)
    lam_u = _f64(lam_u, (p.d,) + p.shape)
    dw_total = 0.0
    for t0 in sorted(checkpoints, reverse=True):
        nseg = min(K, nsteps - t0)
        states = [checkpoints[t0]]
        for _ in range(nseg - 1):
            states.append(step(p, *states[-1]))
        for s in reversed(states):
            lam_r, lam_u, dw = vjp(p, s[0], s[1], lam_r, lam_u)
            dw_total += dw
    return lam_r, lam_u, dw_total, (rho, u)
