"""ctypes binding of ``liblwacm.so`` (the C ABI in ``include/lwacm.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  The functions
keep the C names; ``Solver`` bundles them for one problem.  There is no CPU
fallback: without the built library every call raises.
"""
import ctypes
import os
import warnings
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LWACM_LIBRARY selects another build of the same sources (the host-sanitizer
# build of tests/test_sanitizers.py); there is no other implementation
LIBRARY_PATH = os.environ.get("LWACM_LIBRARY") or os.path.join(_HERE, "liblwacm.so")

LWACM_D2Q9, LWACM_D3Q19 = 9, 19
LWACM_FP32, LWACM_FP16_DEV = 0, 1
LWACM_OK, LWACM_EINVAL, LWACM_ENOMEM, LWACM_EDEVICE, LWACM_ENONFINITE, LWACM_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5)
LWACM_ESCRATCH = -6
LWACM_WOMEGA = 1  # success with a warning: a relaxation frequency below 1
LWACM_KERNEL_AUTO, LWACM_KERNEL_GENERIC, LWACM_KERNEL_MARCH, LWACM_KERNEL_MARCH2 = 0, 1, 2, 3
LWACM_ROUND_NEAREST, LWACM_ROUND_STOCHASTIC = 0, 1

# The library's link order (the index of lwacm_init's link-wall distances d_q):
# D2Q9 is the first nine links of D3Q19.
LINK_VELOCITIES = {
    19: ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (1, 1, 0), (-1, -1, 0),
         (1, -1, 0), (-1, 1, 0), (0, 0, 1), (1, 0, 1), (-1, 0, 1), (0, 1, 1), (0, -1, 1),
         (0, 0, -1), (-1, 0, -1), (1, 0, -1), (0, -1, -1), (0, 1, -1)),
}
LINK_VELOCITIES[9] = LINK_VELOCITIES[19][:9]

_lib = None
_vp = ctypes.c_void_p


class LWACMError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lwacm_strerror(code)} ({code})")


def load_library():
    """Load liblwacm.so (torch is imported first so the HIP runtime it already
    loaded is the one the library binds to)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY_PATH):
        raise RuntimeError(f"{LIBRARY_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIBRARY_PATH)
    i, d, ll, sz = ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lwacm_state_bytes": (sz, [i, i, i, i, i]),
        "lwacm_init": (i, [ctypes.POINTER(_vp), i, i, i, i, d, i, _vp, _vp, _vp, _vp, i, _vp,
                           _vp, _vp]),
        "lwacm_set_fp16_scales": (i, [_vp, i, i]),
        "lwacm_set_fp16_rounding": (i, [_vp, i, ctypes.c_uint32]),
        "lwacm_set_variant": (i, [_vp, i]),
        "lwacm_set_march_chunk": (i, [_vp, i]),
        "lwacm_set_omega_p": (i, [_vp, ctypes.c_double]),
        "lwacm_set_force_field": (i, [_vp, _vp]),
        "lwacm_set_thermal": (i, [_vp, d, _vp, _vp, _vp, i]),
        "lwacm_set_thermal_lattice": (i, [_vp, i]),
        "lwacm_adjoint_thermal_step": (i, [_vp, _vp, _vp, _vp, _vp, _vp, i]),
        "lwacm_set_wall_velocity_links": (i, [_vp, _vp]),
        "lwacm_set_semi_implicit": (i, [_vp, i]),
        "lwacm_temperature": (i, [_vp, ctypes.POINTER(_vp)]),
        "lwacm_wall_force": (i, [_vp, i, dp, dp]),
        "lwacm_set_state": (i, [_vp, _vp, _vp]),
        "lwacm_step": (i, [_vp, i]),
        "lwacm_diagnostics": (i, [_vp, dp, dp]),
        "lwacm_set_diag_history": (i, [_vp, _vp, i]),
        "lwacm_moments": (i, [_vp, _vp, _vp, dp, dp]),
        "lwacm_save_state": (i, [_vp, _vp]),
        "lwacm_load_state": (i, [_vp, _vp, ll]),
        "lwacm_current_state": (_vp, [_vp]),
        "lwacm_step_count": (ll, [_vp]),
        "lwacm_adjoint_seed": (i, [_vp, _vp, _vp, _vp]),
        "lwacm_adjoint_step": (i, [_vp, _vp, _vp, _vp, _vp, i]),
        "lwacm_adjoint_step2": (i, [_vp, _vp, _vp, _vp, _vp, _vp, i]),
        "lwacm_forward_states": (i, [_vp, _vp, ll, i, _vp]),
        "lwacm_adjoint_sweep": (i, [_vp, _vp, ll, i, _vp, _vp, _vp]),
        "lwacm_destroy": (None, [_vp]),
        "lwacm_coefficients": (i, [d, ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(ctypes.c_float)]),
        "lwacm_step_static": (i, [i, i, i, i, d, _vp, _vp, i, _vp, ctypes.POINTER(_vp), _vp]),
        "lwacm_strerror": (ctypes.c_char_p, [i]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class LWACMOmegaWarning(UserWarning):
    """A relaxation frequency below 1: accepted, outside the range 1 <= omega < 2
    where the paper finds the method stable."""


def _check(code: int, where: str):
    if code == LWACM_WOMEGA:
        warnings.warn(f"{where}: {lwacm_strerror(code)}", LWACMOmegaWarning, stacklevel=3)
        return
    if code != LWACM_OK:
        raise LWACMError(code, where)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# ------------------------------------------------ C names, thin wrappers
def lwacm_strerror(code: int) -> str:
    return load_library().lwacm_strerror(code).decode()


def lwacm_state_bytes(lattice: int, nx: int, ny: int, nz: int, storage: int) -> int:
    return int(load_library().lwacm_state_bytes(lattice, nx, ny, nz, storage))


def lwacm_init(lattice, nx, ny, nz, omega, storage, state_a: torch.Tensor,
               state_b: torch.Tensor, mask: Optional[torch.Tensor], wall_u, g,
               stream: ctypes.c_void_p, q: Optional[torch.Tensor] = None) -> ctypes.c_void_p:
    lib = load_library()
    ctx = ctypes.c_void_p()
    wall_arr, n_ids = None, 0
    if wall_u is not None:
        flat = [float(v) for row in wall_u for v in row]
        n_ids = len(flat) // 3
        wall_arr = (ctypes.c_float * len(flat))(*flat)
    g_arr = None
    if g is not None:
        gg = list(g) + [0.0] * (3 - len(g))
        g_arr = (ctypes.c_float * 3)(*gg)
    code = lib.lwacm_init(ctypes.byref(ctx), lattice, nx, ny, nz, float(omega), storage,
                          _ptr(state_a), _ptr(state_b), _ptr(mask),
                          ctypes.cast(wall_arr, _vp) if wall_arr is not None else None, n_ids,
                          _ptr(q), ctypes.cast(g_arr, _vp) if g_arr is not None else None, stream)
    _check(code, "lwacm_init")
    return ctx


def lwacm_set_fp16_scales(ctx, k_rho: int, k_u: int):
    _check(load_library().lwacm_set_fp16_scales(ctx, k_rho, k_u), "lwacm_set_fp16_scales")


def lwacm_set_fp16_rounding(ctx, mode: int, seed: int = 0):
    _check(load_library().lwacm_set_fp16_rounding(ctx, mode, seed & 0xFFFFFFFF),
           "lwacm_set_fp16_rounding")


def lwacm_set_march_chunk(ctx, planes: int):
    _check(load_library().lwacm_set_march_chunk(ctx, planes), "lwacm_set_march_chunk")


def lwacm_set_omega_p(ctx, omega_p: float):
    _check(load_library().lwacm_set_omega_p(ctx, float(omega_p)), "lwacm_set_omega_p")


def lwacm_set_force_field(ctx, g: Optional[torch.Tensor]):
    """g: (D, nz, ny, nx) float32 contiguous on the solver's device, or None.
    The tensor must stay alive while it is set."""
    _check(load_library().lwacm_set_force_field(ctx, _ptr(g)), "lwacm_set_force_field")


def lwacm_set_semi_implicit(ctx, on: bool):
    _check(load_library().lwacm_set_semi_implicit(ctx, int(bool(on))), "lwacm_set_semi_implicit")


def lwacm_set_wall_velocity_links(ctx, uw: Optional[torch.Tensor]):
    """uw: (Q, D, nz, ny, nx) float32 contiguous on the solver's device (the
    library's link order), or None.  The tensor must stay alive while set."""
    _check(load_library().lwacm_set_wall_velocity_links(ctx, _ptr(uw)),
           "lwacm_set_wall_velocity_links")


def lwacm_set_thermal(ctx, omega_t: float, T_a: Optional[torch.Tensor],
                      T_b: Optional[torch.Tensor], wall_T: Optional[Sequence[float]] = None):
    """T_a, T_b: two (nz, ny, nx) float32 contiguous tensors on the solver's
    device (T_a holds T now), kept alive while set; both None switch the
    temperature off.  wall_T[m]: temperature of the walls with mask id m
    (NaN: adiabatic)."""
    arr, n = None, 0
    if wall_T is not None:
        n = len(wall_T)
        arr = (ctypes.c_float * max(n, 1))(*[float(v) for v in wall_T])
    _check(load_library().lwacm_set_thermal(ctx, float(omega_t), _ptr(T_a), _ptr(T_b), arr, n),
           "lwacm_set_thermal")


def lwacm_set_thermal_lattice(ctx, q_t: int):
    """Temperature lattice: 0 or the flow's Q, 5 (D2Q5) under D2Q9, 7 (D3Q7)
    under D3Q19."""
    _check(load_library().lwacm_set_thermal_lattice(ctx, int(q_t)), "lwacm_set_thermal_lattice")


def lwacm_adjoint_thermal_step(ctx, state_t: torch.Tensor, T_t: torch.Tensor,
                               lamT_in: torch.Tensor, lamT_out: torch.Tensor, mu: torch.Tensor,
                               final_t0: bool):
    """Reverse mode of one temperature step: lamT_out = dL/dT_t; dL/du_t
    added to mu (the flow sweep's mu_{t-1}, or the field-major initial-state
    gradient when final_t0)."""
    _check(load_library().lwacm_adjoint_thermal_step(ctx, _ptr(state_t), _ptr(T_t), _ptr(lamT_in),
                                                     _ptr(lamT_out), _ptr(mu), int(bool(final_t0))),
           "lwacm_adjoint_thermal_step")


def lwacm_temperature(ctx) -> int:
    """Device address of the buffer holding the current T."""
    out = _vp()
    _check(load_library().lwacm_temperature(ctx, ctypes.byref(out)), "lwacm_temperature")
    return out.value


def lwacm_wall_force(ctx, wall_id: int, center=(0.0, 0.0, 0.0)):
    """(F[3], T[3]) on the walls with mask id ``wall_id`` (momentum exchange),
    torque about ``center`` (node coordinates x, y, z)."""
    c = (ctypes.c_double * 3)(*[float(v) for v in (list(center) + [0.0, 0.0, 0.0])[:3]])
    out = (ctypes.c_double * 6)()
    _check(load_library().lwacm_wall_force(ctx, int(wall_id), c, out), "lwacm_wall_force")
    return list(out[:3]), list(out[3:])


def lwacm_set_variant(ctx, variant: int):
    _check(load_library().lwacm_set_variant(ctx, variant), "lwacm_set_variant")


def lwacm_set_state(ctx, drho: torch.Tensor, u: torch.Tensor):
    _check(load_library().lwacm_set_state(ctx, _ptr(drho), _ptr(u)), "lwacm_set_state")


def lwacm_step(ctx, nsteps: int):
    _check(load_library().lwacm_step(ctx, int(nsteps)), "lwacm_step")


def lwacm_diagnostics(ctx) -> Tuple[float, float]:
    m, e = ctypes.c_double(), ctypes.c_double()
    _check(load_library().lwacm_diagnostics(ctx, ctypes.byref(m), ctypes.byref(e)),
           "lwacm_diagnostics")
    return m.value, e.value


def lwacm_set_diag_history(ctx, hist: Optional[torch.Tensor]):
    cap = 0 if hist is None else hist.numel() // 2
    _check(load_library().lwacm_set_diag_history(ctx, _ptr(hist), cap), "lwacm_set_diag_history")


def lwacm_moments(ctx, drho: Optional[torch.Tensor], u: Optional[torch.Tensor],
                  want_diagnostics: bool = True):
    lib = load_library()
    if want_diagnostics:
        m, e = ctypes.c_double(), ctypes.c_double()
        _check(lib.lwacm_moments(ctx, _ptr(drho), _ptr(u), ctypes.byref(m), ctypes.byref(e)),
               "lwacm_moments")
        return m.value, e.value
    _check(lib.lwacm_moments(ctx, _ptr(drho), _ptr(u), None, None), "lwacm_moments")
    return None


def lwacm_save_state(ctx, dst: torch.Tensor):
    _check(load_library().lwacm_save_state(ctx, _ptr(dst)), "lwacm_save_state")


def lwacm_load_state(ctx, src: torch.Tensor, step: int):
    _check(load_library().lwacm_load_state(ctx, _ptr(src), int(step)), "lwacm_load_state")


def lwacm_current_state(ctx) -> int:
    return int(load_library().lwacm_current_state(ctx) or 0)


def lwacm_step_count(ctx) -> int:
    return int(load_library().lwacm_step_count(ctx))


def lwacm_adjoint_seed(ctx, state_T: torch.Tensor, lam_T: torch.Tensor, mu: torch.Tensor):
    _check(load_library().lwacm_adjoint_seed(ctx, _ptr(state_T), _ptr(lam_T), _ptr(mu)),
           "lwacm_adjoint_seed")


def lwacm_adjoint_step(ctx, state_t: torch.Tensor, mu_in: torch.Tensor, mu_out: torch.Tensor,
                       dL_domega: torch.Tensor, final_t0: bool):
    _check(load_library().lwacm_adjoint_step(ctx, _ptr(state_t), _ptr(mu_in), _ptr(mu_out),
                                             _ptr(dL_domega), int(bool(final_t0))),
           "lwacm_adjoint_step")


def lwacm_adjoint_step2(ctx, state_t: torch.Tensor, state_tm1: torch.Tensor, mu_in: torch.Tensor,
                        mu_out: torch.Tensor, dL_domega: torch.Tensor, final_t0: bool) -> bool:
    """Two reverse steps in one launch; False (nothing done) where the two-step
    kernel does not apply, so the caller runs lwacm_adjoint_step twice."""
    code = load_library().lwacm_adjoint_step2(ctx, _ptr(state_t), _ptr(state_tm1), _ptr(mu_in),
                                              _ptr(mu_out), _ptr(dL_domega), int(bool(final_t0)))
    if code == LWACM_EUNSUPPORTED:
        return False
    _check(code, "lwacm_adjoint_step2")
    return True


def lwacm_forward_states(ctx, state0: torch.Tensor, t0: int, nsteps: int,
                         states: torch.Tensor):
    """States after steps t0 .. t0 + nsteps - 1 from state0 (step index t0)
    into consecutive slots of `states` (uint8, >= nsteps state sizes)."""
    _check(load_library().lwacm_forward_states(ctx, _ptr(state0), int(t0), int(nsteps),
                                               _ptr(states)), "lwacm_forward_states")


def lwacm_adjoint_sweep(ctx, states: torch.Tensor, t0: int, nsteps: int, mu: torch.Tensor,
                        mu_tmp: torch.Tensor, dL_domega: torch.Tensor):
    """Reverse steps t0 + nsteps - 1 .. t0 over the states in `states` (slot
    t - t0 = state_t); mu in place: mu_{t0+nsteps-1} in, mu_{t0-1} (or the
    field-major gradient when t0 == 0) out."""
    _check(load_library().lwacm_adjoint_sweep(ctx, _ptr(states), int(t0), int(nsteps), _ptr(mu),
                                              _ptr(mu_tmp), _ptr(dL_domega)),
           "lwacm_adjoint_sweep")


def lwacm_destroy(ctx):
    if ctx:
        load_library().lwacm_destroy(ctx)


def lwacm_coefficients(omega: float) -> Tuple[float, float]:
    """(a, A): the FP32 coefficients the kernels use for omega (host only)."""
    a, A = ctypes.c_float(), ctypes.c_float()
    _check(load_library().lwacm_coefficients(float(omega), ctypes.byref(a), ctypes.byref(A)),
           "lwacm_coefficients")
    return a.value, A.value


def lwacm_step_static(lattice: int, nx: int, ny: int, nz: int, omega: float,
                      state_a: torch.Tensor, state_b: torch.Tensor, nsteps: int,
                      diag: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """nsteps periodic FP32 steps with no context and no allocation; the state
    (node-interleaved FP32) starts in state_a.  Returns whichever of state_a
    and state_b holds the state after the last step.  diag: optional device
    float64 tensor of 2 elements (mass deviation, energy)."""
    if stream is None:
        stream = _stream_handle(state_a.device)
    out = _vp()
    _check(load_library().lwacm_step_static(lattice, nx, ny, nz, float(omega), _ptr(state_a),
                                            _ptr(state_b), int(nsteps), _ptr(diag),
                                            ctypes.byref(out), stream),
           "lwacm_step_static")
    return state_a if out.value == state_a.data_ptr() else state_b


# ------------------------------------------------------------- Solver
class Solver:
    """One LW-ACM problem on one GPU: owns the two state buffers (torch), the
    mask tensor and the library context; every method forwards to the C ABI.

    Fields are (nz, ny, nx) tensors for rho - 1 and (D, nz, ny, nx) for u.
    """

    def __init__(self, lattice: int, nx: int, ny: int, nz: int = 1, omega: float = 1.0,
                 storage: int = LWACM_FP32, mask: Optional[torch.Tensor] = None,
                 wall_u: Optional[Sequence[Sequence[float]]] = None,
                 g: Optional[Sequence[float]] = None, device="cuda",
                 variant: int = LWACM_KERNEL_AUTO, fp16_scales: Optional[Tuple[int, int]] = None,
                 fp16_rounding: Optional[Tuple[int, int]] = None,
                 omega_p: Optional[float] = None, qd: Optional[torch.Tensor] = None):
        load_library()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise RuntimeError("the LW-ACM library runs on a GPU only")
        self.lattice, self.nx, self.ny, self.nz = lattice, nx, ny, nz
        self.D = 2 if lattice == LWACM_D2Q9 else 3
        self.omega = float(omega)
        self.storage = storage
        nbytes = lwacm_state_bytes(lattice, nx, ny, nz, storage)
        if nbytes == 0:
            raise LWACMError(LWACM_EINVAL, "lwacm_state_bytes")
        self.state_bytes = nbytes
        self._a = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.mask = None
        if mask is not None:
            self.mask = torch.as_tensor(mask, dtype=torch.uint8).to(self.device).contiguous()
            if self.mask.numel() != nx * ny * nz:
                raise LWACMError(LWACM_EINVAL, "mask size")
        # link-wall distances (Q, nz, ny, nx) for interpolated bounce-back, kept alive here
        self.qd = None
        if qd is not None:
            self.qd = torch.as_tensor(qd, dtype=torch.float32).to(self.device).contiguous()
            if self.qd.numel() != lattice * nx * ny * nz:
                raise LWACMError(LWACM_EINVAL, "qd size")
        self.ctx = lwacm_init(lattice, nx, ny, nz, omega, storage, self._a, self._b, self.mask,
                              wall_u, g, _stream_handle(self.device), q=self.qd)
        if fp16_scales is not None:
            lwacm_set_fp16_scales(self.ctx, *fp16_scales)
        if fp16_rounding is not None:
            lwacm_set_fp16_rounding(self.ctx, *fp16_rounding)
        if omega_p is not None:
            lwacm_set_omega_p(self.ctx, omega_p)
        if variant != LWACM_KERNEL_AUTO:
            lwacm_set_variant(self.ctx, variant)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def set_state(self, drho: torch.Tensor, u: torch.Tensor):
        drho = drho.to(self.device, torch.float32).contiguous()
        u = u.to(self.device, torch.float32).contiguous()
        if drho.numel() != self.nx * self.ny * self.nz or u.numel() != self.D * drho.numel():
            raise LWACMError(LWACM_EINVAL, "set_state sizes")
        lwacm_set_state(self.ctx, drho, u)

    def step(self, n: int = 1):
        lwacm_step(self.ctx, n)

    def set_force_field(self, g: Optional[torch.Tensor]):
        """Node-by-node acceleration (D, nz, ny, nx) for the following steps, or
        None; the solver keeps the FP32 copy it passes alive while it is set."""
        if g is not None:
            g = g.to(self.device, torch.float32).contiguous()
            if g.numel() != self.D * self.nx * self.ny * self.nz:
                raise LWACMError(LWACM_EINVAL, "set_force_field size")
        self._g_field = g
        lwacm_set_force_field(self.ctx, g)

    def set_wall_velocity_links(self, uw: Optional[torch.Tensor]):
        """Wall velocities link by link (Q, D, nz, ny, nx) in the library's
        link order, or None (the per-id table); the solver keeps the FP32 copy
        it passes alive while set."""
        if uw is not None:
            uw = uw.to(self.device, torch.float32).contiguous()
            if uw.numel() != self.lattice * self.D * self.nx * self.ny * self.nz:
                raise LWACMError(LWACM_EINVAL, "set_wall_velocity_links size")
        self._uwl = uw
        lwacm_set_wall_velocity_links(self.ctx, uw)

    def set_thermal(self, omega_t: float, T: Optional[torch.Tensor],
                    wall_T: Optional[Sequence[float]] = None, q_t: int = 0):
        """Advance a temperature field T (nz, ny, nx) with every following step
        (thermal LW-ACM, relaxation omega_t) on the temperature lattice q_t
        (0: the flow's; 5 or 7: D2Q5 / D3Q7); None switches it off.  The solver
        owns the two FP32 buffers it passes to the library."""
        if T is None:
            lwacm_set_thermal(self.ctx, 1.0, None, None)
            self._T = None
            return
        T = T.to(self.device, torch.float32).contiguous()
        if T.numel() != self.nx * self.ny * self.nz:
            raise LWACMError(LWACM_EINVAL, "set_thermal size")
        a = T.clone().reshape(self.shape)
        b = torch.empty_like(a)
        lwacm_set_thermal_lattice(self.ctx, q_t)
        lwacm_set_thermal(self.ctx, omega_t, a, b, wall_T)
        self._T = (a, b)

    def wall_force(self, wall_id: int, center=(0.0, 0.0, 0.0)):
        """Force and torque (lattice units) on the walls with mask id wall_id."""
        return lwacm_wall_force(self.ctx, wall_id, center)

    def temperature(self) -> torch.Tensor:
        """A copy of T at the current step, (nz, ny, nx) float32."""
        if getattr(self, "_T", None) is None:
            raise LWACMError(LWACM_EINVAL, "temperature: no temperature field")
        addr = lwacm_temperature(self.ctx)
        cur = self._T[0] if addr == self._T[0].data_ptr() else self._T[1]
        return cur.clone()

    def moments(self, diagnostics: bool = False):
        drho = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        u = torch.empty((self.D,) + self.shape, dtype=torch.float32, device=self.device)
        diag = lwacm_moments(self.ctx, drho, u, want_diagnostics=diagnostics)
        return (drho, u, diag) if diagnostics else (drho, u)

    def diagnostics(self):
        return lwacm_diagnostics(self.ctx)

    def new_state_buffer(self) -> torch.Tensor:
        return torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)

    def save_state(self, dst: Optional[torch.Tensor] = None) -> torch.Tensor:
        dst = self.new_state_buffer() if dst is None else dst
        lwacm_save_state(self.ctx, dst)
        return dst

    def load_state(self, src: torch.Tensor, step: int = 0):
        lwacm_load_state(self.ctx, src, step)

    @property
    def step_count(self) -> int:
        return lwacm_step_count(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lwacm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
