/*
 * lwacm.h -- C ABI of the MI355X (gfx950) LW-ACM library.
 *
 * The library advances the link-wise artificial compressibility method
 * (LW-ACM; Asinari, Ohwada, Chiavazzo, Di Rienzo, arXiv:1111.2142) on the
 * D2Q9 and D3Q19 lattices.  Every node pulls the stored moments of its
 * upstream link neighbours, evaluates the link equilibria and their odd
 * parts, applies the update of Eq. ACM2.0 (Section 2.1) and sums the new
 * moments.  No populations are stored: the state is D+1 fields per node.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid: nx * ny * nz nodes (nz = 1 for D2Q9), node index
 *    ((z * ny) + y) * nx + x, x fastest.  Every axis is periodic; walls are
 *    solid nodes of the mask.
 *  - State buffers (caller-owned device memory, lwacm_state_bytes() bytes
 *    each): node-interleaved, the D+1 values of node i side by side at
 *    elements (D+1)*i .. (D+1)*i + D: rho - 1, then u_x, u_y (, u_z), so a
 *    D3Q19 node is one 16-byte (FP32) or 8-byte (FP16) access.  Callers treat
 *    the buffers as opaque (lwacm_set_state, lwacm_moments, save/load
 *    convert or copy them).  Storage LWACM_FP32 holds float; storage
 *    LWACM_FP16_DEV holds IEEE half values of (field * 2^k), with k set by
 *    lwacm_set_fp16_scales (default 14 for both).  Initial states are
 *    rounded to nearest even; step outputs are rounded stochastically by
 *    default (lwacm_set_fp16_rounding).  Arithmetic is always FP32.
 *  - FP32 field arguments (d_drho, d_u, d_lambda, d_mu) are device arrays
 *    in field-major (structure of arrays) order: d_drho has nodes floats,
 *    d_u has D * nodes (all u_x, then all u_y, ...), d_lambda and d_mu have
 *    (D+1) * nodes (field 0 first).
 *  - Every call is asynchronous on the stream given to lwacm_init unless it
 *    returns host values (stated per call).  Pointers are not retained
 *    beyond the call unless stated.
 *  - Errors: calls return LWACM_OK (0) or a negative code; no C++
 *    exception crosses the ABI.  A failed launch returns LWACM_EDEVICE.
 *    The one positive code, LWACM_WOMEGA, is a success with a warning.
 *    lwacm_strerror() names every code.
 */
#ifndef LWACM_H
#define LWACM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lwacm_ctx lwacm_ctx; /* opaque; owned by the library */

enum { LWACM_D2Q9 = 9, LWACM_D3Q19 = 19 };
enum { LWACM_FP32 = 0, LWACM_FP16_DEV = 1 };
enum {
    LWACM_OK = 0,
    LWACM_EINVAL = -1,      /* bad argument (null pointer, size, omega, mask value) */
    LWACM_ENOMEM = -2,      /* the library could not allocate its scratch */
    LWACM_EDEVICE = -3,     /* a HIP call or kernel launch failed */
    LWACM_ENONFINITE = -4,  /* mass or kinetic energy is not finite (blow-up) */
    LWACM_EUNSUPPORTED = -5, /* valid request the library does not implement */
    LWACM_ESCRATCH = -6,     /* lwacm_step_static: problem beyond its fixed scratch */
    /* Success with a warning: a relaxation frequency (omega, omega_p or
     * omega_t) below 1.  The paper finds the method stable for 1 <= omega < 2
     * (Section "Physical and lattice units", after Eq. viscosity2); smaller values are accepted and the
     * call has taken effect. */
    LWACM_WOMEGA = 1
};

/* Rounding of step outputs into FP16 storage (lwacm_set_fp16_rounding). */
enum { LWACM_ROUND_NEAREST = 0, LWACM_ROUND_STOCHASTIC = 1 };

/* Kernel selection for lwacm_set_variant (forward and reverse steps). */
enum {
    LWACM_KERNEL_AUTO = 0,    /* fastest kernels that support the problem */
    LWACM_KERNEL_GENERIC = 1, /* one thread per node, neighbours from global memory */
    LWACM_KERNEL_MARCH = 2,   /* D3Q19 z-marching tile kernels (nx % 32 == 0, ny % 16 == 0;
                                 the forward one without body force), one step per launch */
    LWACM_KERNEL_MARCH2 = 3   /* as MARCH, and the forward steps of FP32 problems two per
                                 launch (nz >= 8; no walls or halfway walls, moving or not; no
                                 interpolated walls, link velocities, body force or separate
                                 omega_p): the intermediate state stays on chip, halving the
                                 HBM bytes per update; results are bitwise those of single
                                 steps.  AUTO includes it. */
};

/* Bytes of one state buffer: (D+1) * nodes * (4 for FP32, 2 for FP16).
 * Returns 0 for an invalid lattice, size or storage. */
size_t lwacm_state_bytes(int lattice, int nx, int ny, int nz, int storage);

/*
 * Create a context for one problem, as the paper states it (Sections 2.1,
 * 2.3-2.4 and 3): lattice, grid, relaxation frequency omega (viscosity
 * nu = (1/omega - 1/2)/3, Eq. viscosity2), walls, body acceleration.
 *
 *  lattice      LWACM_D2Q9 or LWACM_D3Q19 (Appendix A).
 *  nx, ny, nz   grid size, each >= 1; nz must be 1 for D2Q9.
 *  omega        0 < omega < 2, else LWACM_EINVAL.  The paper finds LW-ACM
 *               stable for 1 <= omega < 2; 0 < omega < 1 is accepted and
 *               the call returns LWACM_WOMEGA (a success) instead of
 *               LWACM_OK.  The kernels use a = 1 - h and A = 3 h with
 *               h = 2/omega - 1 rounded as lwacm_coefficients states.
 *  storage      LWACM_FP32 or LWACM_FP16_DEV.
 *  d_state_a/b  two caller-owned device buffers of lwacm_state_bytes() bytes
 *               (the two toggled arrays); kept until lwacm_destroy.  The
 *               current state starts in d_state_a.
 *  d_mask       NULL (all fluid) or nodes uint8 values kept until destroy:
 *               0 fluid, m >= 1 a solid node whose wall moves with
 *               h_wall_u[3m .. 3m+2].  Fluid nodes next to a solid node use
 *               halfway bounce-back (Eqs. ACM2.0cbb-ACM2.0cccbb2) with the
 *               moving-wall term of Eq. ACM2.0ccccbb.  Solid nodes are
 *               never updated.  Values >= n_wall_ids (>= 2 when h_wall_u is
 *               NULL) give LWACM_EINVAL.
 *  h_wall_u     host table of n_wall_ids velocities (3 floats each), or NULL
 *               (all walls at rest); copied.  n_wall_ids <= 16.
 *  d_q          link-wall distances for interpolated bounce-back
 *               (Section "Moving complex boundaries", Eqs. ACM2.0cc and
 *               ACM2.0move), or NULL for halfway walls (q = 1/2).  Q FP32
 *               fields of nx*ny*nz values (SoA, node index as the state's),
 *               caller-owned device memory kept alive until lwacm_destroy:
 *               d_q[j*n + x] is the fraction 0 < q <= 1 of the link from the
 *               fluid node x to x + v_j at which the wall cuts it, read only
 *               where x + v_j is solid.  j is the library's link index:
 *                 0 rest, 1 (+x), 2 (-x), 3 (+y), 4 (-y), 5 (+x+y), 6 (-x-y),
 *                 7 (+x-y), 8 (-x+y), 9 (+z), 10 (+x+z), 11 (-x+z), 12 (+y+z),
 *                 13 (-y+z), 14 (-z), 15 (-x-z), 16 (+x-z), 17 (-y-z), 18 (+y-z)
 *               (D2Q9: 0..8).  For q < 1/2 the rule also takes the
 *               node x - v_j; where that node is solid too, the halfway rule
 *               is used.  D3Q19 problems the tile kernels take run there
 *               (halfway terms plus a per-step correction of the fluid nodes
 *               next to a wall, made by a small kernel over those nodes);
 *               for them d_q is read once, here, like the mask: change
 *               neither afterwards.  Other problems run on the generic kernel,
 *               which reads d_q at every step.  The reverse steps return
 *               LWACM_EUNSUPPORTED.
 *  h_g          host body acceleration g[3] (Eq. force), or NULL; copied.
 *  stream       HIP stream every call of this context is issued on.
 *
 * On success (LWACM_OK or LWACM_WOMEGA) *out holds the context; on failure
 * *out is NULL.  The call synchronises the stream once (mask validation).
 */
int lwacm_init(lwacm_ctx **out, int lattice, int nx, int ny, int nz, double omega, int storage,
               void *d_state_a, void *d_state_b, const uint8_t *d_mask, const float *h_wall_u,
               int n_wall_ids, const float *d_q, const float *h_g, hipStream_t stream);

/* The FP32 coefficients the kernels use for omega (host only, no device
 * work): a = 2 - 2/omega, the post-combine factor of Eq. ACM2.0, and
 * A = 3 (2/omega - 1), the odd-part factor of the pre-combined link term
 * (Eqs. ACM2.0b).  Both come from h = 2/omega - 1 rounded to a multiple of
 * the finest power of two q for which 1 - h and 3 h are both FP32 numbers,
 * so a = 1 - h and A = 3 h exactly and a + A/3 = 1 (a uniform state is then a
 * fixed point of the FP32 step); h moves by at most q/2 (at most 2^-23 for
 * 1 <= omega < 2).  Returns LWACM_EINVAL for a null pointer or omega outside
 * (0, 2), LWACM_WOMEGA for omega < 1, else LWACM_OK. */
int lwacm_coefficients(double omega, float *a, float *A);

/* FP16 storage scales: stored value = field * 2^k (k_rho for rho - 1, k_u for
 * u).  0 <= k <= 24.  Takes effect at the next lwacm_set_state. */
int lwacm_set_fp16_scales(lwacm_ctx *c, int k_rho, int k_u);

/* Rounding of step outputs for FP16 storage.  LWACM_ROUND_STOCHASTIC (the
 * default, seed 0) rounds |v * 2^k| up to the next FP16 magnitude when
 * F + R >= 2^13, F being the first 13 bits of its position between the two
 * neighbouring FP16 magnitudes and R the top 13 bits of a random word (the
 * rounding of gfx950's stochastic conversion).  The words of node idx =
 * (z ny + y) nx + x are (a, b, a << 13, b << 13) for rho - 1, u_x, u_y, u_z,
 * with (a, b) the pcg2d hash (Jarzynski and Olano, JCGT 2020) of
 * (idx, t ^ seed), t the index of the step that produces the state.  The
 * stored value is then unbiased (to 2^-13 of a spacing), so velocity changes
 * smaller than an FP16 spacing
 * (1e-6 per step against 1e-5 spacing in the 256^3 Taylor-Green flow) are
 * kept on average instead of being rounded away, and a recomputed step
 * draws the same bits.  LWACM_ROUND_NEAREST rounds to nearest even.
 * LWACM_EINVAL for another mode; no effect with FP32 storage. */
int lwacm_set_fp16_rounding(lwacm_ctx *c, int mode, uint32_t seed);

/* Choose the kernel (LWACM_KERNEL_*); LWACM_EUNSUPPORTED if the kernel
 * cannot run this problem. */
int lwacm_set_variant(lwacm_ctx *c, int variant);

/* Planes per workgroup of the forward D3Q19 tile kernel: 32, 64 or 128
 * (LWACM_EINVAL otherwise; LWACM_EUNSUPPORTED if the tile kernel cannot run
 * this problem).  lwacm_init picks the depth that minimises the plane steps
 * per compute unit, ceil(workgroups / CUs) * (depth + 2); this call
 * overrides it (tuning, tests).  Results do not depend on the depth. */
int lwacm_set_march_chunk(lwacm_ctx *c, int planes);

/* Separate relaxation frequency omega_p of the continuity (density) update
 * (Section "finite-difference formulation", item 3; Appendix E, where the
 * density update takes b = 2 - 2/omega_p and the momentum update keeps
 * a = 2 - 2/omega).  The density of a step is the zeroth moment of the
 * populations of Eq. ACM2.0 evaluated with omega_p: in the link update, the
 * bounce-back and the moving-wall correction alike; the momentum is their
 * first moment with omega, and u = momentum / density.  The
 * pseudo-compressibility term of the continuity equation then scales with
 * 1/nu(omega_p) (Eq. viscosity2), so nu(omega_p) > nu(omega) reduces the
 * compressibility error of under-resolved runs.  0 < omega_p < 2, else
 * LWACM_EINVAL (omega_p < 1: LWACM_WOMEGA, a success); omega_p == omega
 * (the default after lwacm_init) is the single-relaxation step; omega_p !=
 * omega with link-wall distances (d_q) or with wall velocities given link by
 * link gives LWACM_EUNSUPPORTED.  With omega_p != omega the forward step runs
 * on the single-step tile kernel (D3Q19 without walls, nz >= 8) or else on
 * the generic kernel (every lattice, walls and force allowed), never on the
 * two-step kernel, and the reverse steps return LWACM_EUNSUPPORTED.  Takes
 * effect from the next lwacm_step. */
int lwacm_set_omega_p(lwacm_ctx *c, double omega_p);

/* Body acceleration given node by node (Eq. force with a space- and
 * time-dependent g, as in the paper's generalized Taylor-Green vortex, Eq.
 * external-force).  d_g: D FP32 fields of nx*ny*nz values (SoA, node index as
 * the state's), caller-owned device memory read by every following step until
 * the next call; it replaces the uniform g of lwacm_init while set, and NULL
 * returns to that g (or to no forcing).  The step adds rho(x, t) g(x) to the
 * momentum of node x (Eq. force, with the density before the step).  A g that
 * changes in time is set before each lwacm_step(c, 1), with the field of the
 * step's starting time.  The forward step then runs on the single-step tile
 * kernel (D3Q19, nz >= 8, omega_p == omega) or else on the generic kernel,
 * never on the two-step kernel; the reverse steps return LWACM_EUNSUPPORTED
 * while a field is set.  LWACM_EINVAL for a null context. */
int lwacm_set_force_field(lwacm_ctx *c, const float *d_g);

/* Semi-implicit pressure update (Section "The main algorithm: Finite
 * difference formulation", item 2, Eq. FDcompact_si): on != 0 makes every
 * following step compute the velocity as the explicit step does and then the
 * pressure (density) from the already updated velocity field with the old
 * density, f_p(u+, v+, p): the zeroth moment of the Eq. ACM2.0 populations
 * evaluated with u+ in place of u (walls included; the forcing adds nothing
 * to it).  A second pass over the grid on the generic kernel; the mass and
 * energy of the step are those of the final state.  LWACM_EUNSUPPORTED with
 * FP16 storage, a separate omega_p, link-wall distances, link velocities or
 * a tile-kernel variant; the reverse steps return LWACM_EUNSUPPORTED while it
 * is on.  on == 0 returns to the explicit step. */
int lwacm_set_semi_implicit(lwacm_ctx *c, int on);

/* Wall velocities given link by link, for walls whose velocity varies along
 * them (a rotating cylinder: the paper's circular Couette flow, Section
 * "Circular Couette flow"), in the moving-wall term of Eq. ACM2.0ccccbb
 * (halfway walls) or Eq. ACM2.0move (with lwacm_init's d_q).
 *   d_uw  D * Q FP32 fields of nx*ny*nz values (SoA, node index as the
 *         state's), caller-owned device memory read by every following step
 *         while set: d_uw[(j * D + k) * n + x] is component k of the velocity
 *         of the wall where the link from the fluid node x to x + v_j (the
 *         library's link order, as for d_q) crosses it, in lattice units;
 *         read only where x + v_j is solid.  It replaces the per-id table of
 *         lwacm_init for every wall while set; NULL returns to the table.
 * The forward step then runs on the D3Q19 tile kernels with the per-step
 * wall correction (as with d_q; the call synchronises the stream once to
 * set it up) or else on the generic kernel; the reverse steps return
 * LWACM_EUNSUPPORTED while it is set.  lwacm_wall_force leaves wall motion
 * out (bodies at rest), so the links into the wall it is asked about must
 * carry zero velocity.  LWACM_EINVAL without a mask; LWACM_EUNSUPPORTED with
 * a separate omega_p. */
int lwacm_set_wall_velocity_links(lwacm_ctx *c, const float *d_uw);

/* Temperature advected by the flow: the thermal LW-ACM (Appendix
 * "Asymptotic analysis for energy equation", Eq. ACM2.0t with the even part
 * of Eq. feqe) on the flow's lattice (or a smaller one: see
 * lwacm_set_thermal_lattice).  Its only state is T per node; its
 * equilibrium w_i [T (1 + 3 v_i.u) + 9/2 (v_i.u)^2 - 3/2 |u|^2] has the
 * moments the appendix requires (T, T u, u u + T/3 I), u being the flow
 * velocity at the same node and time; T diffuses with
 * alpha = (1/omega_t - 1/2) / 3 (Eq. diffusivity2) and does not act on the
 * flow.  From this call on every lwacm_step also advances T by one step per
 * flow step, reading the flow state of the step's starting time.
 *   omega_t   relaxation frequency, 0 < omega_t < 2 (stable for
 *             1 <= omega_t < 2 as the appendix notes; omega_t < 1 returns
 *             LWACM_WOMEGA, a success).
 *   d_T_a, d_T_b  two distinct caller-owned device buffers of nx*ny*nz FP32
 *             values (node index as the state's), kept alive while the
 *             temperature is on; d_T_a holds T now.  Steps write them in
 *             turn: lwacm_temperature names the one holding the current T.
 *             Both NULL: the temperature is switched off.
 *   h_wall_T  host table of n_wall_T temperatures by mask id (copied), or
 *             NULL with n_wall_T = 0.  A fluid node next to a solid node
 *             with id m sends back the term it sends into the wall: with the
 *             same sign where h_wall_T[m] is NaN, m >= n_wall_T or the table
 *             is NULL (adiabatic wall), or with the opposite sign plus
 *             (2/omega_t - 1) 2 w_i h_wall_T[m] (wall at that temperature,
 *             halfway between the fluid and the solid node).  The paper
 *             gives no thermal wall rule; this halfway reading keeps a linear
 *             profile between two such walls exactly steady.  n_wall_T <= 16.
 *             Solid nodes keep their T.
 * T stays FP32 with either flow storage; with FP16 flow storage the
 * temperature step reads u from the FP16 state (its load scales).  With walls on a D3Q19 flow the call allocates
 * (once per context) and fills, on the context's stream, a table of 8 bytes
 * per node: each node's links into fixed-temperature walls and the sum of
 * 36 w_i T_w over them, which the flow kernel's fused temperature step
 * reads; LWACM_ENOMEM if it cannot.
 * LWACM_EINVAL for bad arguments, LWACM_EUNSUPPORTED with the two-step
 * kernel requested (the two-step kernel is not used while the temperature
 * is on).  The flow's reverse steps cover the flow only;
 * lwacm_adjoint_thermal_step is the temperature's. */
int lwacm_set_thermal(lwacm_ctx *c, double omega_t, float *d_T_a, float *d_T_b,
                      const float *h_wall_T, int n_wall_T);

/* The temperature lattice (Appendix "Asymptotic analysis for energy
 * equation": the number of its links may differ from the flow's, Q_t != Q).
 *   q_t  0 or the flow's Q: the flow's lattice (the default);
 *        5 under a D2Q9 flow (D2Q5) or 7 under D3Q19 (D3Q7): the rest link
 *        and the axis links, weights 1/3, 1/6 (D2Q5) and 0, 1/6 (D3Q7) -- the
 *        axis weight 1/6 is what the required second moment T/3 I fixes.
 *        These lattices cannot carry the u u part of the second moment
 *        (O(eps^2) under the diffusive scaling), so their equilibrium is
 *        w_i T (1 + 3 v_i.u), with moments T, T u and T/3 I; alpha is the
 *        same (Eq. diffusivity2), and the wall rule of lwacm_set_thermal
 *        applies link by link.  They run on the one-thread-per-node kernel.
 * May be called before or after lwacm_set_thermal; it takes effect from the
 * next step and stays until changed.  LWACM_EINVAL for any other q_t. */
int lwacm_set_thermal_lattice(lwacm_ctx *c, int q_t);

/* Reverse mode of one temperature step (not in the paper: the exact
 * derivative of the step of lwacm_set_thermal, on the lattice and walls set
 * there).  Step t advances T_t to T_{t+1} with the flow velocity u_t of
 * state_t, the input of the flow step of the same time.  Given
 * lamT_{t+1} = dL/dT_{t+1}, this call writes lamT_t = dL/dT_t through the
 * step to d_lamT_out and adds g = dL/du_t through the step to the flow's
 * reverse sweep in d_mu, in the form lwacm_adjoint_step writes there:
 *   final_t0 == 0: d_mu holds mu_{t-1} (node-interleaved); since mu_{t-1} is
 *                  linear in lambda_u, mu_R -= g . u_t / rho_t, mu_J += g / rho_t;
 *   final_t0 != 0: d_mu holds the gradient with respect to the initial
 *                  (rho - 1, u), field-major; its u fields gain g.
 * Call it after lwacm_adjoint_step for the same t (or with d_mu = the seed's
 * output for the last step, final_t0 as that step's).  Solid nodes pass
 * lamT through and add nothing.
 *   d_state_t  state_t (storage format, FP32 or FP16)
 *   d_T_t      T_t, nx*ny*nz FP32 values
 *   d_lamT_in, d_lamT_out  nx*ny*nz FP32 values each, distinct buffers
 * LWACM_EINVAL for null pointers, aliased lam buffers, or when the
 * temperature is off (lwacm_set_thermal gives omega_t and the walls'
 * temperatures).  Asynchronous on the context's stream. */
int lwacm_adjoint_thermal_step(lwacm_ctx *c, const void *d_state_t, const float *d_T_t,
                               const float *d_lamT_in, float *d_lamT_out, float *d_mu,
                               int final_t0);

/* Force and torque that the fluid exerts on the walls with mask id wall_id,
 * by momentum exchange (Section "Moving complex boundaries", Eqs. MEA3, MEA4
 * and MEA5), from the current state.  Every link j from a fluid node x to a
 * solid node x + v_j of that id contributes
 *   p_j = v_j [f*_j(x) + f**_BB(j)(x)],
 * f*_j the pre-combined population x sends into the wall and f**_BB(j) the
 * one the wall returns before post-combining: f*_j itself for halfway walls,
 * the interpolation of Eq. ACM2.0cc when lwacm_init was given d_q (bodies at
 * rest: no wall-motion term).  F = sum p_j, T = sum (x - x_c) x p_j, x the node
 * the link starts from, in lattice units (node coordinates; the hydrostatic
 * part rho/3 per wall node is included; the diffusive-scaling forms MEA6 and
 * MEA7 are the caller's).  Summed in FP64 in a fixed order.
 *   wall_id   1..255: the mask id of the body.
 *   h_center  host double[3], the point x_c (NULL: the origin).
 *   h_out     host double[6]: F_x, F_y, F_z, T_x, T_y, T_z (D2Q9: F_z = T_x =
 *             T_y = 0).
 * Synchronises the context's stream.  On its first call it allocates a small
 * device buffer and six pinned host doubles, and lists the fluid nodes next
 * to a wall (one pass over the mask, in node order); every call then visits
 * only those nodes.  LWACM_EINVAL without a mask or for a bad id or pointer,
 * LWACM_EUNSUPPORTED with FP16 storage or for an id with a non-zero wall
 * velocity (the paper states the exchange for bodies at rest). */
int lwacm_wall_force(lwacm_ctx *c, int wall_id, const double *h_center, double *h_out);

/* Device pointer of the buffer that holds T at the current step (one of the
 * two given to lwacm_set_thermal).  LWACM_EINVAL when the temperature is off. */
int lwacm_temperature(lwacm_ctx *c, float **d_T);

/* Load the state from FP32 fields (rho - 1 and u, SoA), converting to the
 * storage format, and set rho0 (the mean fluid density used by moving walls,
 * Section 3.2) to the mean of 1 + d_drho over fluid nodes.  Resets the step
 * counter.  Synchronises the stream (rho0 reduction). */
int lwacm_set_state(lwacm_ctx *c, const float *d_drho, const float *d_u);

/* Advance nsteps >= 0 time steps (Eq. ACM2.0 with forcing Eq. force and the
 * wall rules), toggling the two state buffers.  Each step also reduces the
 * mass sum(rho) and kinetic energy 1/2 sum|u|^2 of its output over fluid
 * nodes in FP64 (per-block partials, fixed-order final sum: bitwise
 * reproducible); see lwacm_diagnostics.  Where LWACM_KERNEL_MARCH2 applies,
 * pairs of steps run as one launch (an odd count starts with a single step);
 * the state, the diagnostics and the history are the same as with single
 * steps.  D2Q9 problems in FP32 storage without a diagnostics history,
 * link-wall distances, link velocities, a separate omega_p, a force field, a
 * temperature or the semi-implicit update run up to 8 steps per launch in
 * LDS (variant AUTO): the state is bitwise that of single steps, the mass and
 * energy equal to FP64 rounding.  Asynchronous. */
int lwacm_step(lwacm_ctx *c, int nsteps);

/* Mass and energy of the state after the most recent lwacm_step (host
 * doubles; synchronises the stream).  LWACM_ENONFINITE if either is not
 * finite; LWACM_EINVAL if no step ran since lwacm_set_state/load_state. */
int lwacm_diagnostics(lwacm_ctx *c, double *h_mass, double *h_energy);

/* Optional device history: step k (counted from lwacm_set_state) also writes
 * its (mass deviation sum(rho - 1), energy 1/2 sum|u|^2) over fluid nodes, in
 * FP64, to d_hist[2 * (k % capacity)].  The deviation keeps full precision;
 * the mass is it plus the number of fluid nodes.  NULL disables. */
int lwacm_set_diag_history(lwacm_ctx *c, double *d_hist, int capacity);

/* Current state as FP32 fields: d_drho (rho - 1) and d_u (either may be
 * NULL), and, if h_mass/h_energy are non-NULL, the FP64 mass sum(rho) and
 * energy 1/2 sum|u|^2 over fluid nodes (then the call synchronises and may
 * return LWACM_ENONFINITE). */
int lwacm_moments(lwacm_ctx *c, float *d_drho, float *d_u, double *h_mass, double *h_energy);

/* Copy the current state buffer (storage format) to / from caller memory of
 * lwacm_state_bytes() bytes, for checkpoints.  load_state keeps rho0 and sets
 * the step counter to `step`. */
int lwacm_save_state(lwacm_ctx *c, void *d_dst);
int lwacm_load_state(lwacm_ctx *c, const void *d_src, long long step);

/* Device pointer to the current state buffer (storage format). */
const void *lwacm_current_state(lwacm_ctx *c);

/* Steps taken since lwacm_set_state (or the value given to load_state). */
long long lwacm_step_count(lwacm_ctx *c);

/*
 * Reverse mode (not in the paper: the exact derivative of the step above).
 *
 * Notation: one forward step maps state_t to state_{t+1}; its outputs are
 * rho+ = 1 + D and u+ = J / rho+ with D = sum of link terms and J the new
 * momentum.  The reverse sweep carries mu_t = (dL/dD, dL/dJ) of step t:
 * (D+1) * nodes FP32 values, node-interleaved like the state (mu_R, mu_J of
 * node i at (D+1)*i ..), an intermediate the caller only passes along.
 * lambda_T (input of the seed) and the final gradient are field-major.
 *
 * lwacm_adjoint_seed: mu_{T-1} from the loss cotangent lambda_T = (dL/d(rho-1),
 *   dL/du) of the final state and that state (storage format):
 *   mu_R = lambda_rho - lambda_u . u / rho, mu_J = lambda_u / rho; zero on
 *   solid nodes.
 * lwacm_adjoint_step: given state_t (storage format, the input of step t)
 *   and mu_t, computes lambda_t = dL/d state_t and writes
 *     final_t0 == 0: mu_{t-1} = (lambda_rho - lambda_u . u_t / rho_t, lambda_u / rho_t)
 *     final_t0 != 0: lambda_t itself (the gradient with respect to the
 *                    initial (rho - 1, u)), field-major,
 *   and adds this step's dL/domega to *d_dL_domega (device FP64 scalar,
 *   fixed-order reduction: bitwise reproducible).  rho0 and the walls are
 *   constants of the problem.  d_mu_out must not alias d_mu_in.
 * Both are asynchronous.
 */
int lwacm_adjoint_seed(lwacm_ctx *c, const void *d_state_T, const float *d_lambda_T, float *d_mu);
int lwacm_adjoint_step(lwacm_ctx *c, const void *d_state_t, const float *d_mu_in, float *d_mu_out,
                       double *d_dL_domega, int final_t0);

/*
 * lwacm_adjoint_step2: two reverse steps in one launch (D3Q19 tile-kernel
 * grids without walls, nz >= 8; variant AUTO or MARCH2): the same result as
 *     lwacm_adjoint_step(c, d_state_t,   d_mu_in, tmp,      w, 0);
 *     lwacm_adjoint_step(c, d_state_tm1, tmp,     d_mu_out, w, final_t0);
 * (bitwise in d_mu_out; *d_dL_domega receives the same two additions where
 * both kernels split the planes among workgroups alike, nz <= 64, else the
 * same sums grouped by 128-plane chunks: equal to FP64 rounding) with
 * the intermediate mu kept on chip: 32 instead of 48 bytes of HBM per node
 * and step.  d_state_t and d_state_tm1 are the inputs of forward steps t and
 * t - 1 (storage format); d_mu_in = mu_t, node-interleaved.  final_t0: the
 * second step is step 0, write its lambda field-major.  LWACM_EUNSUPPORTED
 * (nothing launched) where the kernel does not apply; then call
 * lwacm_adjoint_step twice.  d_mu_out must not alias d_mu_in.  Asynchronous.
 */
int lwacm_adjoint_step2(lwacm_ctx *c, const void *d_state_t, const void *d_state_tm1,
                        const float *d_mu_in, float *d_mu_out, double *d_dL_domega, int final_t0);

/*
 * The two halves of a checkpointed reverse sweep over one segment, each one
 * call (the recompute-and-reverse scheme of the checkpointed gradient: a
 * state every K steps, the segment's states recomputed from it, then K
 * reverse steps).
 *
 * lwacm_forward_states: from d_state0 (storage format, the state at step
 *   index t0) runs nsteps forward steps with the context's problem and
 *   kernels and writes the state after step t0 + k (k = 0 .. nsteps - 1)
 *   to d_states + k * lwacm_state_bytes(..): the same fields as nsteps
 *   calls of lwacm_step from that state (bitwise; t0 selects the FP16
 *   stochastic-rounding words), one launch per step (with walls on the
 *   D3Q19 tile kernels, which do not rewrite solid nodes, d_state0 is first
 *   copied into every slot).  The
 *   context's own buffers, step count and diagnostics are untouched.
 *   d_state0 must not overlap d_states.  LWACM_EUNSUPPORTED with a
 *   temperature field.  Asynchronous.
 * lwacm_adjoint_sweep: nsteps reverse steps t = t0 + nsteps - 1 down to t0,
 *   d_states + (t - t0) * lwacm_state_bytes(..) holding state_t (the input
 *   of forward step t).  d_mu holds mu_{t0 + nsteps - 1} on entry and on
 *   return mu_{t0 - 1}, or, when t0 == 0, the gradient with respect to the
 *   initial (rho - 1, u), field-major (as lwacm_adjoint_step with final_t0);
 *   d_mu_tmp is scratch of the same size.  Pairs of steps run in one launch
 *   where lwacm_adjoint_step2 applies, and D2Q9 FP32 problems without
 *   link-wall distances or link velocities run up to 8 steps per launch in
 *   LDS.  The steps' dL/domega are added to *d_dL_domega after the last
 *   step, in the order separate calls add them: d_mu equals that of the
 *   separate calls bitwise, and so does *d_dL_domega except with 8 D2Q9
 *   steps per launch, whose per-step sums run over 32 x 32 tiles instead
 *   (equal to FP64 rounding).
 *   The first call for a longer sweep allocates the library's per-step
 *   partials (nsteps x blocks doubles).  Unsupported cases as
 *   lwacm_adjoint_step.  Asynchronous.
 */
int lwacm_forward_states(lwacm_ctx *c, const void *d_state0, long long t0, int nsteps,
                         void *d_states);
int lwacm_adjoint_sweep(lwacm_ctx *c, const void *d_states, long long t0, int nsteps,
                        float *d_mu, float *d_mu_tmp, double *d_dL_domega);

/* Release the library's scratch.  Caller buffers are untouched. */
void lwacm_destroy(lwacm_ctx *c);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): nsteps
 * forward steps of a periodic problem without walls or forcing in FP32
 * storage, with no context and no allocation.  The result is bitwise that of
 *     lwacm_init(lattice, nx, ny, nz, omega, LWACM_FP32, a, b, NULL, NULL, 0,
 *                NULL, NULL, stream), state in a, lwacm_step(ctx, nsteps)
 * (same kernels, same two-steps-per-launch pairing), including the FP64
 * mass and energy of the last step.
 *   lattice, nx, ny, nz, omega   as for lwacm_init (omega < 1 gives
 *               LWACM_WOMEGA after the steps ran).
 *   d_state_a   caller-owned device buffer of lwacm_state_bytes(..., LWACM_FP32)
 *               bytes holding the state, node-interleaved: rho - 1, u_x, u_y
 *               (, u_z) of node i at floats (D+1)*i ..
 *   d_state_b   a second buffer of the same size (distinct).  The steps
 *               toggle the two buffers once per launch (a launch runs one or
 *               two steps), so which of them ends with the result depends
 *               on the kernels: *h_state_out names it.
 *   d_diag      device double[2], or NULL: receives, once the call's work
 *               has run, the mass deviation sum(rho - 1) and the kinetic
 *               energy 1/2 sum|u|^2 of the last step's output (FP64,
 *               fixed-order sums; mass = nodes + d_diag[0]).
 *   h_state_out host pointer that receives d_state_a or d_state_b: the
 *               buffer holding the state after the last step (d_state_a when
 *               nsteps == 0).  The other one holds an earlier state.  May be
 *               NULL.
 *   stream      HIP stream of every launch; the call is asynchronous.
 * Scratch: the per-block partial sums live in a fixed device array of
 * 8 * 8192 + 2 doubles (about 512 KiB) that each GPU holds for the life of
 * the process; problems whose kernels need more than 8192 blocks get
 * LWACM_ESCRATCH before anything is launched (the D3Q19 tile kernels use
 * (nx/32)(ny/16)ceil(nz/depth) blocks: 256^3 needs 256).  Every call on a
 * GPU shares that GPU's array and leaves its last contents there; calls
 * that overlap in time on one GPU (other streams or threads) race on it and
 * must be serialised by the caller.  Nothing in it needs to start at zero.
 * LWACM_EINVAL for bad sizes, omega or buffers.
 */
int lwacm_step_static(int lattice, int nx, int ny, int nz, double omega, float *d_state_a,
                      float *d_state_b, int nsteps, double *d_diag, float **h_state_out,
                      hipStream_t stream);

/* Static text for an error code. */
const char *lwacm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LWACM_H */
