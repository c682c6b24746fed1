// lwacm_internal.hpp -- kernel argument blocks and launcher declarations
// shared by the kernel files and the C ABI (host side of the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lwacm {

constexpr int kMaxWallIds = 16;

// Everything a kernel needs to know about the problem, passed by value.
struct ProblemArgs {
    int Q, D, nx, ny, nz;
    long long n;             // nodes
    float a;                 // 2 - 2/omega, the post-combine factor of Eq. ACM2.0
    float A;                 // 3 (1 - a) = 3 (2/omega - 1); a + A/3 == 1 exactly in FP32
    // Separate relaxation omega_p of the density update (the continuity
    // equation): the density sums the link terms with Ap = 3 (2/omega_p - 1)
    // and the moving-wall terms wall_term_p; 0: omega_p == omega.
    int split;
    float Ap;
    float wall_term_p[kMaxWallIds][3];  // (2/omega_p - 1) * 6 * rho0 * u_w per wall id
    float g[3];              // body acceleration (Eq. force)
    const float *g_field;    // or, when set, D fields of n accelerations (SoA) node by node
    int has_force;           // g or g_field given (no two-step kernel for forced problems)
    float wall_term[kMaxWallIds][3];  // (1 - a) * 6 * rho0 * u_w per wall id (Eq. ACM2.0ccccbb)
    float wall_da[kMaxWallIds][3];  // 6 * rho0 * u_w: minus d(wall_term)/da
    float wall_u[kMaxWallIds][3];   // wall velocities u_w per wall id (0 for fluid id 0)
    float wall_scale;               // (1 - a) * 6 * rho0: wall_term = wall_scale * u_w
    float wall6rho0;                // 6 * rho0: wall_da = wall6rho0 * u_w
    float ld_scale[2];       // storage -> value: 2^-k (rho - 1, u); 1 for FP32
    float st_scale[2];       // value -> storage: 2^k
    int fp16_sr;             // FP16 storage: 1 stochastic rounding of step outputs, 0 nearest
    uint32_t sr_word;        // second pcg2d input of this step: t ^ seed
    const uint8_t *mask;     // nullptr: all fluid
    const float *qd;         // link-wall distances, Q fields of n values (SoA), or nullptr: q = 1/2
    // wall velocities link by link (Q * D fields of n values: component k of
    // link j at (j * D + k) * n + x), or nullptr: the per-id table
    const float *uwl;
    // D3Q19 tile kernels with interpolated walls or link velocities: per node
    // next to a wall, the step's whole wall term (interpolated or halfway
    // terms of its wall links, wall motion included) in units of 36 w, added
    // before normalisation; nullptr: the halfway rule with the per-id
    // moving-wall sums
    const float4 *corr;
    int march_nzc;           // planes per workgroup of the forward tile kernel (0: unused)
    // the temperature step fused into the single-step tile kernel (thermal
    // problems, march_thermal_supported): T at the step's time and one step
    // later, h = 2/omega_t - 1 and kap = 2 - 2/omega_t; T_in null: no fusion
    const float *T_in;
    float *T_out;
    float t_h, t_kap;
    // with walls: per node, the links into fixed-temperature walls (bit i) and
    // the FP32 bits of the sum of 36 w_i T_w over them (lwacm_set_thermal)
    const uint2 *T_wall;
};

// Scratch and destination of the fixed-order grid reductions: a kernel stores
// NV partial sums per block, then launch_reduce() adds them in order.
struct ReduceArgs {
    double *partials;  // NV * nblocks doubles
    double *out;       // NV doubles
    double *out2;      // optional second copy (history), may be null
    int accumulate;    // 1: out[0] += total instead of out[k] = total
    double out_scale;  // total is multiplied by this before it is written
    // Deferred second pass of the previous step (forward steps only): block 0
    // of this launch adds prev_nblocks pairs of prev_partials (stored by the
    // previous kernel) into prev_out / prev_out2.  prev_nblocks == 0: none.
    const double *prev_partials;
    unsigned prev_nblocks;
    double *prev_out;
    double *prev_out2;
    // Two-step launches (launch_fwd_march2): partials of the second step, and
    // a second deferred sum (the second step of a previous two-step launch),
    // finished after the first.  Single-step kernels ignore these fields.
    double *partials_b;
    const double *prev_partials_b;
    unsigned prev_nblocks_b;
    double *prev_out_b;
    double *prev_out2_b;
};

// Second pass of a grid reduction over nblocks blocks of NV (1 or 2) values.
hipError_t launch_reduce(const ReduceArgs &r, int nv, unsigned nblocks, hipStream_t stream);
// The block partials of several reverse steps, one slice of `stride` doubles
// each (zero-padded past the launch's own blocks, nblocks the largest count):
// *out += total_s * scale for each slice s in order, as separate calls of the
// reverse step add them.
hipError_t launch_reduce_slices(const double *partials, size_t stride, unsigned nblocks,
                                unsigned nslices, double *totals, double scale, double *out,
                                hipStream_t stream);

// The forward launchers store per-block partials only; the caller runs the
// second pass (launch_reduce, or deferred into the next step's launch).
// Generic kernels: one thread per node, neighbours read from global memory.
hipError_t launch_fwd_generic(const ProblemArgs &p, int storage, bool force, const void *src,
                              void *dst, const ReduceArgs &r, unsigned nblocks,
                              hipStream_t stream);
// Second pass of a semi-implicit step (FP32 storage): the density from the
// old density (src) and the new velocity (dst), written into dst.
hipError_t launch_density_si(const ProblemArgs &p, const float *src, float *dst,
                             const ReduceArgs &r, unsigned nblocks, hipStream_t stream);
hipError_t launch_adj_generic(const ProblemArgs &p, int storage, const void *state,
                              const float *mu_in, float *mu_out, int final_t0,
                              const ReduceArgs &r, unsigned nblocks, hipStream_t stream);
hipError_t launch_adj_seed(const ProblemArgs &p, int storage, const void *state,
                           const float *lambda, float *mu, hipStream_t stream);
hipError_t launch_set_state(const ProblemArgs &p, int storage, const float *drho,
                            const float *u, void *dst, hipStream_t stream);
hipError_t launch_moments(const ProblemArgs &p, int storage, const void *src, float *drho,
                          float *u, const ReduceArgs &r, unsigned nblocks, hipStream_t stream);
hipError_t launch_mask_scan(const ProblemArgs &p, unsigned *d_out2, hipStream_t stream);

// D3Q19 z-marching tile kernel.  Masked problems also need the per-node
// classes and solid-upstream bit sets made by launch_classify (n bytes and
// n unsigned).  Returns hipErrorNotSupported if the problem does not fit.
bool march_supported(const ProblemArgs &p);
int march_choose_nzc(const ProblemArgs &p, int ncu);  // chunk depth for a device of ncu CUs
unsigned march_num_blocks(const ProblemArgs &p);       // uses p.march_nzc
// Moving walls also need a per-node float4 of geometry sums (wallg, n
// entries; may be null when every wall is at rest).
constexpr unsigned kMovingWallFlag = 1u << 31;  // in bits: node sees a moving wall
hipError_t launch_classify(const ProblemArgs &p, uint8_t *cls, unsigned *bits, float4 *wallg,
                           hipStream_t s);
// D3Q19 reverse step as a z-marching tile kernel (any mask, with or without
// force); mu_in / mu_out node-interleaved, or field-major output when
// final_t0.  Masked problems need the bit sets (and wallg for moving walls)
// of launch_classify.
bool adj_march_supported(const ProblemArgs &p);
unsigned adj_march_num_blocks(const ProblemArgs &p);
hipError_t launch_adj_march(const ProblemArgs &p, int storage, const void *state,
                            const float *mu_in, float *mu_out, const unsigned *bits,
                            const float4 *wallg, int final_t0, const ReduceArgs &r,
                            hipStream_t stream);
// D3Q19 single-step tile kernel with the temperature step in the same pass
// (p.T_in, p.T_out): FP32 or FP16 state, no walls or halfway walls (with the
// table p.T_wall), no force, omega_p or wall correction.
bool march_thermal_supported(const ProblemArgs &p);
hipError_t launch_fwd_march(const ProblemArgs &p, int storage, const void *src, void *dst,
                            const uint8_t *cls, const unsigned *bits, const float4 *wallg,
                            const ReduceArgs &r, hipStream_t stream);
// Two D3Q19 reverse steps per launch (steps t and t - 1, unmasked, nz >= 8):
// mu_in = mu_t, state_t and state_tm1 the inputs of forward steps t and
// t - 1; writes mu_{t-2}, or the field-major gradient when final_t0.  Stores
// the two steps' dL/da partials in r.partials and r.partials_b (one double
// per block each) and adds them to r.out in that order.
bool adj_march2_supported(const ProblemArgs &p);
unsigned adj_march2_num_blocks(const ProblemArgs &p);
hipError_t launch_adj_march2(const ProblemArgs &p, int storage, const void *state_t,
                             const void *state_tm1, const float *mu_in, float *mu_out,
                             int final_t0, const ReduceArgs &r, hipStream_t stream);
// Two D3Q19 forward steps per launch on FP32 state (same tiles as the
// single-step kernel, its chunk depth halved while deeper than nz; halfway
// walls (bb_bits and wallg from k_classify), no body force, no separate
// omega_p, no per-step wall correction, nz >= 8).  Stores the first step's
// partials in r.partials and the second step's in r.partials_b (2 doubles
// per block each); finishes up to two deferred sums of earlier steps.
bool march2_supported(const ProblemArgs &p);
unsigned march2_num_blocks(const ProblemArgs &p);
hipError_t launch_fwd_march2(const ProblemArgs &p, const float *src, float *dst,
                             const unsigned *bb_bits, const float4 *wallg, const ReduceArgs &r,
                             hipStream_t stream);

// Several D2Q9 steps per launch (FP32 storage; no link-wall distances, link
// velocities, omega_p or force field): 32 x 32 output tiles, up to
// kMultiSteps steps per launch in LDS, one partial pair per tile.
constexpr int kMultiTile = 32;
constexpr int kMultiSteps = 8;
bool d2q9_multi_supported(const ProblemArgs &p);
unsigned d2q9_multi_num_blocks(const ProblemArgs &p);
// Up to kMultiSteps D2Q9 reverse steps per launch (FP32, the forward
// multi-step kernel's problems): forward-step states in caller slots of
// slot_floats floats, slot slot_hi for the first (latest) step, the rest
// below it; mu node-interleaved in and out (field-major lambda out when
// final_last: the last step is step 0); each step's per-workgroup dL/da in
// partials[(slice0 + s) * stride + block] (blocks: d2q9_multi_num_blocks).
hipError_t launch_adj_d2q9_multi(const ProblemArgs &p, const float *states, size_t slot_floats,
                                 int slot_hi, int ksteps, int final_last, const float *mu_in,
                                 float *mu_out, double *partials, size_t stride, unsigned slice0,
                                 hipStream_t s);
// slots non-null: the state after each of the ksteps steps goes to slots +
// s * slot_floats (s = 0 .. ksteps - 1) instead of the last one to dst.
hipError_t launch_fwd_d2q9_multi(const ProblemArgs &p, const float *src, float *dst, int ksteps,
                                 const ReduceArgs &r, hipStream_t stream, float *slots = nullptr,
                                 size_t slot_floats = 0);

// Number of blocks the generic grid-stride kernels use for n nodes.
unsigned generic_grid(long long n);

constexpr int kGenericBlock = 256;
constexpr unsigned kGenericMaxBlocks = 4096;

}  // namespace lwacm
