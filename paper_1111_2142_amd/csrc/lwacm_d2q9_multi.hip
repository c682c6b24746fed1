// lwacm_d2q9_multi.hip -- several D2Q9 steps per launch (temporal blocking).
//
// The 2D workloads are small (64^2 to 512^2 nodes: under a microsecond of
// HBM time per step), so one launch per step is bound by the interval between
// dependent launches (about 4 us on this device), not by the step.  Here a
// workgroup owns a 32 x 32 tile of output nodes, loads the tile and a halo of
// K nodes on every side (periodic wrap) into LDS once, and advances the
// region K steps in LDS: step s is computed on the region less s nodes on
// each side, which is exactly what the next step needs, so after K steps the
// tile is exact.  Each node is updated by the same function as the one-step
// kernel (link_update in lwacm_generic_update.hpp), so the fields are bitwise
// those of K single steps.  The mass and energy of the last step are summed
// per workgroup in FP64 (a different order than the one-step kernel's, so
// equal to FP64 rounding only).
//
// FP32 storage, halfway walls with the per-id table, uniform force; problems
// with link-wall distances, link velocities, a separate omega_p, a force
// field, the semi-implicit update, a temperature or a diagnostics history run
// one step per launch.
#include "lwacm_device.hpp"
#include "lwacm_generic_update.hpp"
#include "lwacm_internal.hpp"

namespace lwacm {

namespace {

constexpr int MT = kMultiTile;       // output tile side
constexpr int MK = kMultiSteps;      // halo width = most steps per launch
constexpr int MW = MT + 2 * MK;      // region side
constexpr int MTHREADS = 1024;       // 32 x 32 threads

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    int m = v % n;
    return m < 0 ? m + n : m;
}

constexpr int MR = 2;  // rows per thread: a strip of MR nodes shares its neighbours' loads

template <bool MASK, bool FORCE>
__global__ __launch_bounds__(MTHREADS) void k_fwd_d2q9_multi(ProblemArgs p, const float *__restrict__ src,
                                                             float *__restrict__ dst, int ksteps,
                                                             ReduceArgs r, float *__restrict__ slots,
                                                             size_t slot_floats)
{
    // per node of the region, two steps' buffers: (rho - 1, u_x, u_y, w) with
    // w = node_B(u) <= -0 at a fluid node (computed once where the node is
    // written, not at each of its eight readers) and w = mask id >= 1 at a
    // solid node
    __shared__ float4 buf[2][MW * MW];
    const int ntx = (p.nx + MT - 1) / MT;
    const int tile_x0 = (int)(blockIdx.x % ntx) * MT;
    const int tile_y0 = (int)(blockIdx.x / ntx) * MT;
    const int tid = threadIdx.x;

    // region load: node (lx, ly) of the region is global node
    // (tile_x0 - MK + lx, tile_y0 - MK + ly) wrapped; every thread issues all
    // of its loads before the first LDS store, so their latencies overlap
    constexpr int NL = (MW * MW + MTHREADS - 1) / MTHREADS;
    float4 v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int j = tid + k * MTHREADS;
        if (j < MW * MW) {
            const int ly = j / MW, lx = j - (j / MW) * MW;
            const int gx = wrap_mod(tile_x0 - MK + lx, p.nx);
            const int gy = wrap_mod(tile_y0 - MK + ly, p.ny);
            const long long g = (long long)gy * p.nx + gx;
            v[k] = make_float4(src[3 * g], src[3 * g + 1], src[3 * g + 2],
                               MASK ? (float)p.mask[g] : 0.0f);
        }
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int j = tid + k * MTHREADS;
        if (j < MW * MW) {
            const float u[3] = {v[k].y, v[k].z, 0.0f};
            buf[0][j] = make_float4(v[k].x, u[0], u[1], v[k].w > 0.0f ? v[k].w : node_B(u));
        }
    }
    __syncthreads();

    // step s computes the region's rows and columns [s, MW - s), an even
    // number m of them, as m / 2 x m work items of MR = 2 nodes of one
    // column (a strip), numbered row of strips by row of strips so that a
    // wave's lanes take neighbouring columns; the strip's 3 x 4
    // neighbourhood is read from LDS once and kept in registers
    static_assert(MR == 2 && MW % 2 == 0, "strips of two rows tile every step's square");
    for (int s = 1; s <= ksteps; ++s) {
        const int b0 = (s - 1) & 1, b1 = s & 1;
        const int m = MW - 2 * s;
        const int items = (m / MR) * m;
        // item / m in FP32: (item + 1/2) / m lies at least 1/(2m) from an
        // integer and m <= 46, far above the rounding of the product
        const float inv_m = 1.0f / (float)m;
        for (int it = tid; it < items; it += MTHREADS) {
            const int strip = (int)(((float)it + 0.5f) * inv_m);
            const int lx = s + (it - strip * m);
            const int ly0 = s + strip * MR;
            float4 w[MR + 2][3];
#pragma unroll
            for (int rr = 0; rr < MR + 2; ++rr)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    w[rr][cc] = buf[b0][(ly0 - 1 + rr) * MW + lx - 1 + cc];
#pragma unroll
            for (int rr = 0; rr < MR; ++rr) {
                const int ly = ly0 + rr;
                const int l = ly * MW + lx;
                const float4 own = w[rr + 1][1];
                // slots: every step's state goes out, tile node by tile node
                const int sgx = tile_x0 - MK + lx, sgy = tile_y0 - MK + ly;
                const bool put = slots && lx >= MK && lx < MK + MT && ly >= MK && ly < MK + MT &&
                                 sgx < p.nx && sgy < p.ny;
                float *const so = put ? slots + (size_t)(s - 1) * slot_floats +
                                            3 * ((size_t)sgy * p.nx + sgx)
                                      : nullptr;
                if (MASK && own.w > 0.0f) {  // solid: unchanged
                    buf[b1][l] = own;
                    if (put) {
                        so[0] = own.x;
                        so[1] = own.y;
                        so[2] = own.z;
                    }
                    continue;
                }
                const float ux[3] = {own.y, own.z, 0.0f};
                auto fmask = [&](int dx, int dy, int) -> uint8_t {
                    const float v = w[rr + 1 + dy][1 + dx].w;
                    return (MASK && v > 0.0f) ? (uint8_t)v : (uint8_t)0;
                };
                auto fstate = [&](int dx, int dy, int, float &dr, float (&u)[3], float &B) {
                    const float4 v = w[rr + 1 + dy][1 + dx];
                    dr = v.x;
                    u[0] = v.y;
                    u[1] = v.z;
                    u[2] = 0.0f;
                    B = v.w;
                };
                const long long gidx = (long long)wrap_mod(tile_y0 - MK + ly, p.ny) * p.nx +
                                       wrap_mod(tile_x0 - MK + lx, p.nx);
                float out[3], e;
                link_update<9, MASK, FORCE, false>(p, gidx, own.x, ux, own.w, fmask, fstate, out, e);
                const float un[3] = {out[1], out[2], 0.0f};
                buf[b1][l] = make_float4(out[0], out[1], out[2], node_B(un));
                if (put) {
                    so[0] = out[0];
                    so[1] = out[1];
                    so[2] = out[2];
                }
            }
        }
        __syncthreads();
    }

    // the tile's nodes after ksteps steps, and their mass and energy
    const int bf = ksteps & 1;
    double acc[2] = {0.0, 0.0};
    for (int j = tid; j < MT * MT; j += MTHREADS) {
        const int oy = j / MT, ox = j - (j / MT) * MT;
        const int gx = tile_x0 + ox, gy = tile_y0 + oy;
        if (gx >= p.nx || gy >= p.ny) continue;
        const float4 v = buf[bf][(oy + MK) * MW + (ox + MK)];
        const long long g = (long long)gy * p.nx + gx;
        if (!slots) {  // with slots the last step's state is already out
            dst[3 * g] = v.x;
            dst[3 * g + 1] = v.y;
            dst[3 * g + 2] = v.z;
        }
        if (MASK && v.w > 0.0f) continue;
        float e = 0.0f;
        e = fmaf(v.y, v.y, e);
        e = fmaf(v.z, v.z, e);
        acc[0] += (double)v.x;
        acc[1] += 0.5 * (double)e;
    }
    store_block_partials<2>(acc, r.partials, blockIdx.x);
    if (blockIdx.x == 0 && r.prev_nblocks)
        finish_previous_sums(r.prev_partials, r.prev_nblocks, r.prev_out, r.prev_out2);
}

// Several D2Q9 reverse steps per launch, the same temporal blocking: the
// region's mu (with the mask id) is loaded into LDS once; reverse step s (the
// forward step of slot slot_hi - s + 1 of the caller's state slots) is
// computed on the region less s nodes on each side from the node's own state,
// read from its slot, and the mu of its neighbours y + v_k in LDS.  Each node
// goes through adj_node_update, as in the one-step reverse kernel, so mu is
// bitwise that of ksteps single reverse steps.  Each step's dL/da of the
// tile's nodes is summed per workgroup into slice slice0 + s - 1 of the
// partials (a different order of addition than the one-step kernel's blocks):
// per wave during the step, over the waves after the last step, so a step
// ends with a single barrier.
// final_last: the last step is step 0, its lambda goes out field-major.
template <bool MASK>
__global__ __launch_bounds__(MTHREADS) void k_adj_d2q9_multi(ProblemArgs p,
                                                             const float *__restrict__ states,
                                                             size_t slot_floats, int slot_hi,
                                                             int ksteps, int final_last,
                                                             const float *__restrict__ mu_in,
                                                             float *__restrict__ mu_out,
                                                             double *__restrict__ partials,
                                                             size_t stride, unsigned slice0)
{
    // per node of the region, two steps' buffers: (mu_R, mu_Jx, mu_Jy, mask id)
    __shared__ float4 buf[2][MW * MW];
    // each step's dL/da per wave, added up after the last step
    constexpr int NWAVES = MTHREADS / kWave;
    __shared__ double stepsum[MK][NWAVES];
    const int ntx = (p.nx + MT - 1) / MT;
    const int tile_x0 = (int)(blockIdx.x % ntx) * MT;
    const int tile_y0 = (int)(blockIdx.x / ntx) * MT;
    const int tid = threadIdx.x;

    constexpr int NL = (MW * MW + MTHREADS - 1) / MTHREADS;
    float4 v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int j = tid + k * MTHREADS;
        if (j < MW * MW) {
            const int ly = j / MW, lx = j - (j / MW) * MW;
            const long long g = (long long)wrap_mod(tile_y0 - MK + ly, p.ny) * p.nx +
                                wrap_mod(tile_x0 - MK + lx, p.nx);
            v[k] = make_float4(mu_in[3 * g], mu_in[3 * g + 1], mu_in[3 * g + 2],
                               MASK ? (float)p.mask[g] : 0.0f);
        }
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int j = tid + k * MTHREADS;
        if (j < MW * MW) buf[0][j] = v[k];
    }
    __syncthreads();

    static_assert(MR == 2 && MW % 2 == 0, "strips of two rows tile every step's square");
    for (int s = 1; s <= ksteps; ++s) {
        const int b0 = (s - 1) & 1, b1 = s & 1;
        const bool fin = final_last && s == ksteps;
        const float *st = states + (size_t)(slot_hi - s + 1) * slot_floats;
        const int m = MW - 2 * s;
        const int items = (m / MR) * m;
        const float inv_m = 1.0f / (float)m;
        double da_sum = 0.0;
        for (int it = tid; it < items; it += MTHREADS) {
            const int strip = (int)(((float)it + 0.5f) * inv_m);
            const int lx = s + (it - strip * m);
            const int ly0 = s + strip * MR;
            float4 w[MR + 2][3];
#pragma unroll
            for (int rr = 0; rr < MR + 2; ++rr)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    w[rr][cc] = buf[b0][(ly0 - 1 + rr) * MW + lx - 1 + cc];
#pragma unroll
            for (int rr = 0; rr < MR; ++rr) {
                const int ly = ly0 + rr;
                const int l = ly * MW + lx;
                const float4 own = w[rr + 1][1];
                const int gx = tile_x0 - MK + lx, gy = tile_y0 - MK + ly;
                const bool tile = lx >= MK && lx < MK + MT && ly >= MK && ly < MK + MT &&
                                  gx < p.nx && gy < p.ny;
                const long long g = (long long)wrap_mod(gy, p.ny) * p.nx + wrap_mod(gx, p.nx);
                if (MASK && own.w != 0.0f) {  // solid: mu (or lambda) zero
                    if (fin) {
                        if (tile) mu_out[g] = mu_out[p.n + g] = mu_out[2 * p.n + g] = 0.0f;
                    } else {
                        buf[b1][l] = make_float4(0.0f, 0.0f, 0.0f, own.w);
                    }
                    continue;
                }
                const float uy[3] = {st[3 * g + 1], st[3 * g + 2], 0.0f};
                const float dry = st[3 * g];
                const float muJ[3] = {own.y, own.z, 0.0f};
                auto fmask = [&](int dx, int dy, int) -> uint8_t {
                    return MASK ? (uint8_t)w[rr + 1 + dy][1 + dx].w : (uint8_t)0;
                };
                auto fmu = [&](int dx, int dy, int, float &mr, float (&mt)[3]) {
                    const float4 q = w[rr + 1 + dy][1 + dx];
                    mr = q.x;
                    mt[0] = q.y;
                    mt[1] = q.z;
                    mt[2] = 0.0f;
                };
                float lr, lu[3], da;
                adj_node_update<9, MASK>(p, dry, uy, own.x, muJ, fmask, fmu, lr, lu, da);
                if (tile) da_sum += (double)da;
                if (fin) {
                    if (tile) {
                        mu_out[g] = lr;
                        mu_out[p.n + g] = lu[0];
                        mu_out[2 * p.n + g] = lu[1];
                    }
                } else {
                    float mR, mJ[3];
                    adj_fold<2>(dry, uy, lr, lu, mR, mJ);
                    buf[b1][l] = make_float4(mR, mJ[0], mJ[1], own.w);
                }
            }
        }
        // the wave's sum now; the sum over the waves, in wave order (the
        // order of block_sum), after the last step, one thread per step
        const double wsum = wave_sum(da_sum);
        if ((tid & (kWave - 1)) == 0) stepsum[s - 1][tid / kWave] = wsum;
        __syncthreads();  // ends the step
    }
    if (tid < ksteps) {
        double sum = 0.0;
        for (int w = 0; w < NWAVES; ++w) sum += stepsum[tid][w];
        partials[(size_t)(slice0 + tid) * stride + blockIdx.x] = sum;
    }

    if (!final_last) {
        const int bf = ksteps & 1;
        for (int j = tid; j < MT * MT; j += MTHREADS) {
            const int oy = j / MT, ox = j - (j / MT) * MT;
            const int gx = tile_x0 + ox, gy = tile_y0 + oy;
            if (gx >= p.nx || gy >= p.ny) continue;
            const float4 q = buf[bf][(oy + MK) * MW + (ox + MK)];
            const long long g = (long long)gy * p.nx + gx;
            mu_out[3 * g] = q.x;
            mu_out[3 * g + 1] = q.y;
            mu_out[3 * g + 2] = q.z;
        }
    }
}

}  // namespace

bool d2q9_multi_supported(const ProblemArgs &p)
{
    return p.Q == 9 && p.nz == 1 && !p.qd && !p.uwl && !p.split && !p.g_field && p.nx >= 1 &&
           p.ny >= 1;
}

unsigned d2q9_multi_num_blocks(const ProblemArgs &p)
{
    return (unsigned)(((long long)(p.nx + MT - 1) / MT) * ((p.ny + MT - 1) / MT));
}

hipError_t launch_adj_d2q9_multi(const ProblemArgs &p, const float *states, size_t slot_floats,
                                 int slot_hi, int ksteps, int final_last, const float *mu_in,
                                 float *mu_out, double *partials, size_t stride, unsigned slice0,
                                 hipStream_t s)
{
    if (!d2q9_multi_supported(p) || ksteps < 1 || ksteps > MK || slot_hi < ksteps - 1)
        return hipErrorInvalidValue;
    const unsigned nb = d2q9_multi_num_blocks(p);
    if (p.mask)
        k_adj_d2q9_multi<true><<<nb, MTHREADS, 0, s>>>(p, states, slot_floats, slot_hi, ksteps,
                                                       final_last, mu_in, mu_out, partials, stride,
                                                       slice0);
    else
        k_adj_d2q9_multi<false><<<nb, MTHREADS, 0, s>>>(p, states, slot_floats, slot_hi, ksteps,
                                                        final_last, mu_in, mu_out, partials,
                                                        stride, slice0);
    return hipGetLastError();
}

hipError_t launch_fwd_d2q9_multi(const ProblemArgs &p, const float *src, float *dst, int ksteps,
                                 const ReduceArgs &r, hipStream_t s, float *slots,
                                 size_t slot_floats)
{
    if (!d2q9_multi_supported(p) || ksteps < 1 || ksteps > MK) return hipErrorInvalidValue;
    const unsigned nb = d2q9_multi_num_blocks(p);
    const bool force = p.has_force != 0;
    if (p.mask) {
        if (force)
            k_fwd_d2q9_multi<true, true><<<nb, MTHREADS, 0, s>>>(p, src, dst, ksteps, r, slots,
                                                             slot_floats);
        else
            k_fwd_d2q9_multi<true, false><<<nb, MTHREADS, 0, s>>>(p, src, dst, ksteps, r, slots,
                                                             slot_floats);
    } else {
        if (force)
            k_fwd_d2q9_multi<false, true><<<nb, MTHREADS, 0, s>>>(p, src, dst, ksteps, r, slots,
                                                             slot_floats);
        else
            k_fwd_d2q9_multi<false, false><<<nb, MTHREADS, 0, s>>>(p, src, dst, ksteps, r, slots,
                                                             slot_floats);
    }
    return hipGetLastError();
}

}  // namespace lwacm
