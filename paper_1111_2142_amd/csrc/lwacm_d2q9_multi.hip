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
constexpr int MSIDE = 32;

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    int m = v % n;
    return m < 0 ? m + n : m;
}

constexpr int MR = 2;  // rows per thread: a strip of MR nodes shares its neighbours' loads

template <bool MASK, bool FORCE>
__global__ __launch_bounds__(MTHREADS) void k_fwd_d2q9_multi(ProblemArgs p, const float *__restrict__ src,
                                                             float *__restrict__ dst, int ksteps,
                                                             ReduceArgs r)
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
                if (MASK && own.w > 0.0f) {  // solid: unchanged
                    buf[b1][l] = own;
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
        dst[3 * g] = v.x;
        dst[3 * g + 1] = v.y;
        dst[3 * g + 2] = v.z;
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

hipError_t launch_fwd_d2q9_multi(const ProblemArgs &p, const float *src, float *dst, int ksteps,
                                 const ReduceArgs &r, hipStream_t s)
{
    if (!d2q9_multi_supported(p) || ksteps < 1 || ksteps > MK) return hipErrorInvalidValue;
    const unsigned nb = d2q9_multi_num_blocks(p);
    const bool force = p.has_force != 0;
    if (p.mask) {
        if (force)
            k_fwd_d2q9_multi<true, true><<<nb, MTHREADS, 0, s>>>(p, src, dst, ksteps, r);
        else
            k_fwd_d2q9_multi<true, false><<<nb, MTHREADS, 0, s>>>(p, src, dst, ksteps, r);
    } else {
        if (force)
            k_fwd_d2q9_multi<false, true><<<nb, MTHREADS, 0, s>>>(p, src, dst, ksteps, r);
        else
            k_fwd_d2q9_multi<false, false><<<nb, MTHREADS, 0, s>>>(p, src, dst, ksteps, r);
    }
    return hipGetLastError();
}

}  // namespace lwacm
