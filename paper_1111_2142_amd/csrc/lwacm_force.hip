// lwacm_force.hip -- force and torque on a wall by momentum exchange
// (Section "Moving complex boundaries", Eqs. MEA3, MEA4 and MEA5).
//
// For every link j from a fluid node x to a solid node x + v_j of the chosen
// wall id the fluid gives the wall the momentum
//   p_j = v_j [f*_j(x) + f**_BB(j)(x)],
// f*_j the pre-combined population x sends into the wall and f**_BB(j) the one
// the wall sends back before post-combining (f*_j itself for halfway walls;
// the interpolation of Eq. ACM2.0cc with the link's q otherwise; bodies at
// rest, so no wall-motion term).  In the deviation form of the link term,
// f*_j = w_j (1 + L_j), and the interpolation weights sum to one, so
// p_j = v_j w_j (2 + L_j + L**_j).  F = sum p_j and T = sum (x - x_c) x p_j are
// summed in FP64: per thread, per block in LDS, then over the blocks in a
// fixed order, so a call's result does not depend on scheduling.
#include "lwacm_device.hpp"
#include "lwacm_force.hpp"

namespace lwacm {

namespace {

template <int Q>
__device__ __forceinline__ void node_du(const float *state, long long idx, float &dr, float (&u)[3])
{
    if constexpr (Q == 19) {
        const float4 s = reinterpret_cast<const float4 *>(state)[idx];
        dr = s.x;
        u[0] = s.y;
        u[1] = s.z;
        u[2] = s.w;
    } else {
        dr = state[3 * idx];
        u[0] = state[3 * idx + 1];
        u[1] = state[3 * idx + 2];
        u[2] = 0.0f;
    }
}

__device__ __forceinline__ int wrap1(int a, int n)
{
    return a < 0 ? a + n : (a >= n ? a - n : a);
}

template <int Q>
__global__ __launch_bounds__(kForceBlock) void k_wall_force(ForceArgs f)
{
    const long long n = (long long)f.nx * f.ny * f.nz;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long idx = (long long)blockIdx.x * kForceBlock + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * kForceBlock) {
        if (f.mask[idx] != 0) continue;
        const long long t = idx / f.nx;
        const int x = (int)(idx - t * f.nx);
        const int z = (int)(t / f.ny);
        const int y = (int)(t - (long long)z * f.ny);
        float dr, u[3];
        node_du<Q>(f.state, idx, dr, u);
        const float rho = 1.0f + dr;
        const float B = -1.5f * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int j = 1; j < Q; ++j) {
            const int cx = link_cx(j), cy = link_cy(j), cz = link_cz(j);
            const long long iw = ((long long)wrap1(z + cz, f.nz) * f.ny + wrap1(y + cy, f.ny)) * f.nx +
                                 wrap1(x + cx, f.nx);
            if (f.mask[iw] != f.wall_id) continue;
            const float c = cx * u[0] + cy * u[1] + cz * u[2];
            const float Lj = link_term_unweighted(dr, rho, c, B, f.A);
            float Lb = Lj;
            if (f.qd) {
                const float qv = f.qd[(long long)j * n + idx];
                if (qv < 0.5f) {
                    const long long is =
                        ((long long)wrap1(z - cz, f.nz) * f.ny + wrap1(y - cy, f.ny)) * f.nx +
                        wrap1(x - cx, f.nx);
                    if (f.mask[is] == 0) {
                        float ds, us[3];
                        node_du<Q>(f.state, is, ds, us);
                        const float cs = cx * us[0] + cy * us[1] + cz * us[2];
                        const float Bs = -1.5f * (us[0] * us[0] + us[1] * us[1] + us[2] * us[2]);
                        const float Lz = link_term_unweighted(ds, 1.0f + ds, cs, Bs, f.A);
                        Lb = fmaf(2.0f * qv, Lj, (1.0f - 2.0f * qv) * Lz);
                    }
                } else {
                    const float Li = link_term_unweighted(dr, rho, -c, B, f.A);
                    const float h = 0.5f / qv;
                    Lb = fmaf(h, Lj, (1.0f - h) * Li);
                }
            }
            const double pw = (double)Lattice<Q>::w36(j) / 36.0 * (2.0 + (double)Lj + (double)Lb);
            const double p[3] = {cx * pw, cy * pw, cz * pw};
            const double r[3] = {x - f.xc[0], y - f.xc[1], z - f.xc[2]};
            acc[0] += p[0];
            acc[1] += p[1];
            acc[2] += p[2];
            acc[3] += r[1] * p[2] - r[2] * p[1];
            acc[4] += r[2] * p[0] - r[0] * p[2];
            acc[5] += r[0] * p[1] - r[1] * p[0];
        }
    }
    __shared__ double red[6][kForceBlock];
#pragma unroll
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (unsigned s = kForceBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) f.partials[6 * (long long)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// The same sums over the list of fluid nodes next to a wall (node order):
// each thread takes list entries in a fixed grid-stride order, so the sums
// are reproducible.
template <int Q>
__global__ __launch_bounds__(kForceBlock) void k_wall_force_list(ForceArgs f)
{
    const long long n = (long long)f.nx * f.ny * f.nz;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (unsigned k = blockIdx.x * kForceBlock + threadIdx.x; k < f.nlist;
         k += gridDim.x * kForceBlock) {
        const long long idx = f.list[k];
        const long long t = idx / f.nx;
        const int x = (int)(idx - t * f.nx);
        const int z = (int)(t / f.ny);
        const int y = (int)(t - (long long)z * f.ny);
        float dr, u[3];
        node_du<Q>(f.state, idx, dr, u);
        const float rho = 1.0f + dr;
        const float B = -1.5f * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
#pragma unroll
        for (int j = 1; j < Q; ++j) {
            const int cx = link_cx(j), cy = link_cy(j), cz = link_cz(j);
            const long long iw = ((long long)wrap1(z + cz, f.nz) * f.ny + wrap1(y + cy, f.ny)) * f.nx +
                                 wrap1(x + cx, f.nx);
            if (f.mask[iw] != f.wall_id) continue;
            const float c = cx * u[0] + cy * u[1] + cz * u[2];
            const float Lj = link_term_unweighted(dr, rho, c, B, f.A);
            float Lb = Lj;
            if (f.qd) {
                const float qv = f.qd[(long long)j * n + idx];
                if (qv < 0.5f) {
                    const long long is =
                        ((long long)wrap1(z - cz, f.nz) * f.ny + wrap1(y - cy, f.ny)) * f.nx +
                        wrap1(x - cx, f.nx);
                    if (f.mask[is] == 0) {
                        float ds, us[3];
                        node_du<Q>(f.state, is, ds, us);
                        const float cs = cx * us[0] + cy * us[1] + cz * us[2];
                        const float Bs = -1.5f * (us[0] * us[0] + us[1] * us[1] + us[2] * us[2]);
                        const float Lz = link_term_unweighted(ds, 1.0f + ds, cs, Bs, f.A);
                        Lb = fmaf(2.0f * qv, Lj, (1.0f - 2.0f * qv) * Lz);
                    }
                } else {
                    const float Li = link_term_unweighted(dr, rho, -c, B, f.A);
                    const float h = 0.5f / qv;
                    Lb = fmaf(h, Lj, (1.0f - h) * Li);
                }
            }
            const double pw = (double)Lattice<Q>::w36(j) / 36.0 * (2.0 + (double)Lj + (double)Lb);
            const double p[3] = {cx * pw, cy * pw, cz * pw};
            const double r[3] = {x - f.xc[0], y - f.xc[1], z - f.xc[2]};
            acc[0] += p[0];
            acc[1] += p[1];
            acc[2] += p[2];
            acc[3] += r[1] * p[2] - r[2] * p[1];
            acc[4] += r[2] * p[0] - r[0] * p[2];
            acc[5] += r[0] * p[1] - r[1] * p[0];
        }
    }
    __shared__ double red[6][kForceBlock];
#pragma unroll
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (unsigned s = kForceBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) f.partials[6 * (long long)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Sum of the block partials in a fixed order: thread t adds the blocks
// t, t + 256, ... in turn, then a tree over the 256 threads in LDS.
__global__ __launch_bounds__(kForceBlock) void k_wall_force_sum(const double *partials,
                                                                unsigned nblocks, double *out)
{
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (unsigned b = threadIdx.x; b < nblocks; b += kForceBlock)
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] += partials[6 * b + k];
    __shared__ double red[6][kForceBlock];
#pragma unroll
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (unsigned s = kForceBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

hipError_t launch_wall_force(const ForceArgs &f, unsigned nblocks, hipStream_t stream)
{
    if (nblocks == 0 || nblocks > kForceMaxBlocks || !f.mask || !f.state) return hipErrorInvalidValue;
    if (f.Q != 19 && !(f.Q == 9 && f.nz == 1)) return hipErrorInvalidValue;
    if (f.list) {
        if (f.Q == 19)
            k_wall_force_list<19><<<nblocks, kForceBlock, 0, stream>>>(f);
        else
            k_wall_force_list<9><<<nblocks, kForceBlock, 0, stream>>>(f);
    } else if (f.Q == 19) {
        k_wall_force<19><<<nblocks, kForceBlock, 0, stream>>>(f);
    } else {
        k_wall_force<9><<<nblocks, kForceBlock, 0, stream>>>(f);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wall_force_sum, dim3(1), dim3(kForceBlock), 0, stream, f.partials, nblocks,
                       f.out);
    return hipGetLastError();
}

}  // namespace lwacm
