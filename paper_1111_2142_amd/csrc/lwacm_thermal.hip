// lwacm_thermal.hip -- the temperature lattice of the thermal LW-ACM.
//
// Appendix "Asymptotic analysis for energy equation", Eq. ACM2.0t: a second
// lattice (the flow's own, Q_t = Q, or its rest and axis links alone, Q_t =
// 5 or 7: see below) whose only state is T.  With
// c = v_i . u and q = 9/2 c^2 - 3/2 |u|^2 its equilibrium is
// g^(e)_i = w_i [T (1 + 3 c) + q] (moments T, T u and u u + T/3 I) and the
// even part of Eq. feqe is w_i (T + q).  Eq. ACM2.0t then reads, with
// kap = 2 - 2/omega_t and h = 1 - kap,
//   T(x, t+1) = kap T(x) + sum_i w_i [h (T(y) + q(y)) + 3 T(y) c(y)],  y = x - v_i,
// where the own even parts sum to kap T(x) (sum_i w_i q = 0 on both
// lattices).  u is the flow velocity at the same time, read from the flow
// state the flow step of that time reads.
//
// Walls, halfway like the flow's: where x - v_i is solid the term x sends
// along the opposite link, w_i [h (T(x) + q(x)) - 3 T(x) c(x)], comes back
// unchanged (adiabatic wall) or with its sign reversed plus 2 h w_i T_w (wall
// at temperature T_w, anti-bounce-back).  The paper states no thermal wall
// rule; a linear profile between two such walls is an exact steady state.
//
// Q_t != Q (the appendix allows it): D2Q5 under a D2Q9 flow, D3Q7 under
// D3Q19, the rest link and the axis links with 36 w = 6 on the axis links and
// 36 - 12 D on the rest link (12 and 0): the second moment T/3 I fixes the
// axis weight.  These lattices cannot carry the u u part of the second
// moment (O(eps^2) under diffusive scaling), so their equilibrium is the
// linear w_i T (1 + 3 c): the terms above with q = 0.  They run the gather
// kernel.
//
// Where it can, the library runs the step inside the D3Q19 flow tile kernel
// (lwacm_march.hip, THERM); the kernels here serve the other cases.
// D3Q19 with nx % 32 == 0 and ny % 16 == 0 runs the tile kernel: a workgroup
// owns a 32 x 16 column tile and marches up a chunk of z planes; each plane's
// T, u (and mask) with a one-node halo are staged once through LDS into a ring
// of three planes, and every thread reads its 19 upstream nodes from there.
// HBM then sees each node's state and T about once (the halo columns are
// mostly L2 hits), so the kernel is bound by HBM at 24 B per node.  Other
// shapes, D2Q9, FP16 flow states and the D2Q5/D3Q7 lattices run the gather
// kernel: one thread per node, the upstream nodes read through L1/L2.  The
// reverse mode and the fused kernel's fixed-temperature wall table are here
// too.
#include "lwacm_device.hpp"
#include "lwacm_thermal.hpp"

namespace lwacm {

namespace {

constexpr int kThermalBX = 64;
constexpr int kThermalBY = 4;

__device__ __forceinline__ int wrap_step(int a, int d, int n)
{
    int r = a - d;
    r += (r < 0) ? n : 0;
    r -= (r >= n) ? n : 0;
    return r;
}

// (rho - 1, u) of node idx from the flow state in storage format S (float or
// FP16 deviations with the load scales)
template <class S, int Q>
__device__ __forceinline__ float load_u(const ThermalArgs &t, long long idx, float (&u)[3])
{
    constexpr int NF = Lattice<Q>::D + 1;
    float v[NF];
    NodeState<S, NF>::load(static_cast<const S *>(t.state), idx, t.ld_scale, v);
    u[0] = v[1];
    u[1] = v[2];
    u[2] = NF == 4 ? v[NF - 1] : 0.0f;
    return v[0];
}

// links of the axis lattice (rest and axis links) and their 36 w
__host__ __device__ constexpr bool axis_link(int i)
{
    return (link_cx(i) != 0) + (link_cy(i) != 0) + (link_cz(i) != 0) <= 1;
}
template <int Q>
__host__ __device__ constexpr float axis_w36(int i)
{
    return i == 0 ? 36.0f - 12.0f * Lattice<Q>::D : 6.0f;
}

// AXIS: the temperature on the axis lattice of the flow's lattice Q
template <int Q, bool MASK, bool AXIS, class S>
__global__ __launch_bounds__(kThermalBX *kThermalBY) void k_thermal_step(ThermalArgs t)
{
    const int x = blockIdx.x * kThermalBX + threadIdx.x;
    const int y = blockIdx.y * kThermalBY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= t.nx || y >= t.ny) return;
    const long long plane = (long long)t.nx * t.ny;
    const long long idx = (long long)z * plane + (long long)y * t.nx + x;
    const float Tx = t.T_in[idx];
    if (MASK && t.mask[idx] != 0) {
        t.T_out[idx] = Tx;
        return;
    }
    float ux[3];
    load_u<S, Q>(t, idx, ux);
    const float bx = AXIS ? 0.0f : -1.5f * (ux[0] * ux[0] + ux[1] * ux[1] + ux[2] * ux[2]);
    float acc = 0.0f;  // sum of 36 w_i times the incoming terms
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (AXIS && (!axis_link(i) || axis_w36<Q>(i) == 0.0f)) continue;
        const int cx = link_cx(i), cy = link_cy(i), cz = link_cz(i);
        const int xs = wrap_step(x, cx, t.nx);
        const int ys = wrap_step(y, cy, t.ny);
        const int zs = wrap_step(z, cz, t.nz);
        const long long is = (long long)zs * plane + (long long)ys * t.nx + xs;
        const float w36 = AXIS ? axis_w36<Q>(i) : Lattice<Q>::w36(i);
        float term;
        bool fluid = true;
        uint8_t m = 0;
        if (MASK) {
            m = t.mask[is];
            fluid = (m == 0);
        }
        if (fluid) {
            float us[3];
            load_u<S, Q>(t, is, us);
            const float Ts = t.T_in[is];
            const float c = cx * us[0] + cy * us[1] + cz * us[2];
            const float q =
                AXIS ? 0.0f
                     : fmaf(4.5f * c, c, -1.5f * (us[0] * us[0] + us[1] * us[1] + us[2] * us[2]));
            term = fmaf(t.h, Ts + q, 3.0f * Ts * c);
        } else {
            const float c = cx * ux[0] + cy * ux[1] + cz * ux[2];
            const float q = AXIS ? 0.0f : fmaf(4.5f * c, c, bx);
            const float sent = fmaf(t.h, Tx + q, -3.0f * Tx * c);
            const float Tw = m < kMaxThermalWallIds ? t.wall_T[m] : __builtin_nanf("");
            term = (Tw != Tw) ? sent : fmaf(2.0f * t.h, Tw, -sent);
        }
        acc = fmaf(w36, term, acc);
    }
    t.T_out[idx] = fmaf(t.kap, Tx, div36(acc));
}

__global__ __launch_bounds__(256) void k_thermal_wall_table(ThermalArgs t, uint2 *out)
{
    const long long n = (long long)t.nx * t.ny * t.nz;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        unsigned fb = 0u;
        float tw = 0.0f;
        if (t.mask[idx] == 0) {
            const long long r = idx / t.nx;
            const int x = (int)(idx - r * t.nx);
            const int z = (int)(r / t.ny);
            const int y = (int)(r - (long long)z * t.ny);
#pragma unroll
            for (int i = 1; i < 19; ++i) {
                const int xs = wrap_step(x, link_cx(i), t.nx);
                const int ys = wrap_step(y, link_cy(i), t.ny);
                const int zs = wrap_step(z, link_cz(i), t.nz);
                const uint8_t m = t.mask[((long long)zs * t.ny + ys) * t.nx + xs];
                const float Tw = m < kMaxThermalWallIds ? t.wall_T[m] : __builtin_nanf("");
                if (m != 0 && Tw == Tw) {
                    fb |= 1u << i;
                    tw = fmaf(Lattice<19>::w36(i), Tw, tw);
                }
            }
        }
        out[idx] = make_uint2(fb, __builtin_bit_cast(unsigned, tw));
    }
}

// ---- reverse mode of one step (gather over the nodes a node's T and u reach)
//
// T(x, t+1) is linear in the T of its upstream nodes and quadratic in their u;
// node z's cotangents collect, for every link i:
//   x = z + v_i fluid: lam(x) d/d(T_z, u_z) of w_i [h (T_z + q) + 3 T_z c],
//     c = v_i . u_z: (w_i (h + 3 c), w_i (3 T_z v_i + h dq)), dq = 9 c v_i - 3 u_z;
//   z - v_i solid: lam(z) d/d(T_z, u_z) of the term z sent along -v_i into the
//     wall, returned with sign s (+1 adiabatic, -1 fixed temperature):
//     s (w_i (h - 3 c), w_i (-3 T_z v_i + h dq));
// plus kap lam(z) from the own even parts (their u terms sum to zero on every
// lattice here).  On the D2Q5/D3Q7 lattices q = 0 and dq = 0.  A solid node
// passes lam through and gives no u cotangent.
template <int Q, bool MASK, bool AXIS, class S>
__global__ __launch_bounds__(kThermalBX *kThermalBY) void k_thermal_adjoint(ThermalAdjArgs a)
{
    const ThermalArgs &t = a.t;
    const int x = blockIdx.x * kThermalBX + threadIdx.x;
    const int y = blockIdx.y * kThermalBY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= t.nx || y >= t.ny) return;
    const long long plane = (long long)t.nx * t.ny;
    const long long n = plane * t.nz;
    const long long idx = (long long)z * plane + (long long)y * t.nx + x;
    const float lz = a.lam_in[idx];
    if (MASK && t.mask[idx] != 0) {
        a.lam_out[idx] = lz;
        return;
    }
    constexpr int D = Lattice<Q>::D;
    float u[3];
    const float dr = load_u<S, Q>(t, idx, u);
    const float Tz = t.T_in[idx];
    float lt = t.kap * lz;
    float gu[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < Q; ++i) {  // the rest link too: its term is w_0 h (T_z + q)
        if (AXIS && (!axis_link(i) || axis_w36<Q>(i) == 0.0f)) continue;
        const int cx = link_cx(i), cy = link_cy(i), cz = link_cz(i);
        const float w = (AXIS ? axis_w36<Q>(i) : Lattice<Q>::w36(i)) * (1.0f / 36.0f);
        const float c = cx * u[0] + cy * u[1] + cz * u[2];
        const float v[3] = {(float)cx, (float)cy, (float)cz};
        float dq[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) dq[k] = AXIS ? 0.0f : fmaf(9.0f * c, v[k], -3.0f * u[k]);
        // downstream node x = z + v_i
        const int xd = wrap_step(x, -cx, t.nx);
        const int yd = wrap_step(y, -cy, t.ny);
        const int zd = wrap_step(z, -cz, t.nz);
        const long long id = (long long)zd * plane + (long long)yd * t.nx + xd;
        if (!MASK || t.mask[id] == 0) {
            const float lx = a.lam_in[id] * w;
            lt = fmaf(lx, fmaf(3.0f, c, t.h), lt);
#pragma unroll
            for (int k = 0; k < D; ++k) gu[k] = fmaf(lx, fmaf(3.0f * Tz, v[k], t.h * dq[k]), gu[k]);
        }
        if (MASK && i != 0) {
            // upstream node z - v_i solid: the wall returned z's own term
            const int xs = wrap_step(x, cx, t.nx);
            const int ys = wrap_step(y, cy, t.ny);
            const int zs = wrap_step(z, cz, t.nz);
            const uint8_t m = t.mask[(long long)zs * plane + (long long)ys * t.nx + xs];
            if (m != 0) {
                const float Tw = m < kMaxThermalWallIds ? t.wall_T[m] : __builtin_nanf("");
                const float ls = ((Tw != Tw) ? lz : -lz) * w;
                lt = fmaf(ls, fmaf(-3.0f, c, t.h), lt);
#pragma unroll
                for (int k = 0; k < D; ++k)
                    gu[k] = fmaf(ls, fmaf(-3.0f * Tz, v[k], t.h * dq[k]), gu[k]);
            }
        }
    }
    a.lam_out[idx] = lt;
    if (a.final_t0) {
#pragma unroll
        for (int k = 0; k < D; ++k) a.mu[(1 + k) * n + idx] += gu[k];
    } else {
        // mu_{t-1} = (lambda_rho - lambda_u . u / rho, lambda_u / rho) is linear
        // in lambda_u: the u cotangent enters both parts
        const float inv = 1.0f / (1.0f + dr);
        float gdu = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) gdu = fmaf(gu[k], u[k], gdu);
        a.mu[(D + 1) * idx] -= gdu * inv;
#pragma unroll
        for (int k = 0; k < D; ++k) a.mu[(D + 1) * idx + 1 + k] += gu[k] * inv;
    }
}

// ---- tile kernel (D3Q19): LDS ring of three planes, one column per thread
constexpr int kTX = 32, kTY = 16;            // tile of columns per workgroup
constexpr int kHX = kTX + 2, kHY = kTY + 2;  // with the one-node halo
constexpr int kCells = kHX * kHY;            // 612 staged nodes per plane
constexpr int kChunk = 32;                   // z planes per workgroup

// Each staged node carries what its terms need: A = h (T - 3/2 |u|^2), 3 T
// and u, so that the term it sends along link i,
//   w_i [h (T + 9/2 c^2 - 3/2 |u|^2) + 3 T c] = w_i [A + c (9/2 h c + 3 T)],
// costs two multiply-adds per link (c = v_i . u).
template <bool MASK>
struct ThermalRing {
    float T3[3][kCells];
    float A[3][kCells];
    float u[3][3][kCells];
    uint8_t m[MASK ? 3 : 1][MASK ? kCells : 1];
};

// One plane's staged nodes in flight in registers: a thread holds the nodes
// tid and tid + 512 (the second only for tid < 100).
constexpr int kPerThread = (kCells + kTX * kTY - 1) / (kTX * kTY);

template <bool MASK>
struct PlaneRegs {
    float4 s[kPerThread];
    float T[kPerThread];
    uint8_t m[kPerThread];
};

template <bool MASK>
__device__ __forceinline__ void fetch_plane(const ThermalArgs &t, PlaneRegs<MASK> &v, int z,
                                            int x0, int y0, int tid)
{
    const long long base = (long long)z * t.nx * t.ny;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int c = tid + k * kTX * kTY;
        if (c < kCells) {
            const int hy = c / kHX, hx = c - hy * kHX;
            int gx = x0 + hx - 1, gy = y0 + hy - 1;
            gx += (gx < 0) ? t.nx : 0;
            gx -= (gx >= t.nx) ? t.nx : 0;
            gy += (gy < 0) ? t.ny : 0;
            gy -= (gy >= t.ny) ? t.ny : 0;
            const long long g = base + (long long)gy * t.nx + gx;
            v.s[k] = static_cast<const float4 *>(t.state)[g];
            v.T[k] = t.T_in[g];
            if constexpr (MASK) v.m[k] = t.mask[g];
        }
    }
}

template <bool MASK>
__device__ __forceinline__ void put_plane(const ThermalArgs &t, ThermalRing<MASK> &r,
                                          const PlaneRegs<MASK> &v, int slot, int tid)
{
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int c = tid + k * kTX * kTY;
        if (c < kCells) {
            const float4 s = v.s[k];
            r.T3[slot][c] = 3.0f * v.T[k];
            r.A[slot][c] = t.h * fmaf(-1.5f, fmaf(s.y, s.y, fmaf(s.z, s.z, s.w * s.w)), v.T[k]);
            r.u[slot][0][c] = s.y;
            r.u[slot][1][c] = s.z;
            r.u[slot][2][c] = s.w;
            if constexpr (MASK) r.m[slot][c] = v.m[k];
        }
    }
}

template <bool MASK>
__global__ __launch_bounds__(kTX *kTY) void k_thermal_march(ThermalArgs t)
{
    __shared__ ThermalRing<MASK> r;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTX + tx;
    // Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b % 8);
    // numbering the tiles XCD by XCD gives each XCD a contiguous run of tiles
    // (x fastest), so the halo columns a tile shares with its x and y
    // neighbours are read through the same L2.
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned lb = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + b / 8u : b;
    const unsigned tiles_x = (unsigned)(t.nx / kTX), tiles_y = (unsigned)(t.ny / kTY);
    const int x0 = (int)(lb % tiles_x) * kTX;
    const int y0 = (int)((lb / tiles_x) % tiles_y) * kTY;
    const int z0 = (int)(lb / (tiles_x * tiles_y)) * kChunk;
    const int z1 = min(z0 + kChunk, t.nz);
    const int zm = z0 == 0 ? t.nz - 1 : z0 - 1;
    PlaneRegs<MASK> v;
    fetch_plane<MASK>(t, v, zm, x0, y0, tid);
    put_plane<MASK>(t, r, v, 0, tid);
    fetch_plane<MASK>(t, v, z0, x0, y0, tid);
    put_plane<MASK>(t, r, v, 1, tid);
    fetch_plane<MASK>(t, v, z0 + 1 == t.nz ? 0 : z0 + 1, x0, y0, tid);
    const int cc = (ty + 1) * kHX + tx + 1;  // this column's cell in a staged plane
    const long long plane = (long long)t.nx * t.ny;
    const long long col = (long long)(y0 + ty) * t.nx + x0 + tx;
    const float H = 4.5f * t.h;
    int sm = 0, s0 = 1, sp = 2;  // ring slots of planes z - 1, z, z + 1
    // Plane z + 1 arrives from the registers; the loads of plane z + 2 are
    // issued before plane z is computed, so their latency overlaps that work.
    for (int z = z0; z < z1; ++z) {
        const long long idx = (long long)z * plane + col;
        const float Tx = t.T_in[idx];
        put_plane<MASK>(t, r, v, sp, tid);
        __syncthreads();
        if (z + 2 <= z1) {
            int z2 = z + 2;
            z2 -= (z2 >= t.nz) ? t.nz : 0;
            fetch_plane<MASK>(t, v, z2, x0, y0, tid);
        }
        if (MASK && r.m[MASK ? s0 : 0][MASK ? cc : 0] != 0) {
            t.T_out[idx] = Tx;
        } else {
            const float ux = r.u[s0][0][cc], uy = r.u[s0][1][cc], uz = r.u[s0][2][cc];
            float acc = 0.0f;
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const int cx = link_cx(i), cy = link_cy(i), cz = link_cz(i);
                const int ss = cz == 0 ? s0 : (cz > 0 ? sm : sp);  // plane z - cz
                const int cs = cc - cy * kHX - cx;
                float term;
                if (MASK && r.m[MASK ? ss : 0][MASK ? cs : 0] != 0) {
                    // the term x sends along the opposite link, reflected
                    const uint8_t m = r.m[MASK ? ss : 0][MASK ? cs : 0];
                    const float c = cx * ux + cy * uy + cz * uz;
                    const float sent = fmaf(c, fmaf(H, c, -r.T3[s0][cc]), r.A[s0][cc]);
                    const float Tw = m < kMaxThermalWallIds ? t.wall_T[m] : __builtin_nanf("");
                    term = (Tw != Tw) ? sent : fmaf(2.0f * t.h, Tw, -sent);
                } else {
                    float c = 0.0f;
                    if (cx) c += cx * r.u[ss][0][cs];
                    if (cy) c += cy * r.u[ss][1][cs];
                    if (cz) c += cz * r.u[ss][2][cs];
                    term = fmaf(c, fmaf(H, c, r.T3[ss][cs]), r.A[ss][cs]);
                }
                acc = fmaf(Lattice<19>::w36(i), term, acc);
            }
            t.T_out[idx] = fmaf(t.kap, Tx, div36(acc));
        }
        __syncthreads();  // plane z - 1's slot is restaged next
        const int s = sm;
        sm = s0;
        s0 = sp;
        sp = s;
    }
}

bool march_shape(const ThermalArgs &t)
{
    return t.Q == 19 && t.QT == 19 && !t.st_half && t.nx % kTX == 0 && t.ny % kTY == 0;
}

template <int Q, class S>
void launch_gather(const ThermalArgs &t, dim3 grid, dim3 block, hipStream_t stream)
{
    const bool axis = t.QT != Q;
    if (t.mask && axis)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_step<Q, true, true, S>), grid, block, 0, stream, t);
    else if (t.mask)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_step<Q, true, false, S>), grid, block, 0, stream, t);
    else if (axis)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_step<Q, false, true, S>), grid, block, 0, stream, t);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_step<Q, false, false, S>), grid, block, 0, stream, t);
}

template <int Q>
hipError_t launch_q(const ThermalArgs &t, hipStream_t stream)
{
    if (Q == 19 && march_shape(t)) {
        const dim3 block(kTX, kTY, 1);
        const long long nb =
            (long long)(t.nx / kTX) * (t.ny / kTY) * ((t.nz + kChunk - 1) / kChunk);
        if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
        const dim3 grid((unsigned)nb, 1, 1);
        if (t.mask)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_march<true>), grid, block, 0, stream, t);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_march<false>), grid, block, 0, stream, t);
        return hipGetLastError();
    }
    const dim3 block(kThermalBX, kThermalBY, 1);
    const dim3 grid((t.nx + kThermalBX - 1) / kThermalBX, (t.ny + kThermalBY - 1) / kThermalBY,
                    t.nz);
    if (t.st_half)
        launch_gather<Q, __half>(t, grid, block, stream);
    else
        launch_gather<Q, float>(t, grid, block, stream);
    return hipGetLastError();
}

template <int Q>
hipError_t launch_adj_q(const ThermalAdjArgs &a, hipStream_t stream)
{
    const ThermalArgs &t = a.t;
    const dim3 block(kThermalBX, kThermalBY, 1);
    const dim3 grid((t.nx + kThermalBX - 1) / kThermalBX, (t.ny + kThermalBY - 1) / kThermalBY,
                    t.nz);
    const bool axis = t.QT != Q;
    if (t.st_half) {
        if (t.mask && axis)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_adjoint<Q, true, true, __half>), grid, block, 0, stream, a);
        else if (t.mask)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_adjoint<Q, true, false, __half>), grid, block, 0, stream, a);
        else if (axis)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_adjoint<Q, false, true, __half>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_adjoint<Q, false, false, __half>), grid, block, 0, stream, a);
    } else {
        if (t.mask && axis)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_adjoint<Q, true, true, float>), grid, block, 0, stream, a);
        else if (t.mask)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_adjoint<Q, true, false, float>), grid, block, 0, stream, a);
        else if (axis)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_adjoint<Q, false, true, float>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_thermal_adjoint<Q, false, false, float>), grid, block, 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_thermal_wall_table(const ThermalArgs &t, uint2 *out, hipStream_t stream)
{
    if (t.Q != 19 || !t.mask || !out) return hipErrorInvalidValue;
    long long nb = ((long long)t.nx * t.ny * t.nz + 255) / 256;
    if (nb > 4096) nb = 4096;
    k_thermal_wall_table<<<(unsigned)nb, 256, 0, stream>>>(t, out);
    return hipGetLastError();
}

hipError_t launch_thermal_adjoint(const ThermalAdjArgs &a, hipStream_t stream)
{
    const ThermalArgs &t = a.t;
    if (t.nx <= 0 || t.ny <= 0 || t.nz <= 0 || t.nz > 65535 ||
        (t.ny + kThermalBY - 1) / kThermalBY > 65535)
        return hipErrorInvalidValue;
    if (t.QT != t.Q && t.QT != (t.Q == 9 ? 5 : 7)) return hipErrorInvalidValue;
    if (t.Q == 9) return t.nz == 1 ? launch_adj_q<9>(a, stream) : hipErrorInvalidValue;
    if (t.Q == 19) return launch_adj_q<19>(a, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_thermal_step(const ThermalArgs &t, hipStream_t stream)
{
    if (t.nx <= 0 || t.ny <= 0 || t.nz <= 0 || t.nz > 65535 ||
        (t.ny + kThermalBY - 1) / kThermalBY > 65535)
        return hipErrorInvalidValue;
    if (t.QT != t.Q && t.QT != (t.Q == 9 ? 5 : 7)) return hipErrorInvalidValue;
    if (t.Q == 9) return t.nz == 1 ? launch_q<9>(t, stream) : hipErrorInvalidValue;
    if (t.Q == 19) return launch_q<19>(t, stream);
    return hipErrorInvalidValue;
}

}  // namespace lwacm
