// lwacm_adjoint_march.hip -- reverse (adjoint) step of the D3Q19 LW-ACM
// update as a z-marching tile kernel.
//
// What it computes (the exact derivative of the forward step, Eq. ACM2.0 in
// pre-combined form, Eqs. ACM2.0b).  A source node y hands its link term
// s_k(y) = w_k [d_y + rho_y (c (A + 4.5 c) + B_y)], c = v_k . u_y, to the node
// t = y + v_k, whose outputs are D = sum s and J = sum v s + a rho u (+ rho g).
// With mu = (dL/dD, dL/dJ) of the downstream nodes, the cotangent that link
// k carries back to y is m_k = mu_R(t) + v_k . mu_J(t) (for a solid t the
// term bounced back into y itself along -v_k: m_k = mu_R(y) - v_k . mu_J(y)).
// Everything y needs from its links are the moments
//     M0 = sum_k w_k m_k,  M1 = sum_k w_k m_k v_k,  M2 = sum_k w_k m_k v_k v_k^T,
// because the link term is quadratic in u:
//     dL/d(rho-1) = M0 (1 + B) + A u.M1 + 4.5 u^T M2 u + mu_J(y).(a u + g),
//     dL/du       = rho [A M1 + 9 M2 u - 3 u M0] + a rho mu_J(y),
//     dL/da       = -3 rho u.M1 + rho mu_J(y).u  (+ the moving-wall term).
//
// Design (gfx950).  A workgroup owns a 32 x 16 tile of columns and a chunk of
// 64 planes, as the forward march kernel.  Every plane of mu (tile plus a
// one-column halo ring) passes once through a rolling window of four LDS
// planes, its four components in separate arrays; each interior thread then reads its 18
// neighbours' mu from the three planes around its own, accumulates the ten
// moments with integer weights 36 w_k (pairs of opposite links share one
// expansion), and finishes the node from its own state, which it loads
// itself (16 B FP32 / 8 B FP16 per node).  Halo waves only load mu into LDS.
// One barrier per plane; four window planes mean a plane is overwritten only
// after every thread has passed the next barrier.  HBM traffic per node:
// state + mu_in + mu_out = 48 B (FP32 state).
#include <type_traits>
#include <utility>

#include "lwacm_device.hpp"
#include "lwacm_internal.hpp"

namespace lwacm {

namespace {

#ifndef LWACM_ADJ_NZC
#define LWACM_ADJ_NZC 64
#endif
#ifndef LWACM_ADJ_RING
#define LWACM_ADJ_RING 2
#endif
constexpr int TX = 32;
constexpr int TY = 16;
constexpr int NZC = LWACM_ADJ_NZC;          // planes per workgroup
constexpr int RING = LWACM_ADJ_RING;        // planes of loads in flight per thread
constexpr int NWIN = 4;                     // LDS window planes
constexpr int NINT = TX * TY;
constexpr int NTHREADS = NINT + 2 * kWave;  // + Y-halo wave + X-halo wave
constexpr int SX = TX + 2;
constexpr int NSLOT = SX * (TY + 2);

static_assert(2 * TX <= kWave && 2 * (TY + 2) <= kWave, "halo rows must fit one wave each");

enum Role { INTERIOR = 0, HALO_Y = 1, HALO_X = 2 };

using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ Rsrc make_rsrc(const void *base, unsigned long long bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0,
                                             (int)(unsigned)bytes, 0x00020000);
}

// (Component access by explicit selection and whole-vector casts only: this
// compiler narrows a 128-bit load when its elements are bit-cast one by one.)
__device__ __forceinline__ f32x4 load_f4(Rsrc r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

template <class T>
struct StateIO;

template <>
struct StateIO<float> {
    using Raw = f32x4;
    static constexpr unsigned kNodeBytes = 16;
    __device__ __forceinline__ static Raw load(Rsrc r, unsigned voff, unsigned soff)
    {
        return load_f4(r, voff, soff);
    }
    __device__ __forceinline__ static void unpack(const Raw &v, const float (&)[2], float &d,
                                                  float &ux, float &uy, float &uz)
    {
        d = v.x;
        ux = v.y;
        uy = v.z;
        uz = v.w;
    }
};

template <>
struct StateIO<__half> {
    using Raw = u32x2;
    static constexpr unsigned kNodeBytes = 8;
    __device__ __forceinline__ static Raw load(Rsrc r, unsigned voff, unsigned soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    }
    __device__ __forceinline__ static float h(unsigned w, int hi, float s)
    {
        return __half2float(__ushort_as_half((unsigned short)(hi ? w >> 16 : w & 0xffffu))) * s;
    }
    __device__ __forceinline__ static void unpack(const Raw &v, const float (&ld)[2], float &d,
                                                  float &ux, float &uy, float &uz)
    {
        d = h(v.x, 0, ld[0]);
        ux = h(v.x, 1, ld[1]);
        uy = h(v.y, 0, ld[1]);
        uz = h(v.y, 1, ld[1]);
    }
};

__device__ __forceinline__ bool has_bit(unsigned bits, int i) { return (bits >> i) & 1u; }

template <class F, int... K>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, K...>)
{
    (f(std::integral_constant<int, K>{}), ...);
}

template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Moments of the link cotangents, with the integer weights 36 w_k.
struct Mom {
    float m0, m1x, m1y, m1z, xx, yy, zz, xy, xz, yz;
};

// A pair of opposite links +-v with weight w36: mp = m(+v), mm = m(-v).
template <int DX, int DY, int DZ>
__device__ __forceinline__ void add_pair(Mom &M, float w36, float mp, float mm)
{
    const float sp = w36 * (mp + mm);  // even part: M0, M2
    const float dm = w36 * (mp - mm);  // odd part: M1
    M.m0 += sp;
    if (DX) M.m1x += DX > 0 ? dm : -dm;
    if (DY) M.m1y += DY > 0 ? dm : -dm;
    if (DZ) M.m1z += DZ > 0 ? dm : -dm;
    if (DX) M.xx += sp;
    if (DY) M.yy += sp;
    if (DZ) M.zz += sp;
    if (DX && DY) M.xy += (DX * DY > 0) ? sp : -sp;
    if (DX && DZ) M.xz += (DX * DZ > 0) ? sp : -sp;
    if (DY && DZ) M.yz += (DY * DZ > 0) ? sp : -sp;
}

// m = mu_R + v . mu_J of the node in window slot s, for link v.  The window
// keeps mu_R, mu_Jx, mu_Jy, mu_Jz in separate arrays (4-byte lane stride,
// no bank conflicts) and a link reads only the components it needs.
template <int DX, int DY, int DZ>
__device__ __forceinline__ float link_m(const float (*W)[NSLOT], int s)
{
    float m = W[0][s];
    if (DX) m = DX > 0 ? m + W[1][s] : m - W[1][s];
    if (DY) m = DY > 0 ? m + W[2][s] : m - W[2][s];
    if (DZ) m = DZ > 0 ? m + W[3][s] : m - W[3][s];
    return m;
}

template <class T, bool MASK>
__global__ __launch_bounds__(NTHREADS) void k_adj_march(ProblemArgs p, const T *__restrict__ state,
                                                        const float *__restrict__ mu_in,
                                                        float *__restrict__ mu_out,
                                                        const unsigned *__restrict__ bb_bits,
                                                        const float4 *__restrict__ wallg,
                                                        int final_t0, ReduceArgs r)
{
    __shared__ float win[NWIN][4][NSLOT];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long n = p.n;
    const long long plane = (long long)nx * ny;

    const unsigned nb = gridDim.x;
    const unsigned b = blockIdx.x;
    const unsigned lb = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + b / 8u : b;
    const int tiles_x = nx / TX;
    const int tiles_y = ny / TY;
    const int tile_x = (int)(lb % (unsigned)tiles_x);
    const unsigned rest = lb / (unsigned)tiles_x;
    const int tile_y = (int)(rest % (unsigned)tiles_y);
    const int zc = (int)(rest / (unsigned)tiles_y);
    const int z0 = zc * NZC;
    const int z1 = min(z0 + NZC, nz);

    // column in tile coordinates [-1, TX] x [-1, TY]
    const int role = tid < NINT ? INTERIOR : (tid < NINT + kWave ? HALO_Y : HALO_X);
    int lx, ly;
    bool active = true;
    if (role == INTERIOR) {
        lx = tid % TX;
        ly = tid / TX;
    } else if (role == HALO_Y) {
        const bool top = lane >= TX;
        lx = top ? lane - TX : lane;
        ly = top ? TY : -1;
        active = lane < 2 * TX;
        if (!active) lx = 0;
    } else {
        const bool right = lane >= TY + 2;
        const int l = right ? lane - (TY + 2) : lane;
        lx = right ? TX : -1;
        ly = l - 1;
        active = lane < 2 * (TY + 2);
        if (!active) ly = 0;
    }
    int gx = tile_x * TX + lx;
    int gy = tile_y * TY + ly;
    gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
    gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
    const unsigned col = (unsigned)(gy * nx + gx);
    const int slot = (ly + 1) * SX + (lx + 1);

    auto wrapz = [&](int pz) { return pz < 0 ? pz + nz : (pz >= nz ? pz - nz : pz); };
    const Rsrc rmu = make_rsrc(mu_in, (unsigned long long)n * 16u);
    const Rsrc rst = make_rsrc(state, (unsigned long long)n * StateIO<T>::kNodeBytes);
    const unsigned mu_plane = (unsigned)(plane * 16);
    const unsigned st_plane = (unsigned)(plane * StateIO<T>::kNodeBytes);
    const unsigned voff_mu = col * 16u;
    const unsigned voff_st = col * StateIO<T>::kNodeBytes;

    // ring of loads: mu of plane pz (every thread) and the state of plane pz
    // (interior threads; finalised one iteration later)
    f32x4 rmu_ring[RING];
    typename StateIO<T>::Raw rst_ring[RING];
#pragma unroll
    for (int j = 0; j < RING; ++j) {
        const int pz = wrapz(min(z0 - 1 + j, z1));
        rmu_ring[j] = load_f4(rmu, voff_mu, (unsigned)pz * mu_plane);
        if (role == INTERIOR) rst_ring[j] = StateIO<T>::load(rst, voff_st, (unsigned)pz * st_plane);
    }

    const float A = p.A, a = p.a;
    float da = 0.0f;
    float own_st[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // state of the plane finalised next

    static_for<NZC + 2>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int rj = k % RING;
        const int pz = z0 - 1 + k;  // plane entering the window
        // ---- mu of plane pz into window slot pz % NWIN (k-indexed: same order)
        if (active) {
            const f32x4 q = rmu_ring[rj];
            win[k % NWIN][0][slot] = q.x;
            win[k % NWIN][1][slot] = q.y;
            win[k % NWIN][2][slot] = q.z;
            win[k % NWIN][3][slot] = q.w;
        }
        float cur_st[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (role == INTERIOR)
            StateIO<T>::unpack(rst_ring[rj], p.ld_scale, cur_st[0], cur_st[1], cur_st[2], cur_st[3]);
        // refill with plane pz + RING (past the chunk: plane z1 again, never used)
        if (k + RING < NZC + 2) {
            const int qz = wrapz(min(pz + RING, z1));
            rmu_ring[rj] = load_f4(rmu, voff_mu, (unsigned)qz * mu_plane);
            if (role == INTERIOR)
                rst_ring[rj] = StateIO<T>::load(rst, voff_st, (unsigned)qz * st_plane);
        }
        __syncthreads();
        const int tz = pz - 1;  // plane finalised now (window holds tz-1, tz, tz+1)
        bool solid = false;
        if (MASK && role == INTERIOR && k >= 2 && tz < z1)
            solid = p.mask[(long long)tz * plane + col] != 0;
        if (solid) {
            // solid nodes carry no cotangent
            const long long idx = (long long)tz * plane + col;
            if (final_t0) {
#pragma unroll
                for (int f = 0; f < 4; ++f) mu_out[f * n + idx] = 0.0f;
            } else {
                reinterpret_cast<float4 *>(mu_out)[idx] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        } else if (role == INTERIOR && k >= 2 && tz < z1) {
            const float(*Wm)[NSLOT] = win[(k - 2) % NWIN];  // plane tz - 1
            const float(*W0)[NSLOT] = win[(k - 1) % NWIN];  // plane tz
            const float(*Wp)[NSLOT] = win[k % NWIN];        // plane tz + 1
            const float4 own = make_float4(W0[0][slot], W0[1][slot], W0[2][slot], W0[3][slot]);
            // cotangents of the 18 moving links from the neighbours t = y + v_k,
            // in (+v, -v) pairs
            float m[18] = {link_m<1, 0, 0>(W0, slot + 1),        link_m<-1, 0, 0>(W0, slot - 1),
                           link_m<0, 1, 0>(W0, slot + SX),       link_m<0, -1, 0>(W0, slot - SX),
                           link_m<0, 0, 1>(Wp, slot),            link_m<0, 0, -1>(Wm, slot),
                           link_m<1, 1, 0>(W0, slot + SX + 1),   link_m<-1, -1, 0>(W0, slot - SX - 1),
                           link_m<1, -1, 0>(W0, slot - SX + 1),  link_m<-1, 1, 0>(W0, slot + SX - 1),
                           link_m<1, 0, 1>(Wp, slot + 1),        link_m<-1, 0, -1>(Wm, slot - 1),
                           link_m<1, 0, -1>(Wm, slot + 1),       link_m<-1, 0, 1>(Wp, slot - 1),
                           link_m<0, 1, 1>(Wp, slot + SX),       link_m<0, -1, -1>(Wm, slot - SX),
                           link_m<0, 1, -1>(Wm, slot + SX),      link_m<0, -1, 1>(Wp, slot - SX)};
            unsigned bits = 0u;
            if (MASK) bits = bb_bits[(long long)tz * plane + col];
            if (MASK && bits != 0u) {
                // a solid t = y + v_k: the term bounced back into y along -v_k,
                // m_k = mu_R(y) - v_k . mu_J(y).  The forward bit set marks
                // solid upstream nodes y - v_i, i.e. link k = opposite(i).
                constexpr int vx[18] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
                constexpr int vy[18] = {0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
                constexpr int vz[18] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
#pragma unroll
                for (int j = 0; j < 18; ++j) {
                    const int i = link_index(-vx[j], -vy[j], -vz[j]);
                    if (has_bit(bits, i)) {
                        float mb = own.x;
                        if (vx[j]) mb = vx[j] > 0 ? mb - own.y : mb + own.y;
                        if (vy[j]) mb = vy[j] > 0 ? mb - own.z : mb + own.z;
                        if (vz[j]) mb = vz[j] > 0 ? mb - own.w : mb + own.w;
                        m[j] = mb;
                    }
                }
            }
            Mom M = {};
            add_pair<1, 0, 0>(M, 2.0f, m[0], m[1]);
            add_pair<0, 1, 0>(M, 2.0f, m[2], m[3]);
            add_pair<0, 0, 1>(M, 2.0f, m[4], m[5]);
            add_pair<1, 1, 0>(M, 1.0f, m[6], m[7]);
            add_pair<1, -1, 0>(M, 1.0f, m[8], m[9]);
            add_pair<1, 0, 1>(M, 1.0f, m[10], m[11]);
            add_pair<1, 0, -1>(M, 1.0f, m[12], m[13]);
            add_pair<0, 1, 1>(M, 1.0f, m[14], m[15]);
            add_pair<0, 1, -1>(M, 1.0f, m[16], m[17]);
            M.m0 = fmaf(12.0f, own.x, M.m0);  // rest link: m = mu_R(y)
            // divide the integer weights out (correctly rounded division by 36)
            const float m0 = div36(M.m0), m1x = div36(M.m1x), m1y = div36(M.m1y), m1z = div36(M.m1z);
            const float xx = div36(M.xx), yy = div36(M.yy), zz = div36(M.zz);
            const float xy = div36(M.xy), xz = div36(M.xz), yz = div36(M.yz);

            const float dr = own_st[0], ux = own_st[1], uy = own_st[2], uz = own_st[3];
            const float rho = 1.0f + dr;
            const float B = -1.5f * fmaf(ux, ux, fmaf(uy, uy, uz * uz));
            const float uM1 = fmaf(ux, m1x, fmaf(uy, m1y, uz * m1z));
            const float M2ux = fmaf(xx, ux, fmaf(xy, uy, xz * uz));
            const float M2uy = fmaf(xy, ux, fmaf(yy, uy, yz * uz));
            const float M2uz = fmaf(xz, ux, fmaf(yz, uy, zz * uz));
            const float uM2u = fmaf(ux, M2ux, fmaf(uy, M2uy, uz * M2uz));
            const float mJu = fmaf(own.y, ux, fmaf(own.z, uy, own.w * uz));
            float lr = fmaf(m0, 1.0f + B, fmaf(A, uM1, 4.5f * uM2u));
            lr = fmaf(own.y, fmaf(a, ux, p.g[0]), lr);
            lr = fmaf(own.z, fmaf(a, uy, p.g[1]), lr);
            lr = fmaf(own.w, fmaf(a, uz, p.g[2]), lr);
            const float arho = a * rho;
            const float lux = fmaf(rho, fmaf(A, m1x, fmaf(9.0f, M2ux, -3.0f * ux * m0)), arho * own.y);
            const float luy = fmaf(rho, fmaf(A, m1y, fmaf(9.0f, M2uy, -3.0f * uy * m0)), arho * own.z);
            const float luz = fmaf(rho, fmaf(A, m1z, fmaf(9.0f, M2uz, -3.0f * uz * m0)), arho * own.w);
            da = fmaf(rho, fmaf(-3.0f, uM1, mJu), da);
            if (MASK && (bits & kMovingWallFlag)) {
                // moving walls: sum over bounced links of w_k (v_k . 6 rho0 u_w) m_k
                const float4 g = wallg[(long long)tz * plane + col];
                const float gw = -fmaf(own.x, g.x, fmaf(own.y, g.y, fmaf(own.z, g.z, own.w * g.w)));
                da = fmaf(p.wall6rho0, div36(gw), da);
            }
            const long long idx = (long long)tz * plane + col;
            if (final_t0) {
                mu_out[idx] = lr;
                mu_out[n + idx] = lux;
                mu_out[2 * n + idx] = luy;
                mu_out[3 * n + idx] = luz;
            } else {
                // fold the normalisation u = J / rho of the step before
                const float inv = 1.0f / rho;
                const float lu_u = fmaf(lux, ux, fmaf(luy, uy, luz * uz));
                reinterpret_cast<float4 *>(mu_out)[idx] =
                    make_float4(lr - lu_u * inv, lux * inv, luy * inv, luz * inv);
            }
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) own_st[f] = cur_st[f];
    });

    double v[1] = {(double)da};
    store_block_partials<1>(v, r.partials, blockIdx.x);
}

template <class T>
hipError_t dispatch(const ProblemArgs &p, const void *state, const float *mu_in, float *mu_out,
                    const unsigned *bits, const float4 *wallg, int final_t0, const ReduceArgs &r,
                    hipStream_t s)
{
    const unsigned nb = adj_march_num_blocks(p);
    const T *st = static_cast<const T *>(state);
    if (p.mask)
        k_adj_march<T, true><<<nb, NTHREADS, 0, s>>>(p, st, mu_in, mu_out, bits, wallg, final_t0, r);
    else
        k_adj_march<T, false><<<nb, NTHREADS, 0, s>>>(p, st, mu_in, mu_out, bits, wallg, final_t0, r);
    return hipGetLastError();
}

}  // namespace

bool adj_march_supported(const ProblemArgs &p)
{
    return p.Q == 19 && p.nx >= TX && p.ny >= TY && p.nx % TX == 0 && p.ny % TY == 0 &&
           p.nz >= 1 && p.n < (1LL << 28);
}

unsigned adj_march_num_blocks(const ProblemArgs &p)
{
    if (!adj_march_supported(p)) return 0;
    return (unsigned)((long long)(p.nx / TX) * (p.ny / TY) * ((p.nz + NZC - 1) / NZC));
}

hipError_t launch_adj_march(const ProblemArgs &p, int storage, const void *state,
                            const float *mu_in, float *mu_out, const unsigned *bits,
                            const float4 *wallg, int final_t0, const ReduceArgs &r,
                            hipStream_t stream)
{
    if (!adj_march_supported(p) || (p.mask && !bits)) return hipErrorNotSupported;
    const hipError_t e =
        storage ? dispatch<__half>(p, state, mu_in, mu_out, bits, wallg, final_t0, r, stream)
                : dispatch<float>(p, state, mu_in, mu_out, bits, wallg, final_t0, r, stream);
    return e != hipSuccess ? e : launch_reduce(r, 1, adj_march_num_blocks(p), stream);
}

}  // namespace lwacm
