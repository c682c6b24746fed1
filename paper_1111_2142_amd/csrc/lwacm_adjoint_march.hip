// lwacm_adjoint_march.hip -- reverse (adjoint) step of the D3Q19 LW-ACM
// update as a z-marching tile kernel.
//
// The per-node arithmetic (moments of the link cotangents, Eqs. ACM2.0b
// differentiated) is in lwacm_adjoint_common.hpp.
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
#include "lwacm_adjoint_common.hpp"

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
            const float(*Wm)[NSLOT] = win[(k + NWIN - 2) % NWIN];  // plane tz - 1
            const float(*W0)[NSLOT] = win[(k + NWIN - 1) % NWIN];  // plane tz
            const float(*Wp)[NSLOT] = win[k % NWIN];                // plane tz + 1
            const long long idx = (long long)tz * plane + col;
            unsigned bits = 0u;
            if (MASK) bits = bb_bits[idx];
            const f32x4 lam = adj_point<MASK, NSLOT, SX>(Wm, W0, Wp, slot, own_st[0], own_st[1],
                                                         own_st[2], own_st[3], bits, wallg, idx,
                                                         p, da);
            if (final_t0) {
                mu_out[idx] = lam.x;
                mu_out[n + idx] = lam.y;
                mu_out[2 * n + idx] = lam.z;
                mu_out[3 * n + idx] = lam.w;
            } else {
                const f32x4 mu = fold_normalisation(lam, own_st[0], own_st[1], own_st[2], own_st[3]);
                reinterpret_cast<float4 *>(mu_out)[idx] = make_float4(mu.x, mu.y, mu.z, mu.w);
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
    // r.out null: the caller adds the block partials itself (lwacm_adjoint_sweep)
    if (e != hipSuccess || !r.out) return e;
    return launch_reduce(r, 1, adj_march_num_blocks(p), stream);
}

}  // namespace lwacm
