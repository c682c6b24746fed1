// lwacm_march.hip -- D3Q19 LW-ACM forward step as a z-marching tile kernel.
//
// Design (gfx950).  A workgroup owns a TX x TY tile of (x, y) columns and a
// chunk of NZC planes; every thread owns one column and walks up the chunk.
// For each plane it loads the node's state once (three planes in flight in
// a register ring), evaluates the node's own pre-combined link terms of
// Eq. ACM2.0b and pushes them towards the columns that consume them.  Links
// are grouped by their (v_x, v_y) direction: the three links sharing a
// direction (v_z = -1, 0, +1) reach the same neighbouring column on three
// consecutive planes, so each column sums them in registers while marching
// and exchanges only two numbers per direction (density part and z-momentum
// part; the x/y momentum parts follow from the direction) plus one number
// per in-plane diagonal: 12 floats per node through LDS, instead of gathering
// 18 neighbour states.
//
// Waves have fixed roles.  Interior waves own the TX x TY tile and evaluate
// all 19 links.  Two halo waves own the ring of columns around the tile and
// evaluate only the five links that point into it: the Y-halo wave holds the
// rows below and above the tile (links with v_y = +1 resp. -1), the X-halo
// wave the columns left and right of it including the corners (v_x = +1 resp.
// -1); one lane-dependent sign selects the direction, so a halo wave runs one
// instruction stream without divergence.
//
// The receiving column adds the exchanged terms, its own (v_x, v_y) = (0, 0)
// links and the post-combine term a rho u (Eqs. ACM2.0b), normalises, and
// stores.  Forced problems (Eq. force) run on the generic kernel, which adds
// the forcing inside each link term where its FP32 rounding does not bias
// long runs.  Halfway bounce-back (Eqs. ACM2.0cbb-ACM2.0ccccbb) is applied at
// the receiving node from a precomputed per-node bit set of solid upstream
// links; solid nodes push zeros and are never written.
//
// Link terms are kept unweighted and summed with the exact integer weights
// 12, 2, 1 (= 36 w_i for rest, axis and diagonal links of D3Q19); the sums
// are divided by 36 once at the end (div36: no systematic rounding bias).
#include <type_traits>
#include <utility>

#include "lwacm_device.hpp"
#include "lwacm_internal.hpp"

namespace lwacm {

namespace {

#ifndef LWACM_MARCH_NBUF
#define LWACM_MARCH_NBUF 2
#endif
#ifndef LWACM_MARCH_RING
#define LWACM_MARCH_RING 3
#endif
constexpr int TX = 32;                // tile width (x, contiguous in memory)
constexpr int TY = 16;                // tile height (y)
// Planes per workgroup: a template parameter (the plane loop is fully
// unrolled), chosen per problem among kChunkDepths by march_choose_nzc().
constexpr int kChunkDepths[3] = {32, 64, 128};
// LDS exchange buffers: 2 = one barrier per plane; 1 = half the LDS (more
// workgroups per CU) at the cost of a second barrier per plane.
constexpr int NBUF = LWACM_MARCH_NBUF;
// Planes of state in flight per thread (register ring).
constexpr int RING = LWACM_MARCH_RING;
constexpr int NINT = TX * TY;                  // interior columns (whole waves)
constexpr int NTHREADS = NINT + 2 * kWave;     // + Y-halo wave + X-halo wave
constexpr int SX = TX + 2;                     // LDS row pitch (slots)
constexpr int NSLOT = SX * (TY + 2);           // slots per exchange group

static_assert(NINT % kWave == 0, "interior must be whole waves");
static_assert(2 * TX <= kWave && 2 * (TY + 2) <= kWave, "halo rows must fit one wave each");

enum Role { INTERIOR = 0, HALO_Y = 1, HALO_X = 2 };

// Exchanged quantities per slot, in arrays of one kind each so that every
// LDS access has a 4- or 8-byte lane stride (no bank conflicts):
//   xp[0..3] = (PE, ZE), (PW, ZW), (PN, ZN), (PS, ZS): density and z parts of
//              the links with (vx, vy) = (+1,0), (-1,0), (0,+1), (0,-1)
//   xd[0..3] = NE, NW, SE, SW: in-plane diagonals (+1,+1,0), (-1,+1,0),
//              (+1,-1,0), (-1,-1,0)

// Per target plane accumulator of an interior column.
// Compile-time loop: f(std::integral_constant<int, K>) for K = 0 .. N-1.
// The plane loop runs through it so that every ring and accumulator index is
// a constant expression from the start and all per-plane state stays in
// registers.
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

struct Acc {
    float pe, ze, pw, zw, pn, zn, ps, zs;  // direction partials (weights folded)
    float ne, nw, se, sw;                  // in-plane diagonals
    float d, jz;                           // own column: rest + (0,0,+-1) links
    float post[3];                         // a rho u of the node itself
    float own[6];                          // E0, 4.5 rho, A rho, u (bounce-back only)
    unsigned bits;                         // solid upstream links (bounce-back only)
    int cls;                               // 0 fluid, 1 fluid next to a wall, 2 solid
};

__device__ __forceinline__ bool has_bit(unsigned bits, int i) { return (bits >> i) & 1u; }

// Global memory goes through buffer resources: one descriptor per state
// buffer in SGPRs, the column's fixed 32-bit byte offset in a VGPR and the
// plane's byte offset as the scalar offset, so a load or store costs no
// per-lane address arithmetic.  The state is node-interleaved, so one node of
// one plane is a single 16-byte (FP32) or 8-byte (FP16) access.
// (march_supported() guarantees that a state buffer fits in 4 GiB.)
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ Rsrc make_rsrc(const void *base, unsigned long long bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0,
                                             (int)(unsigned)bytes, 0x00020000);
}

template <class T>
struct BufIO;

// Element access uses explicit .x/.y/.z/.w selection and whole-vector casts:
// this compiler narrows a 128-bit load to its first dword when elements of
// the loaded vector are taken apart with __builtin_bit_cast one by one.
template <>
struct BufIO<float> {
    using Raw = f32x4;
    static constexpr unsigned kNodeBytes = 16;
    __device__ __forceinline__ static Raw load(Rsrc r, unsigned voff, unsigned soff)
    {
        return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    }
    // field f (0: rho - 1, 1..3: u) of a loaded node
    __device__ __forceinline__ static float value(const Raw &v, int f, float)
    {
        return f == 0 ? v.x : (f == 1 ? v.y : (f == 2 ? v.z : v.w));
    }
    __device__ __forceinline__ static void store(Rsrc r, unsigned voff, unsigned soff, float d,
                                                 float ux, float uy, float uz, const float (&)[2])
    {
        const f32x4 v = {d, ux, uy, uz};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, 0);
        store_data_guard();
    }
    __device__ __forceinline__ static void store_sr(Rsrc r, unsigned voff, unsigned soff, float d,
                                                    float ux, float uy, float uz,
                                                    const float (&sc)[2], const U32x4 &)
    {
        store(r, voff, soff, d, ux, uy, uz, sc);
    }
};

template <>
struct BufIO<__half> {
    using Raw = u32x2;
    static constexpr unsigned kNodeBytes = 8;
    __device__ __forceinline__ static Raw load(Rsrc r, unsigned voff, unsigned soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    }
    __device__ __forceinline__ static float value(const Raw &v, int f, float inv_scale)
    {
        const unsigned w = (f >> 1) ? v.y : v.x;
        const unsigned short h = (unsigned short)((f & 1) ? w >> 16 : w & 0xffffu);
        return __half2float(__ushort_as_half(h)) * inv_scale;
    }
    __device__ __forceinline__ static void put(Rsrc r, unsigned voff, unsigned soff,
                                               unsigned short b0, unsigned short b1,
                                               unsigned short b2, unsigned short b3)
    {
        const Raw v = {(unsigned)b0 | ((unsigned)b1 << 16), (unsigned)b2 | ((unsigned)b3 << 16)};
        __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
        store_data_guard();
    }
    __device__ __forceinline__ static void store(Rsrc r, unsigned voff, unsigned soff, float d,
                                                 float ux, float uy, float uz,
                                                 const float (&st)[2])
    {
        put(r, voff, soff, __half_as_ushort(__float2half_rn(d * st[0])),
            __half_as_ushort(__float2half_rn(ux * st[1])),
            __half_as_ushort(__float2half_rn(uy * st[1])),
            __half_as_ushort(__float2half_rn(uz * st[1])));
    }
    __device__ __forceinline__ static void store_sr(Rsrc r, unsigned voff, unsigned soff, float d,
                                                    float ux, float uy, float uz,
                                                    const float (&st)[2], const U32x4 &h)
    {
        put(r, voff, soff, half_bits_sr(d * st[0], h.x), half_bits_sr(ux * st[1], h.y),
            half_bits_sr(uy * st[1], h.z), half_bits_sr(uz * st[1], h.w));
    }
};

template <class T>
struct Ring {
    typename BufIO<T>::Raw v;  // the node's stored values on one plane
    uint8_t cls;
};

// Unweighted link term with c = v_i . u (Eq. ACM2.0b pre-combining,
// deviation form): L(c) = fma(A rho, c, m) with the even part
// m = fma(4.5 rho c, c, E0).  m is bitwise even in c, so the pair of opposite
// links shares it, and interior and halo threads, which both use exactly
// these operations (the build disables FMA contraction), produce bitwise the
// same term for a given link.
__device__ __forceinline__ float lterm(float c, float E0, float r45, float rA)
{
    return fmaf(rA, c, fmaf(r45 * c, c, E0));
}

template <class T, bool MASK, int NZC>
__global__ __launch_bounds__(NTHREADS) void k_fwd_march(ProblemArgs p, const T *__restrict__ src,
                                                        T *__restrict__ dst,
                                                        const uint8_t *__restrict__ cls_arr,
                                                        const unsigned *__restrict__ bb_bits,
                                                        const float4 *__restrict__ wallg,
                                                        ReduceArgs r)
{
    __shared__ float2 xp[NBUF][4][NSLOT];
    __shared__ float xd[NBUF][4][NSLOT];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long n = p.n;
    const long long plane = (long long)nx * ny;

    // XCD-aware order: consecutive blocks of one XCD get neighbouring tiles.
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

    // Role and column in tile coordinates [-1, TX] x [-1, TY].
    const int role = tid < NINT ? INTERIOR : (tid < NINT + kWave ? HALO_Y : HALO_X);
    int lx, ly;
    float sgn = 1.0f;     // halo direction sign
    bool active = true;   // writes to LDS
    if (role == INTERIOR) {
        lx = tid % TX;
        ly = tid / TX;
    } else if (role == HALO_Y) {
        // lanes [0, TX): row below the tile, pushing north (v_y = +1);
        // lanes [TX, 2 TX): row above, pushing south (v_y = -1).
        const bool top = lane >= TX;
        lx = top ? lane - TX : lane;
        ly = top ? TY : -1;
        sgn = top ? -1.0f : 1.0f;
        active = lane < 2 * TX;
        if (!active) lx = 0;
    } else {
        // lanes [0, TY+2): column left of the tile (corners included), pushing
        // east (v_x = +1); lanes [TY+2, 2(TY+2)): right column, pushing west.
        const bool right = lane >= TY + 2;
        const int l = right ? lane - (TY + 2) : lane;
        lx = right ? TX : -1;
        ly = l - 1;
        sgn = right ? -1.0f : 1.0f;
        active = lane < 2 * (TY + 2);
        if (!active) ly = 0;
    }
    int gx = tile_x * TX + lx;
    int gy = tile_y * TY + ly;
    gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
    gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
    const unsigned col = (unsigned)(gy * nx + gx);  // offset inside a plane (< 2^31)
    const int slot = (ly + 1) * SX + (lx + 1);

    const float A = p.A;
    const float a = p.a;

    // plane index with periodic wrap, as a byte offset inside the state
    constexpr unsigned NB = BufIO<T>::kNodeBytes;
    const unsigned plane_bytes = (unsigned)(plane * (long long)NB);
    auto soff_of = [&](int pz) -> unsigned {
        pz = pz < 0 ? pz + nz : (pz >= nz ? pz - nz : pz);
        return (unsigned)pz * plane_bytes;
    };
    const unsigned long long sbytes = (unsigned long long)n * NB;
    const Rsrc rs = make_rsrc(src, sbytes);
    const Rsrc rd = make_rsrc(dst, sbytes);
    const unsigned voff = col * NB;
    auto issue = [&](Ring<T> &rg, int pz) {
        const unsigned so = soff_of(pz);
        rg.v = BufIO<T>::load(rs, voff, so);
        if (MASK) {
            pz = pz < 0 ? pz + nz : (pz >= nz ? pz - nz : pz);
            rg.cls = cls_arr[(long long)pz * plane + col];
        }
    };

    Ring<T> ring[RING];
#pragma unroll
    for (int j = 0; j < RING; ++j) {
        ring[j].cls = 0;
        issue(ring[j], min(z0 - 1 + j, z1));
    }

    float mass = 0.0f, energy = 0.0f;

    // The two roles run separate loops (a wave-uniform split) with the same
    // sequence of barriers: one per finalised plane.
    if (role == INTERIOR) {
        Acc acc[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[j] = Acc{};
        // Fully unrolled over the chunk: ring slots and accumulators are
        // compile-time indexed, so no loop back edge forces the compiler to
        // copy registers whose loads are still in flight.
        static_for<NZC + 2>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            {
                const int j = k % 3;         // accumulator slot
                const int rj = k % RING;     // ring slot
                const int pz = z0 - 1 + k;  // source plane of this iteration
                Acc &A1 = acc[(j + 1) % 3];  // target plane pz + 1
                Acc &A0 = acc[j];            // target plane pz
                Acc &Am = acc[(j + 2) % 3];  // target plane pz - 1 (finalised now)

                // ---- consume the ring slot of plane pz, refill it with pz + 3
                const float dr = BufIO<T>::value(ring[rj].v, 0, p.ld_scale[0]);
                const float ux = BufIO<T>::value(ring[rj].v, 1, p.ld_scale[1]);
                const float uy = BufIO<T>::value(ring[rj].v, 2, p.ld_scale[1]);
                const float uz = BufIO<T>::value(ring[rj].v, 3, p.ld_scale[1]);
                const int cls = MASK ? (int)ring[rj].cls : 0;
                // refill with plane pz + RING (unconditional; past the chunk it
                // re-reads plane z1, which is cached and never consumed)
                if (k + RING < NZC + 2) issue(ring[rj], min(pz + RING, z1));

                // ---- own link terms in +-c pairs:
                // L(+-c) = E0 + 4.5 rho c^2 +- A rho c, E0 = drho - 1.5 rho |u|^2
                const float rho = 1.0f + dr;
                const float usq = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
                float E0 = fmaf(rho, -1.5f * usq, dr);
                float r45 = 4.5f * rho;
                float rA = A * rho;
                if (MASK && cls >= 2) {  // solid: push nothing
                    E0 = 0.0f;
                    r45 = 0.0f;
                    rA = 0.0f;
                }
                auto pair = [&](float c, float &lp, float &lm) {
                    const float m = fmaf(r45 * c, c, E0);  // = lterm's even part
                    lp = fmaf(rA, c, m);                   // = lterm(c)
                    lm = fmaf(rA, -c, m);                  // = lterm(-c)
                };
                float Lpx, Lmx, Lpy, Lmy, Lpz, Lmz;
                float Lpp0, Lmm0, Lpm0, Lmp0;  // (+x+y), (-x-y), (+x-y), (-x+y)
                float Lp0p, Lm0m, Lp0m, Lm0p;  // (+x,+z), (-x,-z), (+x,-z), (-x,+z)
                float L0pp, L0mm, L0pm, L0mp;  // (+y,+z), (-y,-z), (+y,-z), (-y,+z)
                pair(ux, Lpx, Lmx);
                pair(uy, Lpy, Lmy);
                pair(uz, Lpz, Lmz);
                pair(ux + uy, Lpp0, Lmm0);
                pair(ux - uy, Lpm0, Lmp0);
                pair(ux + uz, Lp0p, Lm0m);
                pair(ux - uz, Lp0m, Lm0p);
                pair(uy + uz, L0pp, L0mm);
                pair(uy - uz, L0pm, L0mp);

                // links with v_z = +1 start the accumulator of plane pz + 1
                A1.pe = Lp0p;
                A1.ze = Lp0p;
                A1.pw = Lm0p;
                A1.zw = Lm0p;
                A1.pn = L0pp;
                A1.zn = L0pp;
                A1.ps = L0mp;
                A1.zs = L0mp;
                A1.d = 2.0f * Lpz;
                A1.jz = 2.0f * Lpz;
                // links with v_z = 0 complete the in-plane part of plane pz
                A0.pe = fmaf(2.0f, Lpx, A0.pe);
                A0.pw = fmaf(2.0f, Lmx, A0.pw);
                A0.pn = fmaf(2.0f, Lpy, A0.pn);
                A0.ps = fmaf(2.0f, Lmy, A0.ps);
                A0.ne = Lpp0;
                A0.nw = Lmp0;
                A0.se = Lpm0;
                A0.sw = Lmm0;
                A0.d = fmaf(12.0f, E0, A0.d);
                const float arho = a * rho;
                A0.post[0] = arho * ux;
                A0.post[1] = arho * uy;
                A0.post[2] = arho * uz;
                if (MASK) {
                    A0.cls = cls;
                    A0.bits = 0u;
                    // only planes this chunk finalises (z0 <= pz < z1 <= nz)
                    if (cls == 1 && pz >= z0 && pz < z1)
                        A0.bits = bb_bits[(long long)pz * plane + col];
                    A0.own[0] = E0;
                    A0.own[1] = r45;
                    A0.own[2] = rA;
                    A0.own[3] = ux;
                    A0.own[4] = uy;
                    A0.own[5] = uz;
                }
                // links with v_z = -1 finish plane pz - 1
                Am.pe += Lp0m;
                Am.ze -= Lp0m;
                Am.pw += Lm0m;
                Am.zw -= Lm0m;
                Am.pn += L0pm;
                Am.zn -= L0pm;
                Am.ps += L0mm;
                Am.zs -= L0mm;
                Am.d = fmaf(2.0f, Lmz, Am.d);
                Am.jz = fmaf(-2.0f, Lmz, Am.jz);

                if (k < 2) return;  // planes below the chunk are halo only
                // ---- exchange the partials of plane pz - 1 through LDS
                if (NBUF == 1 && k > 2) __syncthreads();  // previous plane's reads done
                float2(*P)[NSLOT] = xp[k % NBUF];
                float(*Dg)[NSLOT] = xd[k % NBUF];
                P[0][slot] = make_float2(Am.pe, Am.ze);
                P[1][slot] = make_float2(Am.pw, Am.zw);
                P[2][slot] = make_float2(Am.pn, Am.zn);
                P[3][slot] = make_float2(Am.ps, Am.zs);
                Dg[0][slot] = Am.ne;
                Dg[1][slot] = Am.nw;
                Dg[2][slot] = Am.se;
                Dg[3][slot] = Am.sw;
                __syncthreads();
                const float2 gW = P[0][slot - 1];   // west neighbour: PE, ZE
                const float2 gE = P[1][slot + 1];   // east neighbour: PW, ZW
                const float2 gS = P[2][slot - SX];  // south: PN, ZN
                const float2 gN = P[3][slot + SX];  // north: PS, ZS
                const float dNE = Dg[0][slot - SX - 1];
                const float dNW = Dg[1][slot - SX + 1];
                const float dSE = Dg[2][slot + SX - 1];
                const float dSW = Dg[3][slot + SX + 1];
                const float pE = gW.x, zE = gW.y, pW = gE.x, zW = gE.y;
                const float pN = gS.x, zN = gS.y, pS = gN.x, zS = gN.y;

                const int tz = pz - 1;
                if (tz >= z1) return;  // padding iteration: nothing to finalise
                float D36 = Am.d + ((pE + pW) + (pN + pS)) + ((dNE + dNW) + (dSE + dSW));
                float Jx = (pE - pW) + ((dNE - dNW) + (dSE - dSW));
                float Jy = (pN - pS) + ((dNE + dNW) - (dSE + dSW));
                float Jz = Am.jz + ((zE + zW) + (zN + zS));
                if (MASK && Am.bits != 0u) {
                    // halfway bounce-back: a solid upstream node x - v_i pushed
                    // nothing; the node's own term of the opposite link returns
                    // along i (recomputed from the node's saved coefficients:
                    // the same FMAs as pair(), so the same value).
#pragma unroll
                    for (int i = 1; i < 19; ++i) {
                        if (has_bit(Am.bits, i)) {
                            const int cx = link_cx(i), cy = link_cy(i), cz = link_cz(i);
                            float c = 0.0f;  // v_i . u, summed in the order pair() uses
                            if (cx != 0) c = cx > 0 ? c + Am.own[3] : c - Am.own[3];
                            if (cy != 0) c = cy > 0 ? c + Am.own[4] : c - Am.own[4];
                            if (cz != 0) c = cz > 0 ? c + Am.own[5] : c - Am.own[5];
                            const float m = fmaf(Am.own[1] * c, c, Am.own[0]);
                            const float s = Lattice<19>::w36(i) * fmaf(Am.own[2], -c, m);
                            D36 += s;
                            Jx = fmaf((float)cx, s, Jx);
                            Jy = fmaf((float)cy, s, Jy);
                            Jz = fmaf((float)cz, s, Jz);
                        }
                    }
                    // moving walls (Eq. ACM2.0ccccbb): (1 - a) 6 rho0 times the
                    // node's geometry sums of 36 w_i (1, v_i) (v_i . u_w)
                    if (Am.bits & kMovingWallFlag) {
                        const float4 g = wallg[(long long)tz * plane + col];
                        D36 = fmaf(p.wall_scale, g.x, D36);
                        Jx = fmaf(p.wall_scale, g.y, Jx);
                        Jy = fmaf(p.wall_scale, g.z, Jy);
                        Jz = fmaf(p.wall_scale, g.w, Jz);
                    }
                }
                Jx = div36(Jx) + Am.post[0];
                Jy = div36(Jy) + Am.post[1];
                Jz = div36(Jz) + Am.post[2];
                const float D = div36(D36);
                const float q = normalisation_factor(D);
                const float vx = fmaf(-Jx, q, Jx);
                const float vy = fmaf(-Jy, q, Jy);
                const float vz = fmaf(-Jz, q, Jz);
                if (!MASK || Am.cls < 2) {
                    const unsigned so = (unsigned)tz * plane_bytes;
                    if (std::is_same<T, __half>::value && p.fp16_sr) {
                        const U32x4 h = pcg4d((uint32_t)gx, (uint32_t)gy, (uint32_t)tz, p.sr_word);
                        BufIO<T>::store_sr(rd, voff, so, D, vx, vy, vz, p.st_scale, h);
                    } else {
                        BufIO<T>::store(rd, voff, so, D, vx, vy, vz, p.st_scale);
                    }
                    mass += D;
                    energy = fmaf(vx, vx, fmaf(vy, vy, fmaf(vz, vz, energy)));
                }
            }
        });
    } else {
        // Halo columns: one direction partial (density part p, z part z) and
        // the two in-plane diagonals next to it, for three target planes.
        float hp[3] = {0.0f, 0.0f, 0.0f}, hz[3] = {0.0f, 0.0f, 0.0f};
        float hd1[3] = {0.0f, 0.0f, 0.0f}, hd2[3] = {0.0f, 0.0f, 0.0f};
        static_for<NZC + 2>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            {
                const int j = k % 3;
                const int rj = k % RING;
                const int pz = z0 - 1 + k;
                const int j1 = (j + 1) % 3, jm = (j + 2) % 3;
                const float dr = BufIO<T>::value(ring[rj].v, 0, p.ld_scale[0]);
                const float ux = BufIO<T>::value(ring[rj].v, 1, p.ld_scale[1]);
                const float uy = BufIO<T>::value(ring[rj].v, 2, p.ld_scale[1]);
                const float uz = BufIO<T>::value(ring[rj].v, 3, p.ld_scale[1]);
                const int cls = MASK ? (int)ring[rj].cls : 0;
                // refill with plane pz + RING (unconditional; past the chunk it
                // re-reads plane z1, which is cached and never consumed)
                if (k + RING < NZC + 2) issue(ring[rj], min(pz + RING, z1));
                const float rho = 1.0f + dr;
                const float usq = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
                float E0 = fmaf(rho, -1.5f * usq, dr);
                float r45 = 4.5f * rho;
                float rA = A * rho;
                if (MASK && cls >= 2) {
                    E0 = 0.0f;
                    r45 = 0.0f;
                    rA = 0.0f;
                }
                // the five links with v_y = sgn (Y halo) or v_x = sgn (X halo)
                const float ua = (role == HALO_Y) ? uy : ux;  // along the halo direction
                const float ub = (role == HALO_Y) ? ux : uy;  // across it, in plane
                const float cs = sgn * ua;
                const float Lup = lterm(cs + uz, E0, r45, rA);  // v_z = +1
                const float Lmid = lterm(cs, E0, r45, rA);      // v_z = 0
                const float Ldn = lterm(cs - uz, E0, r45, rA);  // v_z = -1
                hp[j1] = Lup;
                hz[j1] = Lup;
                hp[j] = fmaf(2.0f, Lmid, hp[j]);
                hd1[j] = lterm(cs + ub, E0, r45, rA);  // diagonal, + across
                hd2[j] = lterm(cs - ub, E0, r45, rA);  // diagonal, - across
                hp[jm] += Ldn;
                hz[jm] -= Ldn;
                if (k < 2) return;
                if (NBUF == 1 && k > 2) __syncthreads();
                float2(*P)[NSLOT] = xp[k % NBUF];
                float(*Dg)[NSLOT] = xd[k % NBUF];
                if (active) {
                    const int hi = sgn > 0.0f ? 0 : 1;
                    if (role == HALO_Y) {
                        // (PN, ZN) below the tile or (PS, ZS) above it;
                        // diagonals (NE, NW) below or (SE, SW) above
                        P[2 + hi][slot] = make_float2(hp[jm], hz[jm]);
                        Dg[2 * hi][slot] = hd1[jm];
                        Dg[2 * hi + 1][slot] = hd2[jm];
                    } else {
                        // (PE, ZE) left of the tile or (PW, ZW) right of it;
                        // diagonals NE, SE (left) or NW, SW (right)
                        P[hi][slot] = make_float2(hp[jm], hz[jm]);
                        Dg[hi][slot] = hd1[jm];      // (sgn, +1, 0)
                        Dg[hi + 2][slot] = hd2[jm];  // (sgn, -1, 0)
                    }
                }
                __syncthreads();
            }
        });
    }

    double v[2] = {(double)mass, 0.5 * (double)energy};
    store_block_partials<2>(v, r.partials, blockIdx.x);
    if (blockIdx.x == 0 && r.prev_nblocks)
        finish_previous_sums(r.prev_partials, r.prev_nblocks, r.prev_out, r.prev_out2);
}

// Node classes and solid-upstream bit sets for the bounce-back of the march
// kernel: class 0 fluid with only fluid upstream nodes, 1 fluid with at
// least one solid upstream node (bit i set when x - v_i is solid), 2 solid.
// For a fluid node whose solid upstream nodes include a moving wall, the
// flag bit is set and wallg holds sum_i 36 w_i (v_i . u_w(x - v_i)) times
// (1, v_i) over its bounce-back links: the moving-wall term per unit of
// (1 - a) 6 rho0, which depends on the geometry only.
__global__ __launch_bounds__(256) void k_classify(ProblemArgs p, uint8_t *cls, unsigned *bits,
                                                  float4 *wallg)
{
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < p.n;
         idx += (long long)gridDim.x * blockDim.x) {
        if (p.mask[idx] != 0) {
            cls[idx] = 2;
            bits[idx] = 0u;
            continue;
        }
        const long long t = idx / p.nx;
        const int x = (int)(idx - t * p.nx);
        const int z = (int)(t / p.ny);
        const int y = (int)(t - (long long)z * p.ny);
        unsigned bb = 0u;
        float g[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        bool moving = false;
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            const int cx = link_cx(i), cy = link_cy(i), cz = link_cz(i);
            int ux = x - cx, uy = y - cy, uz = z - cz;
            ux = ux < 0 ? ux + p.nx : (ux >= p.nx ? ux - p.nx : ux);
            uy = uy < 0 ? uy + p.ny : (uy >= p.ny ? uy - p.ny : uy);
            uz = uz < 0 ? uz + p.nz : (uz >= p.nz ? uz - p.nz : uz);
            const int m = p.mask[((long long)uz * p.ny + uy) * p.nx + ux];
            if (m != 0) {
                bb |= 1u << i;
                const float vu = cx * p.wall_u[m][0] + cy * p.wall_u[m][1] + cz * p.wall_u[m][2];
                if (vu != 0.0f) {
                    moving = true;
                    const float s = Lattice<19>::w36(i) * vu;
                    g[0] += s;
                    g[1] += cx * s;
                    g[2] += cy * s;
                    g[3] += cz * s;
                }
            }
        }
        if (moving && wallg) {
            bb |= kMovingWallFlag;
            wallg[idx] = make_float4(g[0], g[1], g[2], g[3]);
        }
        cls[idx] = bb ? 1 : 0;
        bits[idx] = bb;
    }
}

template <class T>
hipError_t dispatch(const ProblemArgs &p, const void *src, void *dst, const uint8_t *cls,
                    const unsigned *bits, const float4 *wallg, const ReduceArgs &r,
                    hipStream_t s)
{
    const unsigned nb = march_num_blocks(p);
    const T *a = static_cast<const T *>(src);
    T *b = static_cast<T *>(dst);
#define LWACM_LAUNCH(Z)                                                                   \
    if (p.mask)                                                                           \
        k_fwd_march<T, true, Z><<<nb, NTHREADS, 0, s>>>(p, a, b, cls, bits, wallg, r);    \
    else                                                                                  \
        k_fwd_march<T, false, Z><<<nb, NTHREADS, 0, s>>>(p, a, b, cls, bits, wallg, r);
    switch (p.march_nzc) {
    case 32: LWACM_LAUNCH(32) break;
    case 64: LWACM_LAUNCH(64) break;
    case 128: LWACM_LAUNCH(128) break;
    default: return hipErrorInvalidValue;
    }
#undef LWACM_LAUNCH
    return hipGetLastError();
}

}  // namespace

bool march_supported(const ProblemArgs &p)
{
    // 32-bit byte offsets inside a state buffer: n * 16 bytes < 4 GiB
    return p.Q == 19 && !p.has_force && p.nx >= TX && p.ny >= TY && p.nx % TX == 0 &&
           p.ny % TY == 0 && p.nz >= 1 && p.n < (1LL << 28);
}

static long long march_blocks_for(const ProblemArgs &p, int nzc)
{
    const long long tiles = (long long)(p.nx / TX) * (p.ny / TY);
    return tiles * ((p.nz + nzc - 1) / nzc);
}

int march_choose_nzc(const ProblemArgs &p, int ncu)
{
    // Per-CU work: the workgroups a CU receives run one after the other or
    // share it, so the step time follows ceil(blocks / CUs) * (chunk planes +
    // the two halo planes).  Ties go to the deeper chunk (fewer halo planes).
    if (ncu < 1) ncu = 1;
    int best = kChunkDepths[0];
    long long best_cost = -1;
    for (int c : kChunkDepths) {
        const long long nb = march_blocks_for(p, c);
        const long long cost = ((nb + ncu - 1) / ncu) * (c + 2);
        if (best_cost < 0 || cost <= best_cost) {
            best = c;
            best_cost = cost;
        }
    }
    return best;
}

unsigned march_num_blocks(const ProblemArgs &p)
{
    if (!march_supported(p) || p.march_nzc <= 0) return 0;
    return (unsigned)march_blocks_for(p, p.march_nzc);
}

hipError_t launch_classify(const ProblemArgs &p, uint8_t *cls, unsigned *bits, float4 *wallg,
                           hipStream_t s)
{
    long long nb = (p.n + 255) / 256;
    if (nb > 4096) nb = 4096;
    k_classify<<<(unsigned)nb, 256, 0, s>>>(p, cls, bits, wallg);
    return hipGetLastError();
}

hipError_t launch_fwd_march(const ProblemArgs &p, int storage, const void *src, void *dst,
                            const uint8_t *cls, const unsigned *bits, const float4 *wallg,
                            const ReduceArgs &r, hipStream_t s)
{
    if (!march_supported(p) || (p.mask && (!cls || !bits))) return hipErrorNotSupported;
    return storage ? dispatch<__half>(p, src, dst, cls, bits, wallg, r, s)
                   : dispatch<float>(p, src, dst, cls, bits, wallg, r, s);
}

}  // namespace lwacm
