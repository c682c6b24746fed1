// lwacm_march_common.hpp -- pieces shared by the D3Q19 z-marching tile
// kernels: compile-time plane loop, per-plane accumulators, buffer-resource
// loads and stores of the node-interleaved state, and the link term.
#pragma once

#include <type_traits>
#include <utility>

#include "lwacm_device.hpp"
#include "lwacm_internal.hpp"

namespace lwacm {

namespace {

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

// Plane loop of N >= 9 iterations in small code: six specialised iterations,
// a loop unrolled by three (the period of the accumulator and load-ring
// rotations, so every register index stays a compile-time constant and the
// back edge needs no copies), then three to five specialised iterations, so
// that every loop iteration has a plane left to prefetch.  The body is called
// as body(k, K) with the iteration index k and a std::integral_constant K:
// K = k in the specialised iterations, K = k % 3 - 3 in the loop, so that
// k % 3, the early-iteration phases and the prefetch condition are all
// compile-time constants.
template <int N, class F>
__device__ __forceinline__ void plane_loop(F &&body)
{
    static_assert(N >= 9, "plane loop needs at least nine iterations");
    constexpr int T = 3 + (N - 9) % 3;  // specialised tail iterations
    static_for<6>([&](auto kc) { body((int)decltype(kc)::value, kc); });
#pragma unroll 1
    for (int k = 6; k < N - T; k += 3) {
        body(k, std::integral_constant<int, -3>{});
        body(k + 1, std::integral_constant<int, -2>{});
        body(k + 2, std::integral_constant<int, -1>{});
    }
    static_for<T>([&](auto tc) {
        constexpr int k = N - T + decltype(tc)::value;
        body(k, std::integral_constant<int, k>{});
    });
}

// What a plane-loop body needs to know about iteration K at compile time.
template <int K, int N, int RING>
struct PlaneIter {
    static constexpr int j = K >= 0 ? K % 3 : K + 3;     // k % 3
    static constexpr int phase = K >= 0 && K < 5 ? K : 5;  // min(k, 5)
    static constexpr bool refill = K < 0 || K + RING < N;  // a plane left to prefetch
};

// Per target plane accumulator of an interior column.
struct Acc {
    float pe, ze, pw, zw, pn, zn, ps, zs;  // direction partials (weights folded)
    float ne, nw, se, sw;                  // in-plane diagonals
    float d, jz;                           // own column: rest + (0,0,+-1) links
    float post[3];                         // a rho u of the node itself
    float bb[4];                           // bounced-back terms: 36 w (1, v) sums (MASK)
    // separate omega_p (SPLIT): 36 w (Ap - A) rho (v . u) over the same links
    // as pe .. sw and as the own column's z links
    // (or, for the fused temperature step, the temperature terms over them)
    float qe, qw, qn, qs, qne, qnw, qse, qsw, qd;
    float tx;                              // the node's own T (fused temperature step)
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

// Cache-policy bits of the state's buffer loads and stores (gfx950: bit 0
// sc0, bit 1 nt, bit 4 sc1).
constexpr int kStateLoadAux = 0;
constexpr int kStateStoreAux = 0;

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
        return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kStateLoadAux));
    }
    // field f (0: rho - 1, 1..3: u) of a loaded node
    __device__ __forceinline__ static float value(const Raw &v, int f, float)
    {
        return f == 0 ? v.x : (f == 1 ? v.y : (f == 2 ? v.z : v.w));
    }
    // a node's new values in storage format
    __device__ __forceinline__ static Raw pack(float d, float ux, float uy, float uz,
                                               const float (&)[2])
    {
        const f32x4 v = {d, ux, uy, uz};
        return v;
    }
    __device__ __forceinline__ static Raw pack_sr(float d, float ux, float uy, float uz,
                                                  const float (&sc)[2], const U32x4 &)
    {
        return pack(d, ux, uy, uz, sc);
    }
    __device__ __forceinline__ static void store_raw(Rsrc r, unsigned voff, unsigned soff,
                                                     const Raw &v)
    {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, kStateStoreAux);
        store_data_guard();
    }
    __device__ __forceinline__ static void store(Rsrc r, unsigned voff, unsigned soff, float d,
                                                 float ux, float uy, float uz, const float (&sc)[2])
    {
        store_raw(r, voff, soff, pack(d, ux, uy, uz, sc));
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
        return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kStateLoadAux);
    }
    __device__ __forceinline__ static float value(const Raw &v, int f, float inv_scale)
    {
        const unsigned w = (f >> 1) ? v.y : v.x;
        const unsigned short h = (unsigned short)((f & 1) ? w >> 16 : w & 0xffffu);
        return __half2float(__ushort_as_half(h)) * inv_scale;
    }
    __device__ __forceinline__ static Raw bits4(unsigned short b0, unsigned short b1,
                                                unsigned short b2, unsigned short b3)
    {
        const Raw v = {(unsigned)b0 | ((unsigned)b1 << 16), (unsigned)b2 | ((unsigned)b3 << 16)};
        return v;
    }
    // a node's new values in storage format: scaled deviations, rounded to
    // nearest or stochastically (random words h)
    __device__ __forceinline__ static Raw pack(float d, float ux, float uy, float uz,
                                               const float (&st)[2])
    {
        return bits4(__half_as_ushort(__float2half_rn(d * st[0])),
                     __half_as_ushort(__float2half_rn(ux * st[1])),
                     __half_as_ushort(__float2half_rn(uy * st[1])),
                     __half_as_ushort(__float2half_rn(uz * st[1])));
    }
    __device__ __forceinline__ static Raw pack_sr(float d, float ux, float uy, float uz,
                                                  const float (&st)[2], const U32x4 &h)
    {
        const Raw v = {half2_bits_sr(d * st[0], h.x, ux * st[1], h.y),
                       half2_bits_sr(uy * st[1], h.z, uz * st[1], h.w)};
        return v;
    }
    __device__ __forceinline__ static void store_raw(Rsrc r, unsigned voff, unsigned soff,
                                                     const Raw &v)
    {
        __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, kStateStoreAux);
        store_data_guard();
    }
    __device__ __forceinline__ static void store(Rsrc r, unsigned voff, unsigned soff, float d,
                                                 float ux, float uy, float uz,
                                                 const float (&st)[2])
    {
        store_raw(r, voff, soff, pack(d, ux, uy, uz, st));
    }
    __device__ __forceinline__ static void store_sr(Rsrc r, unsigned voff, unsigned soff, float d,
                                                    float ux, float uy, float uz,
                                                    const float (&st)[2], const U32x4 &h)
    {
        store_raw(r, voff, soff, pack_sr(d, ux, uy, uz, st, h));
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


// Exchanged quantities per LDS slot, in arrays of one kind each so that every
// LDS access has a 4- or 8-byte lane stride (no bank conflicts):
//   P[0..3] = (PE, ZE), (PW, ZW), (PN, ZN), (PS, ZS): density and z parts of
//             the links with (vx, vy) = (+1,0), (-1,0), (0,+1), (0,-1)
//   Dg[0..3] = NE, NW, SE, SW: in-plane diagonals (+1,+1,0), (-1,+1,0),
//              (+1,-1,0), (-1,-1,0)
template <int NS>
struct Xchg {
    float2 (*P)[NS];
    float (*Dg)[NS];
};

// The 18 moving links of a node with state (drho, u) on source plane pz,
// pre-combined (Eq. ACM2.0b) and pushed, with integer weights 36 w_i folded
// in, into the accumulators of its column: links with v_z = +1 start A1
// (plane pz + 1), links with v_z = 0 complete the in-plane part of A0 (plane
// pz) together with the rest link and the post-combine term a rho u, links
// with v_z = -1 finish Am (plane pz - 1).  Opposite links share the even part
// m(c) = E0 + 4.5 rho c^2 with E0 = drho - 1.5 rho |u|^2; a solid node pushes
// zeros.  With MASK, A0 also keeps the class and the coefficients that the
// bounce-back of its own links needs (its bit set is the caller's).
// Halfway bounce-back (Eq. ACM2.0cbb): when the upstream node x - v_i of a
// fluid node is solid (bit i of its link set), link i brings the node's own
// term for the opposite link -v_i, the term it sends into the wall.  Those
// terms are the L arguments here (unweighted, as push_column computes them),
// so the bounced terms are summed when the node is pushed, away from the
// plane's LDS exchange: bb = sum over the set links of 36 w_i L(-v_i) (1, v_i).
// Only waves with a lane next to a wall take this path (one scalar branch).
// It has no further branches: a branch per link or per face kept the
// compiler from overlapping these sums with the rest of the plane, and cost
// more than evaluating all 18 links.  Each link is selected per lane by
// AND-ing the term's bits with a mask made from bit i (all ones or zero).
__device__ __forceinline__ void push_bounce_back(unsigned bits, float Lpx, float Lmx, float Lpy,
                                                 float Lmy, float Lpz, float Lmz, float Lpp0,
                                                 float Lmm0, float Lpm0, float Lmp0, float Lp0p,
                                                 float Lm0m, float Lp0m, float Lm0p, float L0pp,
                                                 float L0mm, float L0pm, float L0mp, float bb[4])
{
    float sd = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f;
    if (__builtin_amdgcn_ballot_w64(bits > 1u) != 0ull) {
        // link (cx, cy, cz) of weight 36 w, bouncing back the term lo of (-cx, -cy, -cz)
        auto link = [&](auto cxc, auto cyc, auto czc, float lo) {
            constexpr int cx = decltype(cxc)::value, cy = decltype(cyc)::value;
            constexpr int cz = decltype(czc)::value;
            constexpr int i = link_index(cx, cy, cz);
            constexpr float w = Lattice<19>::w36(i);
            // bit i spread over the word: 0xffffffff when set, else 0
            const unsigned m = (unsigned)((int)(bits << (31 - i)) >> 31);
            const float t = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, lo) & m);
            // w t is exact (w = 1 or 2), so each fma rounds like adding 36 w_i L
            sd = fmaf(w, t, sd);
            if (cx != 0) sx = fmaf(cx * w, t, sx);
            if (cy != 0) sy = fmaf(cy * w, t, sy);
            if (cz != 0) sz = fmaf(cz * w, t, sz);
        };
        using P = std::integral_constant<int, 1>;
        using Z = std::integral_constant<int, 0>;
        using M = std::integral_constant<int, -1>;
        link(P{}, Z{}, Z{}, Lmx);
        link(M{}, Z{}, Z{}, Lpx);
        link(Z{}, P{}, Z{}, Lmy);
        link(Z{}, M{}, Z{}, Lpy);
        link(Z{}, Z{}, P{}, Lmz);
        link(Z{}, Z{}, M{}, Lpz);
        link(P{}, P{}, Z{}, Lmm0);
        link(M{}, M{}, Z{}, Lpp0);
        link(P{}, M{}, Z{}, Lmp0);
        link(M{}, P{}, Z{}, Lpm0);
        link(P{}, Z{}, P{}, Lm0m);
        link(M{}, Z{}, M{}, Lp0p);
        link(P{}, Z{}, M{}, Lm0p);
        link(M{}, Z{}, P{}, Lp0m);
        link(Z{}, P{}, P{}, L0mm);
        link(Z{}, M{}, M{}, L0pp);
        link(Z{}, P{}, M{}, L0mp);
        link(Z{}, M{}, P{}, L0pm);
    }
    bb[0] = sd;
    bb[1] = sx;
    bb[2] = sy;
    bb[3] = sz;
}

// bounce: sum the halfway bounced-back terms here; false where a per-step
// wall correction brings the whole wall term instead (interpolated walls,
// link velocities).
template <bool MASK>
__device__ __forceinline__ void push_column(float dr, float ux, float uy, float uz, int cls,
                                            unsigned bits, float A, float a, Acc &A1, Acc &A0,
                                            Acc &Am, bool bounce = true)
{
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
        A0.bits = bits;
        push_bounce_back(bounce ? bits : 0u, Lpx, Lmx, Lpy, Lmy, Lpz, Lmz, Lpp0, Lmm0, Lpm0, Lmp0,
                         Lp0p, Lm0m, Lp0m, Lm0p, L0pp, L0mm, L0pm, L0mp, A0.bb);
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
}

// A column's finished partials of one plane into its LDS slot.
template <int NS>
__device__ __forceinline__ void put_slot(const Xchg<NS> &X, int slot, const Acc &Am)
{
    X.P[0][slot] = make_float2(Am.pe, Am.ze);
    X.P[1][slot] = make_float2(Am.pw, Am.zw);
    X.P[2][slot] = make_float2(Am.pn, Am.zn);
    X.P[3][slot] = make_float2(Am.ps, Am.zs);
    X.Dg[0][slot] = Am.ne;
    X.Dg[1][slot] = Am.nw;
    X.Dg[2][slot] = Am.se;
    X.Dg[3][slot] = Am.sw;
}

struct NodeOut {
    float D, vx, vy, vz;  // new drho and u of Eqs. ACM2.0b
};

// Partials that the eight in-plane neighbour columns pushed into a node's
// column for one plane (LDS slots around `slot`, row pitch SXP).
struct Gathered {
    float pE, zE, pW, zW, pN, zN, pS, zS;  // axis directions: density and z parts
    float dNE, dNW, dSE, dSW;              // in-plane diagonals
};

template <int NS, int SXP>
__device__ __forceinline__ Gathered gather(const Xchg<NS> &X, int slot)
{
    const float2 gW = X.P[0][slot - 1];    // west neighbour: PE, ZE
    const float2 gE = X.P[1][slot + 1];    // east neighbour: PW, ZW
    const float2 gS = X.P[2][slot - SXP];  // south: PN, ZN
    const float2 gN = X.P[3][slot + SXP];  // north: PS, ZS
    Gathered g;
    g.pE = gW.x;
    g.zE = gW.y;
    g.pW = gE.x;
    g.zW = gE.y;
    g.pN = gS.x;
    g.zN = gS.y;
    g.pS = gN.x;
    g.zS = gN.y;
    g.dNE = X.Dg[0][slot - SXP - 1];
    g.dNW = X.Dg[1][slot - SXP + 1];
    g.dSE = X.Dg[2][slot + SXP - 1];
    g.dSW = X.Dg[3][slot + SXP + 1];
    return g;
}

// New moments of a node (Eqs. ACM2.0b): the links arriving from the
// neighbour columns, the column's own partials and post-combine term,
// halfway bounce-back of the links whose upstream node is solid (Eqs.
// ACM2.0cbb-ACM2.0ccccbb: the node's own term of the opposite link returns,
// recomputed from its saved coefficients with the same operations, plus the
// moving-wall term from the geometry sums wallg[widx]), then the
// normalisation by 1 + D.
template <bool MASK, bool SPLIT = false>
__device__ __forceinline__ NodeOut finish(const Gathered &g, const Acc &Am, const ProblemArgs &p,
                                          const float4 *wallg, long long widx, float qsum = 0.0f,
                                          const f32x4 *cw = nullptr)
{
    float D36 = Am.d + ((g.pE + g.pW) + (g.pN + g.pS)) + ((g.dNE + g.dNW) + (g.dSE + g.dSW));
    float Jx = (g.pE - g.pW) + ((g.dNE - g.dNW) + (g.dSE - g.dSW));
    float Jy = (g.pN - g.pS) + ((g.dNE + g.dNW) - (g.dSE + g.dSW));
    float Jz = Am.jz + ((g.zE + g.zW) + (g.zN + g.zS));
    if (MASK) {
        // bounced-back terms (summed when the node was pushed; zero elsewhere)
        D36 += Am.bb[0];
        Jx += Am.bb[1];
        Jy += Am.bb[2];
        Jz += Am.bb[3];
        if (p.corr) {
            // interpolated walls or link velocities (Eqs. ACM2.0cc, ACM2.0move):
            // this step's whole wall term of every node next to a wall, wall
            // motion included, made by the wall-correction kernel (the push
            // summed no bounced-back terms: bb is zero); cw is the value the
            // caller loaded ahead (zero away from the walls)
            if (cw) {
                D36 += cw->x;
                Jx += cw->y;
                Jy += cw->z;
                Jz += cw->w;
            } else if (__builtin_amdgcn_ballot_w64(Am.bits > 1u) != 0ull && Am.bits > 1u) {
                const float4 w = p.corr[widx];
                D36 += w.x;
                Jx += w.y;
                Jy += w.z;
                Jz += w.w;
            }
        } else if (__builtin_amdgcn_ballot_w64((Am.bits & kMovingWallFlag) != 0u) != 0ull &&
                   (Am.bits & kMovingWallFlag)) {
            // moving walls (Eq. ACM2.0ccccbb): (1 - a) 6 rho0 times the node's
            // geometry sums of 36 w_i (1, v_i) (v_i . u_w)
            const float4 w = wallg[widx];
            D36 = fmaf(p.wall_scale, w.x, D36);
            Jx = fmaf(p.wall_scale, w.y, Jx);
            Jy = fmaf(p.wall_scale, w.z, Jy);
            Jz = fmaf(p.wall_scale, w.w, Jz);
        }
    }
    // separate omega_p: the density takes its link terms with Ap in place of A
    if (SPLIT) D36 += qsum;
    Jx = div36(Jx) + Am.post[0];
    Jy = div36(Jy) + Am.post[1];
    Jz = div36(Jz) + Am.post[2];
    NodeOut o;
    o.D = div36(D36);
    const float q = normalisation_factor(o.D);
    o.vx = fmaf(-Jx, q, Jx);
    o.vy = fmaf(-Jy, q, Jy);
    o.vz = fmaf(-Jz, q, Jz);
    return o;
}

template <bool MASK, int NS, int SXP, bool SPLIT = false>
__device__ __forceinline__ NodeOut finalize(const Xchg<NS> &X, int slot, const Acc &Am,
                                            const ProblemArgs &p, const float4 *wallg,
                                            long long widx, float qsum = 0.0f,
                                            const f32x4 *cw = nullptr)
{
    return finish<MASK, SPLIT>(gather<NS, SXP>(X, slot), Am, p, wallg, widx, qsum, cw);
}

// ---- separate omega_p for the density (Section "finite-difference
// formulation", item 3; Appendix E).  The density of the step sums the link
// terms with Ap = 3 (2/omega_p - 1) in place of A; a link term is linear in A
// through A rho (v . u), so the density gains, per incoming link,
// q = 36 w (Ap - A) rho_y (v . u_y).  Columns push q along the links that
// carry the density partials (pe .. sw, and the own column's z links), in
// eight LDS arrays of their own: e, w, n, s, ne, nw, se, sw.
template <int NS>
struct XchgQ {
    float (*Q)[NS];
};

// q of the links pushed by an interior column (the links and targets of
// push_column); rd = (Ap - A) rho, v . u formed as push_column forms it
__device__ __forceinline__ void push_split_column(float rho, float ux, float uy, float uz,
                                                  float dA, Acc &A1, Acc &A0, Acc &Am)
{
    const float rd = dA * rho;
    const float qx = rd * ux, qy = rd * uy, qz = rd * uz;
    const float qpp0 = rd * (ux + uy), qpm0 = rd * (ux - uy);
    const float qp0p = rd * (ux + uz), qp0m = rd * (ux - uz);
    const float q0pp = rd * (uy + uz), q0pm = rd * (uy - uz);
    // v_z = +1: start plane pz + 1
    A1.qe = qp0p;
    A1.qw = -qp0m;
    A1.qn = q0pp;
    A1.qs = -q0pm;
    A1.qd = 2.0f * qz;
    // v_z = 0: plane pz (the rest link has v . u = 0)
    A0.qe = fmaf(2.0f, qx, A0.qe);
    A0.qw = fmaf(-2.0f, qx, A0.qw);
    A0.qn = fmaf(2.0f, qy, A0.qn);
    A0.qs = fmaf(-2.0f, qy, A0.qs);
    A0.qne = qpp0;
    A0.qnw = -qpm0;
    A0.qse = qpm0;
    A0.qsw = -qpp0;
    // v_z = -1: finish plane pz - 1
    Am.qe += qp0m;
    Am.qw -= qp0p;
    Am.qn += q0pm;
    Am.qs -= q0pp;
    Am.qd = fmaf(-2.0f, qz, Am.qd);
}

// q of the five links a halo column pushes into the tile (push_halo's links)
__device__ __forceinline__ void push_split_halo(float rho, float ux, float uy, float uz,
                                                float dA, bool isY, float sgn, float &q1,
                                                float &q0, float &qd1, float &qd2, float &qm)
{
    const float rd = dA * rho;
    const float ua = isY ? uy : ux;
    const float ub = isY ? ux : uy;
    const float cs = sgn * ua;
    q1 = rd * (cs + uz);
    q0 = fmaf(2.0f, rd * cs, q0);
    qd1 = rd * (cs + ub);
    qd2 = rd * (cs - ub);
    qm += rd * (cs - uz);
}

// ---- temperature lattice fused into the single-step kernel (thermal
// LW-ACM, Eq. ACM2.0t with the even part of Eq. feqe, on the flow's
// lattice): the term a node with temperature T and velocity u sends along
// link v is w [h (T + 9/2 c^2 - 3/2 |u|^2) + 3 T c], c = v . u,
// h = 2/omega_t - 1, and the node's new T is (2 - 2/omega_t) T(x) plus the
// sum of the incoming terms.  The terms travel along the links that carry
// the density partials, in the omega_p arrays (q fields, XchgQ), which a
// problem with a temperature does not use.  Opposite links share the even
// part, as in push_column.
//
// Walls (MASK): a solid node pushes nothing and keeps its T.  Where the
// upstream node x - v_i of a fluid node is solid (bit i of its link set), the
// node's own term for the opposite link comes back along i: with its sign kept
// at an adiabatic wall, reversed at a wall held at T_w, which also adds
// 2 h 36 w_i T_w.  tw.x holds the node's links into fixed-temperature walls
// (bit i), tw.y the FP32 bits of the sum of 36 w_i T_w over them; the node's
// returned terms are summed when it is pushed (one wave-level test), like the
// flow's bounce-back.
template <bool MASK>
__device__ __forceinline__ void push_temp_column(float T, float ux, float uy, float uz, float h,
                                                 Acc &A1, Acc &A0, Acc &Am, int cls = 0,
                                                 unsigned bits = 0u, uint2 tw = {0u, 0u})
{
    const float usq = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
    float AT = h * fmaf(-1.5f, usq, T);
    float H = 4.5f * h, T3 = 3.0f * T;
    if (MASK && cls >= 2) {  // solid: push nothing
        AT = 0.0f;
        H = 0.0f;
        T3 = 0.0f;
    }
    auto pair = [&](float c, float &lp, float &lm) {
        const float m = fmaf(H * c, c, AT);
        lp = fmaf(T3, c, m);
        lm = fmaf(T3, -c, m);
    };
    float Tpx, Tmx, Tpy, Tmy, Tpz, Tmz;
    float Tpp0, Tmm0, Tpm0, Tmp0, Tp0p, Tm0m, Tp0m, Tm0p, T0pp, T0mm, T0pm, T0mp;
    pair(ux, Tpx, Tmx);
    pair(uy, Tpy, Tmy);
    pair(uz, Tpz, Tmz);
    pair(ux + uy, Tpp0, Tmm0);
    pair(ux - uy, Tpm0, Tmp0);
    pair(ux + uz, Tp0p, Tm0m);
    pair(ux - uz, Tp0m, Tm0p);
    pair(uy + uz, T0pp, T0mm);
    pair(uy - uz, T0pm, T0mp);
    // v_z = +1: plane pz + 1
    A1.qe = Tp0p;
    A1.qw = Tm0p;
    A1.qn = T0pp;
    A1.qs = T0mp;
    A1.qd = 2.0f * Tpz;
    // v_z = 0: plane pz, with the rest link (c = 0: the term AT, weight 12)
    A0.qe = fmaf(2.0f, Tpx, A0.qe);
    A0.qw = fmaf(2.0f, Tmx, A0.qw);
    A0.qn = fmaf(2.0f, Tpy, A0.qn);
    A0.qs = fmaf(2.0f, Tmy, A0.qs);
    A0.qne = Tpp0;
    A0.qnw = Tmp0;
    A0.qse = Tpm0;
    A0.qsw = Tmm0;
    A0.qd = fmaf(12.0f, AT, A0.qd);
    A0.tx = T;
    if (MASK && __builtin_amdgcn_ballot_w64(bits > 1u) != 0ull) {
        // returned terms: all wall links, and again (twice, negated) the
        // fixed-temperature ones
        float sa = 0.0f, sf = 0.0f;
        auto link = [&](auto cxc, auto cyc, auto czc, float lo) {
            constexpr int i = link_index(decltype(cxc)::value, decltype(cyc)::value,
                                         decltype(czc)::value);
            constexpr float w = Lattice<19>::w36(i);
            const unsigned m = (unsigned)((int)(bits << (31 - i)) >> 31);
            const unsigned f = (unsigned)((int)(tw.x << (31 - i)) >> 31);
            const unsigned lb = __builtin_bit_cast(unsigned, lo);
            sa = fmaf(w, __builtin_bit_cast(float, lb & m), sa);
            sf = fmaf(w, __builtin_bit_cast(float, lb & f), sf);
        };
        using P = std::integral_constant<int, 1>;
        using Z = std::integral_constant<int, 0>;
        using M = std::integral_constant<int, -1>;
        link(P{}, Z{}, Z{}, Tmx);
        link(M{}, Z{}, Z{}, Tpx);
        link(Z{}, P{}, Z{}, Tmy);
        link(Z{}, M{}, Z{}, Tpy);
        link(Z{}, Z{}, P{}, Tmz);
        link(Z{}, Z{}, M{}, Tpz);
        link(P{}, P{}, Z{}, Tmm0);
        link(M{}, M{}, Z{}, Tpp0);
        link(P{}, M{}, Z{}, Tmp0);
        link(M{}, P{}, Z{}, Tpm0);
        link(P{}, Z{}, P{}, Tm0m);
        link(M{}, Z{}, M{}, Tp0p);
        link(P{}, Z{}, M{}, Tm0p);
        link(M{}, Z{}, P{}, Tp0m);
        link(Z{}, P{}, P{}, T0mm);
        link(Z{}, M{}, M{}, T0pp);
        link(Z{}, P{}, M{}, T0mp);
        link(Z{}, M{}, P{}, T0pm);
        A0.qd += fmaf(-2.0f, sf, sa) + 2.0f * h * __builtin_bit_cast(float, tw.y);
    }
    // v_z = -1: plane pz - 1
    Am.qe += Tp0m;
    Am.qw += Tm0m;
    Am.qn += T0pm;
    Am.qs += T0mm;
    Am.qd = fmaf(2.0f, Tmz, Am.qd);
}

// the five temperature terms a halo column pushes into the tile (the links of
// push_halo; the same operations as push_temp_column's pairs)
__device__ __forceinline__ void push_temp_halo(float T, float ux, float uy, float uz, float h,
                                               bool isY, float sgn, float &q1, float &q0,
                                               float &qd1, float &qd2, float &qm,
                                               bool solid = false)
{
    const float usq = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
    float AT = h * fmaf(-1.5f, usq, T);
    float H = 4.5f * h, T3 = 3.0f * T;
    if (solid) {  // a solid node pushes nothing
        AT = 0.0f;
        H = 0.0f;
        T3 = 0.0f;
    }
    auto lt = [&](float c) { return fmaf(T3, c, fmaf(H * c, c, AT)); };
    const float ua = isY ? uy : ux;
    const float ub = isY ? ux : uy;
    const float cs = sgn * ua;
    q1 = lt(cs + uz);
    q0 = fmaf(2.0f, lt(cs), q0);
    qd1 = lt(cs + ub);
    qd2 = lt(cs - ub);
    qm += lt(cs - uz);
}

template <int NS>
__device__ __forceinline__ void put_slot_split(const XchgQ<NS> &X, int slot, const Acc &Am)
{
    X.Q[0][slot] = Am.qe;
    X.Q[1][slot] = Am.qw;
    X.Q[2][slot] = Am.qn;
    X.Q[3][slot] = Am.qs;
    X.Q[4][slot] = Am.qne;
    X.Q[5][slot] = Am.qnw;
    X.Q[6][slot] = Am.qse;
    X.Q[7][slot] = Am.qsw;
}

// the arrays put_halo writes for the same links
template <int NS>
__device__ __forceinline__ void put_halo_split(const XchgQ<NS> &X, int slot, bool isY, float sgn,
                                               float q, float qd1, float qd2)
{
    const int hi = sgn > 0.0f ? 0 : 1;
    const int ip = isY ? 2 + hi : hi;
    const int i1 = isY ? 2 * hi : hi;
    const int i2 = isY ? 2 * hi + 1 : hi + 2;
    X.Q[ip][slot] = q;
    X.Q[4 + i1][slot] = qd1;
    X.Q[4 + i2][slot] = qd2;
}

// the q a node receives from its eight in-plane neighbours (gather's slots)
template <int NS, int SXP>
__device__ __forceinline__ float gather_split(const XchgQ<NS> &X, int slot)
{
    const float qE = X.Q[0][slot - 1], qW = X.Q[1][slot + 1];
    const float qN = X.Q[2][slot - SXP], qS = X.Q[3][slot + SXP];
    const float qNE = X.Q[4][slot - SXP - 1], qNW = X.Q[5][slot - SXP + 1];
    const float qSE = X.Q[6][slot + SXP - 1], qSW = X.Q[7][slot + SXP + 1];
    return ((qE + qW) + (qN + qS)) + ((qNE + qNW) + (qSE + qSW));
}

// A halo column pushes only the five links that point into the tile: those
// with v_y = sgn (isY: a row below or above the tile) or v_x = sgn (a column
// left or right of it, corners included).  The terms go into the halo's
// partials of target planes pz + 1 (p1, z1), pz (p0 and the two in-plane
// diagonals d1 = across +1, d2 = across -1) and pz - 1 (pm, zm).  The same
// operations as push_column's pairs, so interior and halo produce bitwise
// the same term for a given link.
template <bool MASK>
__device__ __forceinline__ void push_halo(float dr, float ux, float uy, float uz, int cls,
                                          float A, bool isY, float sgn, float &p1, float &z1,
                                          float &p0, float &d1, float &d2, float &pm, float &zm)
{
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
    const float ua = isY ? uy : ux;  // along the halo direction
    const float ub = isY ? ux : uy;  // across it, in plane
    const float cs = sgn * ua;
    const float Lup = lterm(cs + uz, E0, r45, rA);  // v_z = +1
    const float Lmid = lterm(cs, E0, r45, rA);      // v_z = 0
    const float Ldn = lterm(cs - uz, E0, r45, rA);  // v_z = -1
    p1 = Lup;
    z1 = Lup;
    p0 = fmaf(2.0f, Lmid, p0);
    d1 = lterm(cs + ub, E0, r45, rA);
    d2 = lterm(cs - ub, E0, r45, rA);
    pm += Ldn;
    zm -= Ldn;
}

// A halo column's finished partials of one plane into the slots that its
// inward neighbours read: (PN, ZN) and diagonals NE, NW below the tile,
// (PS, ZS), SE, SW above it; (PE, ZE), NE, SE left of it, (PW, ZW), NW, SW
// right of it.
template <int NS>
__device__ __forceinline__ void put_halo(const Xchg<NS> &X, int slot, bool isY, float sgn, float p,
                                         float z, float d1, float d2)
{
    const int hi = sgn > 0.0f ? 0 : 1;
    const int ip = isY ? 2 + hi : hi;
    const int i1 = isY ? 2 * hi : hi;
    const int i2 = isY ? 2 * hi + 1 : hi + 2;
    X.P[ip][slot] = make_float2(p, z);
    X.Dg[i1][slot] = d1;
    X.Dg[i2][slot] = d2;
}

// Thread roles of the two-step kernels (tile TX x TY, one thread per
// column): threads [0, TX*TY) own the tile; the next two waves the ring of
// columns around it (rows below/above it with the corners, then the columns
// left/right of it); the last two waves the ring at distance two (columns
// left/right with the corners, then the rows below/above).  For that outer
// ring, isY and sgn give the direction of its inward links (a row below the
// tile pushes north: isY, sgn = +1).  Idle lanes have active = false and a
// valid column (0, 0).
struct Col2 {
    int lx, ly;   // tile coordinates, [-2, TX + 1] x [-2, TY + 1]
    float sgn;
    bool isY, active;
};

template <int TX, int TY>
__device__ __forceinline__ Col2 col2_of(int tid)
{
    constexpr int NINT = TX * TY;
    constexpr int RING0 = NINT, HALO0 = NINT + 2 * kWave;
    constexpr int NRING = 2 * (TX + 2) + 2 * TY;
    constexpr int NHALO = 2 * (TX + 2) + 2 * (TY + 4);
    static_assert(NINT % kWave == 0, "tile must be whole waves");
    static_assert(NRING <= 2 * kWave && NHALO <= 2 * kWave, "rings must fit two waves each");
    Col2 c{0, 0, 1.0f, false, true};
    if (tid < NINT) {
        c.lx = tid % TX;
        c.ly = tid / TX;
    } else if (tid < HALO0) {
        const int q = tid - RING0;
        if (q < TX + 2) {  // row below the tile, corners included
            c.lx = q - 1;
            c.ly = -1;
        } else if (q < 2 * (TX + 2)) {  // row above
            c.lx = q - (TX + 2) - 1;
            c.ly = TY;
        } else if (q < 2 * (TX + 2) + TY) {  // column left of the tile
            c.lx = -1;
            c.ly = q - 2 * (TX + 2);
        } else if (q < NRING) {  // column right of it
            c.lx = TX;
            c.ly = q - 2 * (TX + 2) - TY;
        } else {
            c.active = false;
        }
    } else {
        const int q = tid - HALO0;
        if (q < TY + 4) {  // outer left column (corners included), pushing east
            c.lx = -2;
            c.ly = q - 2;
        } else if (q < 2 * (TY + 4)) {  // outer right column, pushing west
            c.lx = TX + 1;
            c.ly = q - (TY + 4) - 2;
            c.sgn = -1.0f;
        } else if (q < 2 * (TY + 4) + TX + 2) {  // outer bottom row, pushing north
            c.isY = true;
            c.lx = q - 2 * (TY + 4) - 1;
            c.ly = -2;
        } else if (q < NHALO) {  // outer top row, pushing south
            c.isY = true;
            c.lx = q - 2 * (TY + 4) - (TX + 2) - 1;
            c.ly = TY + 1;
            c.sgn = -1.0f;
        } else {
            c.active = false;
        }
    }
    return c;
}

// Workgroup -> (tile_x, tile_y, chunk) with an XCD-aware order: consecutive
// workgroups of one XCD get neighbouring tiles.
struct TileIdx {
    int tile_x, tile_y, zc;
};

__device__ __forceinline__ TileIdx tile_of_block(int nx, int ny, int TXv, int TYv)
{
    const unsigned nb = gridDim.x;
    const unsigned b = blockIdx.x;
    const unsigned lb = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + b / 8u : b;
    const int tiles_x = nx / TXv;
    const int tiles_y = ny / TYv;
    TileIdx t;
    t.tile_x = (int)(lb % (unsigned)tiles_x);
    const unsigned rest = lb / (unsigned)tiles_x;
    t.tile_y = (int)(rest % (unsigned)tiles_y);
    t.zc = (int)(rest / (unsigned)tiles_y);
    return t;
}

__device__ __forceinline__ int wrap_index(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

}  // namespace

}  // namespace lwacm
