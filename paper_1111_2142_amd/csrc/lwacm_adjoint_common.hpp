// lwacm_adjoint_common.hpp -- the per-node arithmetic of the D3Q19 reverse
// (adjoint) step, shared by the one-step and the two-step reverse tile
// kernels: state access, moments of the link cotangents and the node's
// cotangent of its own state.
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
#pragma once

#include "lwacm_march_common.hpp"

namespace lwacm {

namespace {

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
template <int DX, int DY, int DZ, int NS>
__device__ __forceinline__ float link_m(const float (*W)[NS], int s)
{
    float m = W[0][s];
    if (DX) m = DX > 0 ? m + W[1][s] : m - W[1][s];
    if (DY) m = DY > 0 ? m + W[2][s] : m - W[2][s];
    if (DZ) m = DZ > 0 ? m + W[3][s] : m - W[3][s];
    return m;
}

// The cotangent of a node's own state, lambda = (dL/d(rho - 1), dL/du), from
// the window planes Wm, W0, Wp of mu around its plane (slot `slot`, row pitch
// SXP) and its state (dr, u); adds the node's dL/da to da.  With MASK, bits
// is its solid-upstream link set (bit 31: a moving wall, whose geometry sums
// are wallg[widx]).
template <bool MASK, int NS, int SXP>
__device__ __forceinline__ f32x4 adj_point(const float (*Wm)[NS], const float (*W0)[NS],
                                           const float (*Wp)[NS], int slot, float dr, float ux,
                                           float uy, float uz, unsigned bits,
                                           const float4 *wallg, long long widx,
                                           const ProblemArgs &p, float &da)
{
    const float A = p.A, a = p.a;
    const float4 own = make_float4(W0[0][slot], W0[1][slot], W0[2][slot], W0[3][slot]);
    // cotangents of the 18 moving links from the neighbours t = y + v_k, in
    // (+v, -v) pairs
    float m[18] = {link_m<1, 0, 0>(W0, slot + 1),         link_m<-1, 0, 0>(W0, slot - 1),
                   link_m<0, 1, 0>(W0, slot + SXP),       link_m<0, -1, 0>(W0, slot - SXP),
                   link_m<0, 0, 1>(Wp, slot),             link_m<0, 0, -1>(Wm, slot),
                   link_m<1, 1, 0>(W0, slot + SXP + 1),   link_m<-1, -1, 0>(W0, slot - SXP - 1),
                   link_m<1, -1, 0>(W0, slot - SXP + 1),  link_m<-1, 1, 0>(W0, slot + SXP - 1),
                   link_m<1, 0, 1>(Wp, slot + 1),         link_m<-1, 0, -1>(Wm, slot - 1),
                   link_m<1, 0, -1>(Wm, slot + 1),        link_m<-1, 0, 1>(Wp, slot - 1),
                   link_m<0, 1, 1>(Wp, slot + SXP),       link_m<0, -1, -1>(Wm, slot - SXP),
                   link_m<0, 1, -1>(Wm, slot + SXP),      link_m<0, -1, 1>(Wp, slot - SXP)};
    if (MASK && bits != 0u) {
        // a solid t = y + v_k: the term bounced back into y along -v_k,
        // m_k = mu_R(y) - v_k . mu_J(y).  The forward bit set marks solid
        // upstream nodes y - v_i, i.e. link k = opposite(i).
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
    // The moments carry the integer weights 36 w_k.  Every use below is
    // linear in them, so the factor 1/36 is taken out once per result
    // (div36: correctly rounded, no bias) instead of once per moment.
    const float m0 = M.m0, m1x = M.m1x, m1y = M.m1y, m1z = M.m1z;
    const float xx = M.xx, yy = M.yy, zz = M.zz, xy = M.xy, xz = M.xz, yz = M.yz;

    const float rho = 1.0f + dr;
    const float B = -1.5f * fmaf(ux, ux, fmaf(uy, uy, uz * uz));
    const float uM1 = div36(fmaf(ux, m1x, fmaf(uy, m1y, uz * m1z)));
    const float M2ux = fmaf(xx, ux, fmaf(xy, uy, xz * uz));
    const float M2uy = fmaf(xy, ux, fmaf(yy, uy, yz * uz));
    const float M2uz = fmaf(xz, ux, fmaf(yz, uy, zz * uz));
    const float uM2u = fmaf(ux, M2ux, fmaf(uy, M2uy, uz * M2uz));
    const float mJu = fmaf(own.y, ux, fmaf(own.z, uy, own.w * uz));
    float lr = fmaf(div36(m0), 1.0f + B, fmaf(A, uM1, div36(4.5f * uM2u)));
    lr = fmaf(own.y, fmaf(a, ux, p.g[0]), lr);
    lr = fmaf(own.z, fmaf(a, uy, p.g[1]), lr);
    lr = fmaf(own.w, fmaf(a, uz, p.g[2]), lr);
    const float arho = a * rho;
    const float lux = fmaf(rho, div36(fmaf(A, m1x, fmaf(9.0f, M2ux, -3.0f * ux * m0))), arho * own.y);
    const float luy = fmaf(rho, div36(fmaf(A, m1y, fmaf(9.0f, M2uy, -3.0f * uy * m0))), arho * own.z);
    const float luz = fmaf(rho, div36(fmaf(A, m1z, fmaf(9.0f, M2uz, -3.0f * uz * m0))), arho * own.w);
    da = fmaf(rho, fmaf(-3.0f, uM1, mJu), da);
    if (MASK && (bits & kMovingWallFlag)) {
        // moving walls: sum over bounced links of w_k (v_k . 6 rho0 u_w) m_k
        const float4 g = wallg[widx];
        const float gw = -fmaf(own.x, g.x, fmaf(own.y, g.y, fmaf(own.z, g.z, own.w * g.w)));
        da = fmaf(p.wall6rho0, div36(gw), da);
    }
    const f32x4 lam = {lr, lux, luy, luz};
    return lam;
}

// mu of the step before from lambda: the normalisation u = J / rho of that
// step folded in, (lambda_rho - lambda_u . u / rho, lambda_u / rho).  1/rho
// is the hardware reciprocal (1 ulp), not a correctly rounded division.
__device__ __forceinline__ f32x4 fold_normalisation(const f32x4 &lam, float dr, float ux,
                                                    float uy, float uz)
{
    const float inv = __builtin_amdgcn_rcpf(1.0f + dr);
    const float lu_u = fmaf(lam.y, ux, fmaf(lam.z, uy, lam.w * uz));
    const f32x4 mu = {lam.x - lu_u * inv, lam.y * inv, lam.z * inv, lam.w * inv};
    return mu;
}

}  // namespace

}  // namespace lwacm
