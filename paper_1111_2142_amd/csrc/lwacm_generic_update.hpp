// lwacm_generic_update.hpp -- the update of one node by the generic kernels
// (one step per launch, lwacm_generic.hip) and by the multi-step D2Q9 kernel
// (lwacm_d2q9_multi.hip): one function, so both round every operation alike.
#pragma once

#include "lwacm_device.hpp"
#include "lwacm_internal.hpp"

namespace lwacm {

namespace {

template <int Q>
__device__ __forceinline__ float vdot(int i, const float (&u)[3])
{
    // the sum starts from the first nonzero component (not from 0 + ..., which
    // the compiler may not drop); a rest link gives the constant 0
    float c = 0.0f;
    bool set = false;
    if (link_cx(i) != 0) {
        c = (link_cx(i) > 0) ? u[0] : -u[0];
        set = true;
    }
    if (link_cy(i) != 0) {
        const float t = (link_cy(i) > 0) ? u[1] : -u[1];
        c = set ? c + t : t;
        set = true;
    }
    if (Q == 19 && link_cz(i) != 0) {
        const float t = (link_cz(i) > 0) ? u[2] : -u[2];
        c = set ? c + t : t;
    }
    return c;
}

// B = -3/2 |u|^2 of a node, the velocity part of every link term's
// equilibrium (Eq. ACM2.0); one expression for every caller, so that a value
// computed once and stored equals the one computed where it is used
__device__ __forceinline__ float node_B(const float (&u)[3])
{
    return -1.5f * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

// accumulate into acc, or start it with the first term
__device__ __forceinline__ void accum(float &acc, bool &set, float t)
{
    acc = set ? acc + t : t;
    set = true;
}

// The update of one fluid node x (Eq. ACM2.0 in pull form with the wall,
// forcing and omega_p rules below), given its state (drx, ux, Bx = node_B(ux))
// and two accessors of the nodes x + (dx, dy, dz): fmask(dx, dy, dz) returns
// the mask value, fstate(dx, dy, dz, dr, u, B) the state and its node_B.  Writes the new (rho - 1, u) to
// out and |u|^2 to e.  Shared by the one-step kernel (accessors read global
// memory) and the multi-step D2Q9 kernel (accessors read its LDS tile), so
// both round every operation alike.
//
// SPLIT: a separate relaxation omega_p for the density (Section
// "finite-difference formulation", item 3; Appendix E).  The density sums the
// same link terms with Ap = 3 (2/omega_p - 1) in place of A (and the moving
// wall's omega_p term); the momentum keeps A.
template <int Q, bool MASK, bool FORCE, bool SPLIT, class FMask, class FState>
__device__ __forceinline__ void link_update(const ProblemArgs &p, long long idx, float drx,
                                            const float (&ux)[3], float Bx, const FMask &fmask,
                                            const FState &fstate,
                                            float (&out)[Lattice<Q>::D + 1], float &e)
{
    using L = Lattice<Q>;
    constexpr int D = L::D;
    const long long n = p.n;
    const float rx = 1.0f + drx;
    // Forcing (Eq. force) adds the odd part 3 w_i rho_x (v_i . g) to every
    // population.  It enters each link term through the addend of its FMA,
    // where it meets an exact, node-dependent product; added to the final
    // sum instead, the same small constant would round the same way every
    // step and bias long runs.
    float g3[3] = {0.0f, 0.0f, 0.0f};
    if (FORCE)
#pragma unroll
        for (int k = 0; k < D; ++k)
            g3[k] = 3.0f * rx * (p.g_field ? p.g_field[(long long)k * n + idx] : p.g[k]);
    float D36 = 0.0f, J36[3] = {0.0f, 0.0f, 0.0f};
    bool dset = false, jset[3] = {false, false, false};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // the forcing term of the link's addend (absent without a force)
        const float fg = FORCE ? vdot<Q>(i, g3) : 0.0f;
        auto addf = [&](float d) { return FORCE ? d + fg : d; };
        const bool rest = link_cx(i) == 0 && link_cy(i) == 0 && link_cz(i) == 0;
        float s, sp = 0.0f;  // link term; with SPLIT, its density form
        uint8_t m = 0;
        if (MASK && !rest) m = fmask(-link_cx(i), -link_cy(i), -link_cz(i));
        if (rest) {
            // the node's own term: with c = 0 the link term is rho B + (rho - 1)
            s = fmaf(rx, Bx, addf(drx));
            if (SPLIT) sp = s;
        } else if (MASK && m != 0) {
            // bounce-back: own term of the opposite link + moving wall
            const int ib = link_opp(i);
            float uw[3] = {p.wall_term[m][0], p.wall_term[m][1], p.wall_term[m][2]};
            if (p.uwl) {
                // the wall's velocity where the link x -> x + v_ib crosses it
#pragma unroll
                for (int k = 0; k < D; ++k)
                    uw[k] = p.wall_scale * p.uwl[((long long)ib * D + k) * n + idx];
            }
            const float cb = vdot<Q>(ib, ux);
            float sb = link_term_unweighted(addf(drx), rx, cb, Bx, p.A);
            float wsc = 1.0f;  // scale of the halfway moving-wall term
            if (p.qd) {
                // interpolated bounce-back (Eq. ACM2.0cc): the wall cuts the
                // link x -> x + v_ib at the fraction q; the terms are in
                // deviation form, whose mixing weights sum to one
                const float qv = p.qd[(long long)ib * n + idx];
                if (qv < 0.5f) {
                    if (fmask(link_cx(i), link_cy(i), link_cz(i)) == 0) {  // x - v_ib fluid
                        float drz, uz[3], Bz;
                        fstate(link_cx(i), link_cy(i), link_cz(i), drz, uz, Bz);
                        const float sz = link_term_unweighted(addf(drz), 1.0f + drz,
                                                              vdot<Q>(ib, uz), Bz, p.A);
                        sb = fmaf(2.0f * qv, sb, (1.0f - 2.0f * qv) * sz);
                    }
                } else {
                    const float si = link_term_unweighted(addf(drx), rx, vdot<Q>(i, ux), Bx, p.A);
                    const float h = 0.5f / qv;  // 1 / (2q)
                    sb = fmaf(h, sb, (1.0f - h) * si);
                    wsc = h;  // Eq. ACM2.0move: 1/q in place of 2
                }
            }
            s = fmaf(wsc, vdot<Q>(i, uw), sb);
            if (SPLIT) {
                const float uwp[3] = {p.wall_term_p[m][0], p.wall_term_p[m][1],
                                      p.wall_term_p[m][2]};
                sp = link_term_unweighted(addf(drx), rx, cb, Bx, p.Ap) + vdot<Q>(i, uwp);
            }
        } else {
            float dry, uy[3], By;
            fstate(-link_cx(i), -link_cy(i), -link_cz(i), dry, uy, By);
            const float cy = vdot<Q>(i, uy);
            s = link_term_unweighted(addf(dry), 1.0f + dry, cy, By, p.A);
            if (SPLIT) sp = link_term_unweighted(addf(dry), 1.0f + dry, cy, By, p.Ap);
        }
        s *= L::w36(i);
        accum(D36, dset, SPLIT ? sp * L::w36(i) : s);
        if (link_cx(i) != 0) accum(J36[0], jset[0], link_cx(i) > 0 ? s : -s);
        if (link_cy(i) != 0) accum(J36[1], jset[1], link_cy(i) > 0 ? s : -s);
        if (link_cz(i) != 0) accum(J36[2], jset[2], link_cz(i) > 0 ? s : -s);
    }
    const float Dsum = div36(D36);
    // post-combine: sum_i v_i a f^(e,o)_i(x) = a rho_x u_x
    float J[3];
#pragma unroll
    for (int k = 0; k < D; ++k) J[k] = fmaf(p.a * rx, ux[k], div36(J36[k]));
    // u = J / (1 + D) evaluated as J - J * (D / (1 + D)): the rounding of
    // 1 + D then only touches the small correction term, which keeps the
    // FP32 error from accumulating over long runs.
    const float q = normalisation_factor(Dsum);
    e = 0.0f;
    out[0] = Dsum;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        out[k + 1] = fmaf(-J[k], q, J[k]);
        e = fmaf(out[k + 1], out[k + 1], e);
    }
}

// The reverse step at one fluid node y (the exact derivative of link_update,
// in the gather form of its transpose): given y's state (dry, uy), its own
// mu_t (muR_y, muJ_y) and two accessors of the nodes y + (dx, dy, dz) --
// fmask returns the mask value, fmu(dx, dy, dz, mr, mt) their mu_t -- the
// cotangents of y's state lambda_t = (lr, lu) and y's share da of dL/da.
// Shared by the one-step reverse kernel (accessors read global memory) and
// the multi-step D2Q9 reverse kernel (accessors read its LDS tile), so both
// round every operation alike.
template <int Q, bool MASK, class FMask, class FMu>
__device__ __forceinline__ void adj_node_update(const ProblemArgs &p, float dry,
                                                const float (&uy)[3], float muR_y,
                                                const float (&muJ_y)[3], const FMask &fmask,
                                                const FMu &fmu, float &lr, float (&lu)[3],
                                                float &da)
{
    using L = Lattice<Q>;
    constexpr int D = L::D;
    const float ry = 1.0f + dry;
    const float By = -1.5f * (uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2]);
    lr = 0.0f;
    lu[0] = lu[1] = lu[2] = 0.0f;
    da = 0.0f;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        float m;
        uint8_t wm = 0;
        if (MASK) wm = fmask(link_cx(k), link_cy(k), link_cz(k));
        if (MASK && wm != 0) {
            // the term bounces back into y itself along -v_k
            m = muR_y - vdot<Q>(k, muJ_y);
            const float wd[3] = {p.wall_da[wm][0], p.wall_da[wm][1], p.wall_da[wm][2]};
            da = fmaf(L::w36(k) * (1.0f / 36.0f) * vdot<Q>(k, wd), m, da);
        } else {
            float mr, mt[3];
            fmu(link_cx(k), link_cy(k), link_cz(k), mr, mt);
            m = mr + vdot<Q>(k, mt);
        }
        const float cc = vdot<Q>(k, uy);
        const float wm_ = L::w36(k) * (1.0f / 36.0f) * m;
        // d s_k / d(rho-1) = w_k [1 + c (A + 9/2 c) - 3/2 |u|^2]
        lr = fmaf(wm_, 1.0f + cc * fmaf(4.5f, cc, p.A) + By, lr);
        // d s_k / d u = w_k rho [(A + 9 c) v_k - 3 u]
        const float q = wm_ * ry * fmaf(9.0f, cc, p.A);
        if (link_cx(k) != 0) lu[0] += link_cx(k) * q;
        if (link_cy(k) != 0) lu[1] += link_cy(k) * q;
        if (link_cz(k) != 0) lu[2] += link_cz(k) * q;
#pragma unroll
        for (int j = 0; j < D; ++j) lu[j] = fmaf(-3.0f * wm_ * ry, uy[j], lu[j]);
        // d s_k / d a = -3 w_k rho c
        da = fmaf(-3.0f * wm_ * ry, cc, da);
    }
    // post-combine a rho u and forcing rho g of the node's own momentum
    float mJu = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lr = fmaf(muJ_y[j], fmaf(p.a, uy[j], p.g[j]), lr);
        lu[j] = fmaf(p.a * ry, muJ_y[j], lu[j]);
        mJu = fmaf(muJ_y[j], uy[j], mJu);
    }
    da = fmaf(ry, mJu, da);
}

// mu_{t-1} of the node from its lambda_t: the normalisation u = J / rho of
// the previous step folded in
template <int D>
__device__ __forceinline__ void adj_fold(float dry, const float (&uy)[3], float lr,
                                         const float (&lu)[3], float &muR, float (&muJ)[3])
{
    const float inv = 1.0f / (1.0f + dry);
    float lu_u = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) lu_u = fmaf(lu[j], uy[j], lu_u);
    muJ[0] = muJ[1] = muJ[2] = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) muJ[j] = lu[j] * inv;
    muR = lr - lu_u * inv;
}

}  // namespace

}  // namespace lwacm
