// lwacm_device.hpp -- device-side building blocks of the LW-ACM kernels:
// lattice tables, the per-link term of the update, storage conversion and a
// deterministic FP64 grid reduction.  gfx950 only (wave64).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lwacm {

constexpr int kWave = 64;
// Threads that add the per-block partials in the second pass of a grid
// reduction (one stride, then the block's fixed tree).
constexpr unsigned kReduceThreads = 256;

// ---------------------------------------------------------------- lattices
// Link velocities grouped by their z component (Appendix A lists the groups
// rest / axis / diagonal; the order inside is free).  The nine links with
// v_z = 0 come first and are exactly the D2Q9 set, so both lattices share
// indices 0..8:
//   0 rest, 1 (+x), 2 (-x), 3 (+y), 4 (-y), 5 (+x+y), 6 (-x-y), 7 (+x-y), 8 (-x+y),
//   9 (+z), 10 (+x+z), 11 (-x+z), 12 (+y+z), 13 (-y+z),
//   14 (-z), 15 (-x-z), 16 (+x-z), 17 (-y-z), 18 (+y-z).
// Links 14..18 are the opposites of 9..13 in the same order; 1..8 pair up
// as (1,2), (3,4), (5,6), (7,8).
__host__ __device__ constexpr int link_cx(int i)
{
    constexpr int t[19] = {0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 1, -1, 0, 0, 0, -1, 1, 0, 0};
    return t[i];
}
__host__ __device__ constexpr int link_cy(int i)
{
    constexpr int t[19] = {0, 0, 0, 1, -1, 1, -1, -1, 1, 0, 0, 0, 1, -1, 0, 0, 0, -1, 1};
    return t[i];
}
__host__ __device__ constexpr int link_cz(int i)
{
    constexpr int t[19] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1};
    return t[i];
}
__host__ __device__ constexpr int link_opp(int i)
{
    constexpr int t[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 14, 15, 16, 17, 18, 9, 10, 11, 12, 13};
    return t[i];
}

// Index of the D3Q19 link with velocity (cx, cy, cz), -1 if none.
__host__ __device__ constexpr int link_index(int cx, int cy, int cz)
{
    for (int i = 0; i < 19; ++i)
        if (link_cx(i) == cx && link_cy(i) == cy && link_cz(i) == cz) return i;
    return -1;
}

template <int Q>
struct Lattice;

// Weights are carried as the exact integers 36 w_i, and sums are divided by
// 36 once with div36().  FP32 constants such as 1/9 or 1/36 are rounded up
// by ~1e-8, which would scale every step's momentum by (1 + 1e-8) and grow
// a systematic error of ~1e-5 over 1000 steps.

// D2Q9: w = 4/9, 1/9 (axis), 1/36 (diagonal), Eq. weight_factors.
template <>
struct Lattice<9> {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    __host__ __device__ static constexpr float w36(int i)
    {
        return i == 0 ? 16.0f : (i <= 4 ? 4.0f : 1.0f);
    }
};

// D3Q19: w = 1/3, 1/18 (axis), 1/36 (face diagonal), Eq. weight_factors_3d.
template <>
struct Lattice<19> {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    __host__ __device__ static constexpr float w36(int i)
    {
        return i == 0 ? 12.0f : ((i <= 4 || i == 9 || i == 14) ? 2.0f : 1.0f);
    }
};

// x / 36 with a double-word constant: the result is the nearest float in
// all but rare ties, and, unlike x * fl(1/36), carries no systematic bias.
__device__ __forceinline__ float div36(float x)
{
    constexpr float c_hi = 1.0f / 36.0f;
    constexpr float c_lo = (float)(1.0 / 36.0 - (double)(1.0f / 36.0f));
    return fmaf(x, c_hi, x * c_lo);
}

// ------------------------------------------------------ the link term
// Pre-combined population of Eq. ACM2.0b (pre-combining step), in deviation
// form: f*_i - w_i = w_i [drho + rho (c (A + 9/2 c) - 3/2 |u|^2)] with
// c = v_i . u and A = 3 (2/omega - 1) = 3 (1 - a).  It follows from the
// equilibrium of Appendix A and the odd part f^(e,o)_i = 3 w_i rho c.
// The caller passes B = -3/2 |u|^2 and v_i . u.
__device__ __forceinline__ float link_term_unweighted(float drho, float rho, float c, float B,
                                                      float A)
{
    float t = fmaf(4.5f, c, A);
    t = fmaf(c, t, B);
    return fmaf(rho, t, drho);
}

// New velocity u = J / (1 + D) with D = rho - 1 of the updated node, written
// as u = J - J * q with q = D / (1 + D).  Forming 1 + D in FP32 loses the low
// bits of D; in this form that loss only scales the O(D) correction, so the
// per-step error stays at one rounding of u.  The reciprocal is the hardware
// approximation (1 ulp), which is ample for the correction term.
__device__ __forceinline__ float normalisation_factor(float D)
{
    return D * __builtin_amdgcn_rcpf(1.0f + D);
}

// ------------------------------------------- stochastic FP16 rounding
// Counter-based random bits: the pcg2d hash of Jarzynski and Olano, "Hash
// Functions for GPU Rendering", JCGT 9(3), 2020: an LCG step on each of two
// words, then two rounds of "each word adds the other times the LCG
// multiplier" and an xor-shift by 16 (six 32-bit multiplies).  A bijection of
// its 64-bit input, so the counter (node index, t ^ seed) gives every node of
// every step its own pair (a, b).  Field f of the node's stored state is
// rounded with the top 13 bits of word f of (a, b, a << 13, b << 13):
// disjoint bits of the pair, and a recomputed step draws the same bits.
struct U32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U32x4 sr_words(uint32_t idx, uint32_t step_word)
{
    uint32_t a = idx * 1664525u + 1013904223u;
    uint32_t b = step_word * 1664525u + 1013904223u;
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        a += b * 1664525u;
        b += a * 1664525u;
        a ^= a >> 16;
        b ^= b >> 16;
    }
    return U32x4{a, b, a << 13, b << 13};
}

// FP32 -> FP16 with stochastic rounding, two values into one packed word
// (lo in bits 0..15, hi in 16..31): gfx950's v_cvt_sr_f16_f32.  |y| lies
// between two adjacent FP16 magnitudes and goes to the upper one when
// F + (r >> 19) >= 2^13, F the first 13 bits of its position between them
// (in the normal range all of it: FP32 keeps 13 bits below the FP16 spacing).
// The expected stored value is y to 2^-13 of a spacing, so updates smaller
// than one FP16 spacing are not lost; round to nearest would drop them.
// Magnitudes past 65504 that round up become infinite.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t half2_bits_sr(float lo, uint32_t rlo, float hi, uint32_t rhi)
{
    half2_t v = {(_Float16)0.0f, (_Float16)0.0f};
    v = __builtin_amdgcn_cvt_sr_f16_f32(v, lo, rlo, false);
    v = __builtin_amdgcn_cvt_sr_f16_f32(v, hi, rhi, true);
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ unsigned short half_bits_sr(float y, uint32_t r)
{
    return (unsigned short)(half2_bits_sr(y, r, 0.0f, 0u) & 0xffffu);
}

// Wait states after a buffer store whose offset comes from an SGPR.  This
// compiler assumes such a store needs none before its data registers are
// rewritten; on gfx950 the trailing lanes of a wide store then pick up the
// next instruction's results (observed as corrupted nodes in the last plane
// of a tile kernel's chunk).  Two wait states, fenced by scheduling barriers
// so that nothing moves between the store and the nops.
__device__ __forceinline__ void store_data_guard()
{
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 1");
    __builtin_amdgcn_sched_barrier(0);
}

// ------------------------------------------------------- storage formats
// The state is node-interleaved: node idx holds its NF = D + 1 values
// (rho - 1, u_x, u_y[, u_z]) at elements NF * idx .. NF * idx + NF - 1, so a
// D3Q19 node is one 16-byte (FP32) or 8-byte (FP16) access.  FP16 storage
// holds half(value * 2^k) with k_rho for field 0 and k_u for the velocity;
// the scale arguments are 2^-k on load and 2^k on store (exact in FP32).
// store() rounds to nearest even (initial states); store_sr() rounds
// stochastically with one random word per field (step outputs).
template <class T, int NF>
struct NodeState;

template <int NF>
struct NodeState<float, NF> {
    __device__ __forceinline__ static void load(const float *s, long long idx, const float (&)[2],
                                                float (&v)[NF])
    {
        if constexpr (NF == 4) {
            const float4 q = reinterpret_cast<const float4 *>(s)[idx];
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) v[f] = s[NF * idx + f];
        }
    }
    __device__ __forceinline__ static void store(float *s, long long idx, const float (&v)[NF],
                                                 const float (&)[2])
    {
        if constexpr (NF == 4) {
            reinterpret_cast<float4 *>(s)[idx] = make_float4(v[0], v[1], v[2], v[3]);
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) s[NF * idx + f] = v[f];
        }
    }
    __device__ __forceinline__ static void store_sr(float *s, long long idx, const float (&v)[NF],
                                                    const float (&sc)[2], const U32x4 &)
    {
        store(s, idx, v, sc);
    }
};

template <int NF>
struct NodeState<__half, NF> {
    __device__ __forceinline__ static float unpack(uint32_t w, int hi, float scale)
    {
        return __half2float(__ushort_as_half((unsigned short)(hi ? w >> 16 : w & 0xffffu))) * scale;
    }
    __device__ __forceinline__ static void load(const __half *s, long long idx,
                                                const float (&ld)[2], float (&v)[NF])
    {
        if constexpr (NF == 4) {
            const uint2 q = reinterpret_cast<const uint2 *>(s)[idx];
            v[0] = unpack(q.x, 0, ld[0]);
            v[1] = unpack(q.x, 1, ld[1]);
            v[2] = unpack(q.y, 0, ld[1]);
            v[3] = unpack(q.y, 1, ld[1]);
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) v[f] = __half2float(s[NF * idx + f]) * ld[f > 0];
        }
    }
    // bits[f]: FP16 bit pattern of field f
    __device__ __forceinline__ static void put(__half *s, long long idx,
                                               const unsigned short (&bits)[NF])
    {
        if constexpr (NF == 4) {
            reinterpret_cast<uint2 *>(s)[idx] =
                make_uint2((uint32_t)bits[0] | ((uint32_t)bits[1] << 16),
                           (uint32_t)bits[2] | ((uint32_t)bits[3] << 16));
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) s[NF * idx + f] = __ushort_as_half(bits[f]);
        }
    }
    __device__ __forceinline__ static void store(__half *s, long long idx, const float (&v)[NF],
                                                 const float (&st)[2])
    {
        unsigned short b[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) b[f] = __half_as_ushort(__float2half_rn(v[f] * st[f > 0]));
        put(s, idx, b);
    }
    __device__ __forceinline__ static void store_sr(__half *s, long long idx, const float (&v)[NF],
                                                    const float (&st)[2], const U32x4 &r)
    {
        if constexpr (NF == 4) {
            reinterpret_cast<uint2 *>(s)[idx] =
                make_uint2(half2_bits_sr(v[0] * st[0], r.x, v[1] * st[1], r.y),
                           half2_bits_sr(v[2] * st[1], r.z, v[3] * st[1], r.w));
        } else {
            const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
            unsigned short b[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) b[f] = half_bits_sr(v[f] * st[f > 0], rw[f]);
            put(s, idx, b);
        }
    }
};

// --------------------------------------------- deterministic reductions
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    return v;
}

// Sum NV doubles over the block into thread 0 with a fixed tree.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double sh[NV][16];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sh[k][w];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Deterministic grid-wide sums, first pass: each block stores the fixed-tree
// sum of its NV doubles in partials[NV * bid + k]; a second, one-block kernel
// (k_reduce_partials) adds the partials in a fixed order.  The kernel
// boundary makes the partials visible, so no device-scope fences are needed:
// on this chip such a fence writes back and invalidates the whole L2 of an
// XCD, once per block.
// Second pass of the previous step's (mass, energy) sums, run by block 0 of
// the next forward launch: the same fixed order as k_reduce_partials.
__device__ __forceinline__ void finish_previous_sums(const double *prev, unsigned nblocks,
                                                     double *out, double *out2)
{
    double acc[2] = {0.0, 0.0};
    if (threadIdx.x < kReduceThreads)
        for (unsigned b = threadIdx.x; b < nblocks; b += kReduceThreads) {
            acc[0] += prev[2 * (size_t)b];
            acc[1] += prev[2 * (size_t)b + 1];
        }
    block_sum<2>(acc);  // further waves add exact zeros
    if (threadIdx.x == 0) {
        out[0] = acc[0];
        out[1] = acc[1];
        if (out2) {
            out2[0] = acc[0];
            out2[1] = acc[1];
        }
    }
}

template <int NV>
__device__ __forceinline__ void store_block_partials(double (&v)[NV], double *partials, unsigned bid)
{
    block_sum<NV>(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) partials[(size_t)NV * bid + k] = v[k];
}

}  // namespace lwacm
