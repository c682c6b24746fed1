// lwacm_adjoint_march2.hip -- two D3Q19 reverse (adjoint) steps per pass.
//
// The one-step reverse tile kernel moves 48 bytes per node and step (state,
// mu in, mu out) and runs near the HBM bound.  This kernel takes mu_t, the
// state of step t and the state of step t - 1, computes mu_{t-1} on the tile
// grown by one column on every side, keeps it on chip, and computes mu_{t-2}
// (or, on the last step of the sweep, the gradient with respect to the
// initial state) on the tile: 32 bytes per node and step.
//
// Layout (the roles and chunks of the two-step forward kernel): tile
// 32 x 16 columns, 768 threads, a chunk of NZC planes.  Every thread loads
// mu_t of its column (tile, ring, outer ring) into a window of three LDS
// planes (36 x 20 slots); tile and ring threads then compute mu_{t-1} of the
// plane below from that window and their step-t state, into a second window
// (34 x 18 slots); tile threads compute the step-(t - 1) result of the plane
// below that from the second window and their step-(t - 1) state.  Two
// barriers per plane, so three window planes suffice: a plane is rewritten
// only after every thread has passed the barrier that follows its last read.
// Every node is computed by the same function as in the one-step kernel
// (adj_point), so the result is bitwise that of two one-step launches, and so
// are the per-block dL/da partials where both kernels split the planes among
// workgroups alike.
#include "lwacm_adjoint_common.hpp"

namespace lwacm {

namespace {

constexpr int TX = 32;
constexpr int TY = 16;
constexpr int RING = 3;                              // planes of loads in flight per thread
constexpr int NINT = TX * TY;                        // tile columns: waves 0-7
constexpr int HALO0 = NINT + 2 * kWave;              // first thread of the outer ring
constexpr int NTHREADS = NINT + 4 * kWave;
constexpr int SX1 = TX + 4, NS1 = SX1 * (TY + 4);    // mu_t window slots
constexpr int SX2 = TX + 2, NS2 = SX2 * (TY + 2);    // mu_{t-1} window slots
// Chunk depth: 128 planes, halved while deeper than nz.  At 256^3 that is one
// workgroup per compute unit in a single round (the kernel's 136 VGPRs allow
// one 768-thread workgroup per CU); 64-plane chunks, the one-step reverse
// kernel's depth, take two rounds and measured 2.5 % slower.  Where the depths
// differ, the dL/da block partials group the planes differently from the
// one-step kernel's (equal to FP64 rounding of the per-thread partials).
constexpr int kAdjChunk = 128;
int adj2_nzc(const ProblemArgs &p)
{
    int c = kAdjChunk;
    while (c > 8 && c > p.nz) c /= 2;
    return c <= p.nz ? c : 0;
}

template <class T, bool FINAL, int NZC>
__global__ __launch_bounds__(NTHREADS) void k_adj_march2(ProblemArgs p,
                                                         const T *__restrict__ state_a,
                                                         const T *__restrict__ state_b,
                                                         const float *__restrict__ mu_in,
                                                         float *__restrict__ mu_out, ReduceArgs r)
{
    // one spare slot per array: idle lanes write there instead of branching
    __shared__ float w1[3][4][NS1 + 1];
    __shared__ float w2[3][4][NS2 + 1];

    const int tid = threadIdx.x;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long n = p.n;
    const long long plane = (long long)nx * ny;

    const TileIdx ti = tile_of_block(nx, ny, TX, TY);
    // full chunks: a ragged last one is moved down to end at nz; its planes
    // below zs are written twice with the same bits and counted once
    const int zs = ti.zc * NZC;
    const int z0 = min(zs, nz - NZC);
    const int z1 = z0 + NZC;

    const Col2 c2 = col2_of<TX, TY>(tid);
    const int gx = wrap_index(ti.tile_x * TX + c2.lx, nx);
    const int gy = wrap_index(ti.tile_y * TY + c2.ly, ny);
    const unsigned col = (unsigned)(gy * nx + gx);
    const int slot1 = (c2.ly + 2) * SX1 + (c2.lx + 2);
    const int slot2 = (c2.ly + 1) * SX2 + (c2.lx + 1);  // tile and first ring only
    const int wslot1 = c2.active ? slot1 : NS1;
    const int wslot2 = c2.active ? slot2 : NS2;

    auto wrapz = [&](int pz) { return wrap_index(pz, nz); };
    constexpr unsigned NB = StateIO<T>::kNodeBytes;
    const Rsrc rmu = make_rsrc(mu_in, (unsigned long long)n * 16u);
    const Rsrc rsa = make_rsrc(state_a, (unsigned long long)n * NB);
    const Rsrc rsb = make_rsrc(state_b, (unsigned long long)n * NB);
    const Rsrc rout = make_rsrc(mu_out, (unsigned long long)n * 16u);
    const unsigned mu_plane = (unsigned)(plane * 16);
    const unsigned st_plane = (unsigned)(plane * NB);
    const unsigned voff_mu = col * 16u;
    const unsigned voff_st = col * NB;

    // Load rings, indexed by k % 3 at compile time: mu_t of plane pz is in
    // mr[k % 3] at iteration k; the step-t state of plane pz - 1 (first stage)
    // in sa[(k + 2) % 3]; the step-(t - 1) state of plane pz - 2 (second
    // stage) in sb[(k + 1) % 3].  Each slot is refilled after its last use
    // (so the load takes the same registers and the loop needs no copies),
    // for the plane three iterations ahead.
    using Raw = typename StateIO<T>::Raw;
    f32x4 mr[RING];
    Raw sa[RING], sb[RING];
#pragma unroll
    for (int j = 0; j < RING; ++j) mr[j] = load_f4(rmu, voff_mu, (unsigned)wrapz(z0 - 2 + j) * mu_plane);
    if (tid < HALO0) {
        sa[1] = StateIO<T>::load(rsa, voff_st, (unsigned)wrapz(z0 - 1) * st_plane);
        sa[2] = StateIO<T>::load(rsa, voff_st, (unsigned)z0 * st_plane);
        sa[0] = StateIO<T>::load(rsa, voff_st, (unsigned)(z0 + 1) * st_plane);
    }
    if (tid < NINT) {
        sb[2] = StateIO<T>::load(rsb, voff_st, (unsigned)z0 * st_plane);
        sb[0] = StateIO<T>::load(rsb, voff_st, (unsigned)(z0 + 1) * st_plane);
        sb[1] = StateIO<T>::load(rsb, voff_st, (unsigned)(z0 + 2) * st_plane);
    }

    float da_a = 0.0f, da_b = 0.0f;  // dL/da of the two steps (tile threads)
    constexpr int N = NZC + 4;        // planes z0 - 2 .. z1 + 1 of mu_t

    // mu_t of plane pz into the first window (every thread).
    auto enter = [&](int k, auto It) {
        using I = decltype(It);
        __builtin_amdgcn_sched_barrier(0);
        const f32x4 q = mr[I::j];
        w1[I::j][0][wslot1] = q.x;
        w1[I::j][1][wslot1] = q.y;
        w1[I::j][2][wslot1] = q.z;
        w1[I::j][3][wslot1] = q.w;
        __builtin_amdgcn_sched_barrier(0);
        if (I::refill) mr[I::j] = load_f4(rmu, voff_mu, (unsigned)wrapz(z0 + 1 + k) * mu_plane);
    };
    // Step t at plane tq = pz - 1 (z0 - 1 .. z1): mu_{t-1} into the second
    // window (tile and ring threads).
    auto stage_a = [&](int k, auto It, bool tile) {
        using I = decltype(It);
        constexpr int j = I::j, j1 = (j + 1) % 3, jm = (j + 2) % 3;
        float d, ux, uy, uz;
        StateIO<T>::unpack(sa[jm], p.ld_scale, d, ux, uy, uz);
        const int tq = z0 - 3 + k;
        float da = da_a;
        const f32x4 lam = adj_point<false, NS1 + 1, SX1>(w1[j1], w1[jm], w1[j], slot1, d, ux, uy,
                                                         uz, 0u, nullptr, 0, p, da);
        if (tile) da_a = (tq >= zs && tq < z1) ? da : da_a;
        const f32x4 mu = fold_normalisation(lam, d, ux, uy, uz);
        w2[j][0][wslot2] = mu.x;
        w2[j][1][wslot2] = mu.y;
        w2[j][2][wslot2] = mu.z;
        w2[j][3][wslot2] = mu.w;
        __builtin_amdgcn_sched_barrier(0);  // the state's last use is above
        if (I::refill) sa[jm] = StateIO<T>::load(rsa, voff_st, (unsigned)wrapz(z0 + k) * st_plane);
    };

    if (tid < NINT) {
        plane_loop<N>([&](int k, auto kc) {
            using I = PlaneIter<decltype(kc)::value, N, RING>;
            constexpr int j = I::j, j1 = (j + 1) % 3, jm = (j + 2) % 3;
            enter(k, I{});
            if (I::phase < 2) return;
            __syncthreads();
            stage_a(k, I{}, true);
            __syncthreads();
            if (I::phase < 4) return;
            // ---- step t - 1 at plane tz = pz - 2 (z0 .. z1 - 1)
            const int tz = z0 - 4 + k;
            float d, ux, uy, uz;
            StateIO<T>::unpack(sb[j1], p.ld_scale, d, ux, uy, uz);
            float da = da_b;
            const f32x4 lam = adj_point<false, NS2 + 1, SX2>(w2[j1], w2[jm], w2[j], slot2, d, ux, uy,
                                                             uz, 0u, nullptr, 0, p, da);
            da_b = tz >= zs ? da : da_b;
            if (FINAL) {
                // the gradient with respect to the initial state, field-major.
                // (One whole-vector cast, then component selection: this
                // compiler returns the first element for every component when
                // the elements are bit-cast one by one.)
                const unsigned so = (unsigned)tz * (unsigned)(plane * 4);
                const unsigned fs = (unsigned)(n * 4);
                const u32x4 lb = __builtin_bit_cast(u32x4, lam);
                __builtin_amdgcn_raw_buffer_store_b32(lb.x, rout, col * 4u, so, 0);
                store_data_guard();
                __builtin_amdgcn_raw_buffer_store_b32(lb.y, rout, col * 4u, so + fs, 0);
                store_data_guard();
                __builtin_amdgcn_raw_buffer_store_b32(lb.z, rout, col * 4u, so + 2 * fs, 0);
                store_data_guard();
                __builtin_amdgcn_raw_buffer_store_b32(lb.w, rout, col * 4u, so + 3 * fs, 0);
                store_data_guard();
            } else {
                const f32x4 mu = fold_normalisation(lam, d, ux, uy, uz);
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, mu), rout, voff_mu,
                                                       (unsigned)tz * mu_plane, 0);
                store_data_guard();
            }
            __builtin_amdgcn_sched_barrier(0);  // the state's last use is above
            if (I::refill) sb[j1] = StateIO<T>::load(rsb, voff_st, (unsigned)(z0 - 1 + k) * st_plane);
        });
    } else if (tid < HALO0) {
        plane_loop<N>([&](int k, auto kc) {
            using I = PlaneIter<decltype(kc)::value, N, RING>;
            enter(k, I{});
            if (I::phase < 2) return;
            __syncthreads();
            stage_a(k, I{}, false);
            __syncthreads();
        });
    } else {
        plane_loop<N>([&](int k, auto kc) {
            using I = PlaneIter<decltype(kc)::value, N, RING>;
            enter(k, I{});
            if (I::phase < 2) return;
            __syncthreads();
            __syncthreads();
        });
    }

    double sums[2] = {(double)da_a, (double)da_b};
    block_sum<2>(sums);
    if (tid == 0) {
        r.partials[blockIdx.x] = sums[0];
        r.partials_b[blockIdx.x] = sums[1];
    }
}

template <class T, bool FINAL>
void launch_t(const ProblemArgs &p, const void *sa, const void *sb, const float *mu_in,
              float *mu_out, const ReduceArgs &r, unsigned nb, hipStream_t s)
{
    const T *a = static_cast<const T *>(sa);
    const T *b = static_cast<const T *>(sb);
    switch (adj2_nzc(p)) {
    case 8: k_adj_march2<T, FINAL, 8><<<nb, NTHREADS, 0, s>>>(p, a, b, mu_in, mu_out, r); break;
    case 16: k_adj_march2<T, FINAL, 16><<<nb, NTHREADS, 0, s>>>(p, a, b, mu_in, mu_out, r); break;
    case 32: k_adj_march2<T, FINAL, 32><<<nb, NTHREADS, 0, s>>>(p, a, b, mu_in, mu_out, r); break;
    case 64: k_adj_march2<T, FINAL, 64><<<nb, NTHREADS, 0, s>>>(p, a, b, mu_in, mu_out, r); break;
    default: k_adj_march2<T, FINAL, 128><<<nb, NTHREADS, 0, s>>>(p, a, b, mu_in, mu_out, r); break;
    }
}

}  // namespace

bool adj_march2_supported(const ProblemArgs &p)
{
    return adj_march_supported(p) && !p.mask && p.nz >= 8;
}

unsigned adj_march2_num_blocks(const ProblemArgs &p)
{
    if (!adj_march2_supported(p)) return 0;
    const int c = adj2_nzc(p);
    return (unsigned)((long long)(p.nx / TX) * (p.ny / TY) * ((p.nz + c - 1) / c));
}

hipError_t launch_adj_march2(const ProblemArgs &p, int storage, const void *state_t,
                             const void *state_tm1, const float *mu_in, float *mu_out,
                             int final_t0, const ReduceArgs &r, hipStream_t stream)
{
    if (!adj_march2_supported(p) || !r.partials_b) return hipErrorNotSupported;
    const unsigned nb = adj_march2_num_blocks(p);
    if (storage) {
        if (final_t0) launch_t<__half, true>(p, state_t, state_tm1, mu_in, mu_out, r, nb, stream);
        else launch_t<__half, false>(p, state_t, state_tm1, mu_in, mu_out, r, nb, stream);
    } else {
        if (final_t0) launch_t<float, true>(p, state_t, state_tm1, mu_in, mu_out, r, nb, stream);
        else launch_t<float, false>(p, state_t, state_tm1, mu_in, mu_out, r, nb, stream);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the two steps' dL/domega, in the order two one-step calls add them (r.out
    // null: the caller adds the block partials itself, lwacm_adjoint_sweep)
    if (!r.out) return hipSuccess;
    e = launch_reduce(r, 1, nb, stream);
    if (e != hipSuccess) return e;
    ReduceArgs rb = r;
    rb.partials = r.partials_b;
    return launch_reduce(rb, 1, nb, stream);
}

}  // namespace lwacm
