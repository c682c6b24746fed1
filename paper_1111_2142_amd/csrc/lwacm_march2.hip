// lwacm_march2.hip -- two D3Q19 LW-ACM forward steps per pass over the state.
//
// The single-step tile kernel moves 32 bytes per lattice update (16 read, 16
// written) and runs at the HBM bound; its arithmetic (Eqs. ACM2.0b) needs
// less than half of that time.  This kernel reads the state of step t once,
// computes step t + 1 on a tile grown by one column on every side, keeps that
// intermediate state on chip, computes step t + 2 on the tile and writes it:
// 16 bytes per update, in exchange for the first step's extra ring of
// columns.  With FP32 storage the step then becomes bound by arithmetic,
// which is the regime the paper anticipates for the link-wise method.
//
// Layout (tile 32 x 16 columns, one thread per column, marching up a chunk of
// NZC planes, as in the single-step kernel):
//   waves 0-7   the 32 x 16 tile: both steps, all 19 links;
//   waves 8-9   the 100 columns around it: the first step (all links), and
//               the five second-step links that point into the tile;
//   waves 10-11 the 108 columns at distance two: only the five first-step
//               links that point inwards.
// Every role is wave-uniform.  Each iteration of the plane loop loads plane
// pz of step t, pushes its link terms, finalises plane pz - 1 of step t + 1
// (first LDS exchange, 36 x 20 slots), pushes that node's step-(t + 1) link
// terms and finalises plane pz - 2 of step t + 2 (second exchange, 34 x 18
// slots).  The chunk reads planes z0 - 2 .. z1 + 1.
//
// Every node of either step is computed with the same operations, in the
// same order, as in the single-step kernel (the column helpers are shared),
// so two steps of this kernel are bitwise equal to two single steps, and the
// per-block mass and energy partials of both steps are the same numbers.
//
// Walls (MASK): halfway bounce-back and moving walls as in the single-step
// kernel.  Every column loads its node's link set with the node's state; the
// first step's nodes (tile and first ring) sum their bounced-back terms when
// pushed and take the moving-wall term from the geometry sums, and the
// second step uses the link set and class that the first step's push kept.
// A solid node pushes nothing in either step and is not written: both state
// buffers hold its unchanged values.
#include "lwacm_march_common.hpp"

namespace lwacm {

namespace {

constexpr int TX = 32;
constexpr int TY = 16;
constexpr int RING = 3;                              // planes of step t in flight per thread
constexpr int NINT = TX * TY;                        // tile columns: waves 0-7
constexpr int HALO0 = NINT + 2 * kWave;              // first thread of the outer ring
constexpr int NTHREADS = NINT + 4 * kWave;
constexpr int SX1 = TX + 4, NS1 = SX1 * (TY + 4);    // first-step exchange slots
constexpr int SX2 = TX + 2, NS2 = SX2 * (TY + 2);    // second-step exchange slots


// Second pass of up to two previous steps' (mass, energy) sums, by block 0:
// the same fixed order as k_reduce_partials, the older step written first.
__device__ __forceinline__ void finish_previous_sums2(const ReduceArgs &r)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (threadIdx.x < kReduceThreads) {
        for (unsigned b = threadIdx.x; b < r.prev_nblocks; b += kReduceThreads) {
            acc[0] += r.prev_partials[2 * (size_t)b];
            acc[1] += r.prev_partials[2 * (size_t)b + 1];
        }
        for (unsigned b = threadIdx.x; b < r.prev_nblocks_b; b += kReduceThreads) {
            acc[2] += r.prev_partials_b[2 * (size_t)b];
            acc[3] += r.prev_partials_b[2 * (size_t)b + 1];
        }
    }
    block_sum<4>(acc);
    if (threadIdx.x == 0) {
        if (r.prev_nblocks) {
            r.prev_out[0] = acc[0];
            r.prev_out[1] = acc[1];
            if (r.prev_out2) {
                r.prev_out2[0] = acc[0];
                r.prev_out2[1] = acc[1];
            }
        }
        if (r.prev_nblocks_b) {
            r.prev_out_b[0] = acc[2];
            r.prev_out_b[1] = acc[3];
            if (r.prev_out2_b) {
                r.prev_out2_b[0] = acc[2];
                r.prev_out2_b[1] = acc[3];
            }
        }
    }
}

template <int NZC, bool MASK>
__global__ __launch_bounds__(NTHREADS) void k_fwd_march2(ProblemArgs p,
                                                         const float *__restrict__ src,
                                                         float *__restrict__ dst,
                                                         const unsigned *__restrict__ bb_bits,
                                                         const float4 *__restrict__ wallg,
                                                         ReduceArgs r)
{
    // one spare slot per array: idle lanes write there instead of branching
    __shared__ float2 xp1[4][NS1 + 1];
    __shared__ float xd1[4][NS1 + 1];
    __shared__ float2 xp2[4][NS2 + 1];
    __shared__ float xd2[4][NS2 + 1];
    const Xchg<NS1 + 1> X1{xp1, xd1};
    const Xchg<NS2 + 1> X2{xp2, xd2};

    const int tid = threadIdx.x;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long n = p.n;
    const long long plane = (long long)nx * ny;

    const TileIdx ti = tile_of_block(nx, ny, TX, TY);
    // Every chunk is NZC planes deep (nz >= NZC): a ragged last chunk is moved
    // down to end at nz.  Planes it shares with the chunk below are written
    // twice with bitwise the same values and counted in the sums only once,
    // from zs on, so each block sums the planes the single-step kernel's
    // block of the same index sums.
    const int zs = ti.zc * NZC;
    const int z0 = min(zs, nz - NZC);
    const int z1 = z0 + NZC;

    const Col2 c2 = col2_of<TX, TY>(tid);
    const int lx = c2.lx, ly = c2.ly;
    const float sgn = c2.sgn;
    const bool isY = c2.isY, active = c2.active;
    const int gx = wrap_index(ti.tile_x * TX + lx, nx);
    const int gy = wrap_index(ti.tile_y * TY + ly, ny);
    const unsigned col = (unsigned)(gy * nx + gx);  // offset inside a plane (< 2^31)
    const int slot1 = (ly + 2) * SX1 + (lx + 2);
    const int slot2 = (ly + 1) * SX2 + (lx + 1);    // tile and first ring only
    const int wslot1 = active ? slot1 : NS1;        // LDS writes of idle lanes go
    const int wslot2 = active ? slot2 : NS2;        // to the spare slots
    // The first ring pushes only the five second-step links that point into
    // the tile, like a halo column: rows below/above it (corners included)
    // along y, columns left/right of it along x.
    const bool isY2 = ly < 0 || ly >= TY;
    const float sgn2 = (isY2 ? ly >= TY : lx >= TX) ? -1.0f : 1.0f;

    const float A = p.A;
    const float a = p.a;

    // plane index with periodic wrap (nz >= NZC >= 2, so one period suffices)
    auto wrapz = [&](int pz) { return wrap_index(pz, nz); };
    constexpr unsigned NB = BufIO<float>::kNodeBytes;
    const unsigned plane_bytes = (unsigned)(plane * (long long)NB);
    const unsigned long long sbytes = (unsigned long long)n * NB;
    const Rsrc rs = make_rsrc(src, sbytes);
    const Rsrc rd = make_rsrc(dst, sbytes);
    const unsigned voff = col * NB;
    // link sets of the ring's planes (MASK): bit i set when x - v_i is solid,
    // bit 0 alone for a solid node, plus the moving-wall flag
    const Rsrc rbits = make_rsrc(bb_bits, MASK ? (unsigned long long)n * 4u : 0ull);
    unsigned bw[RING] = {0u, 0u, 0u};
    auto issue = [&](int j, Ring<float> &rg, int pz) {
        const unsigned pw = (unsigned)wrapz(pz);
        rg.v = BufIO<float>::load(rs, voff, pw * plane_bytes);
        if (MASK)
            bw[j] = __builtin_amdgcn_raw_buffer_load_b32(rbits, col * 4u, pw * (unsigned)(plane * 4),
                                                         0);
    };
    auto class_of = [](unsigned b) { return (b & 1u) ? 2 : (b ? 1 : 0); };

    Ring<float> ring[RING];
#pragma unroll
    for (int j = 0; j < RING; ++j) issue(j, ring[j], z0 - 2 + j);

    float m1 = 0.0f, e1 = 0.0f, m2 = 0.0f, e2 = 0.0f;
    constexpr int N = NZC + 4;  // planes z0 - 2 .. z1 + 1

    // The three roles run separate loops (wave-uniform), with the same
    // barriers: two per iteration from k = 2 on, after the first-step and
    // after the second-step exchange.  Inside each loop every prefetch and
    // store is unconditional, so the compiler's wait counts keep the next
    // planes' loads in flight.
    Acc acc1[3], acc2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        acc1[j] = Acc{};
        acc2[j] = Acc{};
    }
    // five-link partials of the halo pushes (outer ring: first step; first
    // ring: second step)
    float hp[3] = {0.0f, 0.0f, 0.0f}, hz[3] = {0.0f, 0.0f, 0.0f};
    float hd1[3] = {0.0f, 0.0f, 0.0f}, hd2[3] = {0.0f, 0.0f, 0.0f};
    // The ring slot of iteration k is refilled (with plane pz + RING) only
    // after its last use: the new load then takes the same registers, so the
    // loop's back edge needs no register copies, which would have to wait for
    // the loads in flight.  The scheduling barrier keeps the load there.
    auto refill = [&](int k, auto It) {
        using I = decltype(It);
        __builtin_amdgcn_sched_barrier(0);
        if (I::refill) issue(I::j, ring[I::j], z0 - 2 + k + RING);
    };
    // Step t pushes of the plane loaded for iteration k (pz = z0 - 2 + k).
    auto first_push = [&](int k, auto It) {
        using I = decltype(It);
        __builtin_amdgcn_sched_barrier(0);  // no work of this iteration moves up
        const f32x4 v = ring[I::j].v;
        const unsigned b = bw[I::j];
        push_column<MASK>(v.x, v.y, v.z, v.w, MASK ? class_of(b) : 0, b, A, a,
                          acc1[(I::j + 1) % 3], acc1[I::j], acc1[(I::j + 2) % 3]);
        refill(k, It);
    };
    // Step t + 1 at plane tq = pz - 1 (z0 - 1 .. z1) and its step-(t + 2)
    // pushes; exchange of step t + 2 at plane pz - 2 from iteration 4 on.
    auto middle = [&](int k, auto It, bool tile) {
        using I = decltype(It);
        Acc &Am = acc1[(I::j + 2) % 3];
        put_slot(X1, wslot1, Am);
        __syncthreads();
        const int tq = z0 - 3 + k;
        const NodeOut o = finalize<MASK, NS1 + 1, SX1>(X1, slot1, Am, p, wallg,
                                                       (long long)wrapz(tq) * plane + col);
        // the node's class and link set at plane tq, kept by its first push
        const int cls = MASK ? Am.cls : 0;
        const unsigned bits = MASK ? Am.bits : 0u;
        if (tile) {
            const bool count = tq >= zs && tq < z1 && cls < 2;
            m1 += count ? o.D : 0.0f;
            e1 = count ? fmaf(o.vx, o.vx, fmaf(o.vy, o.vy, fmaf(o.vz, o.vz, e1))) : e1;
        }
        if (tile) {
            push_column<MASK>(o.D, o.vx, o.vy, o.vz, cls, bits, A, a, acc2[(I::j + 1) % 3],
                              acc2[I::j], acc2[(I::j + 2) % 3]);
            if (I::phase >= 4) put_slot(X2, wslot2, acc2[(I::j + 2) % 3]);
        } else {
            constexpr int j = I::j, j1 = (j + 1) % 3, jm = (j + 2) % 3;
            push_halo<MASK>(o.D, o.vx, o.vy, o.vz, cls, A, isY2, sgn2, hp[j1], hz[j1], hp[j],
                            hd1[j], hd2[j], hp[jm], hz[jm]);
            if (I::phase >= 4) put_halo(X2, wslot2, isY2, sgn2, hp[jm], hz[jm], hd1[jm], hd2[jm]);
        }
        __syncthreads();
    };

    if (tid < NINT) {
        plane_loop<N>([&](int k, auto kc) {
            using I = PlaneIter<decltype(kc)::value, N, RING>;
            first_push(k, I{});
            if (I::phase < 2) return;
            middle(k, I{}, true);
            if (I::phase < 4) return;
            // ---- step t + 2 at plane tz = pz - 2 (z0 .. z1 - 1)
            const int tz = z0 - 4 + k;
            const Acc &A2 = acc2[(I::j + 2) % 3];
            const NodeOut o2 = finalize<MASK, NS2 + 1, SX2>(X2, slot2, A2, p, wallg,
                                                            (long long)tz * plane + col);
            const f32x4 out = BufIO<float>::pack(o2.D, o2.vx, o2.vy, o2.vz, p.st_scale);
            const bool solid = MASK && A2.cls >= 2;
            const unsigned so = (unsigned)tz * plane_bytes;
            if (MASK)  // a solid node's store is dropped past the buffer's end: both buffers
                       // hold its state (see the single-step kernel)
                BufIO<float>::store_raw(rd, solid ? 0xfffffff0u : voff + so, 0u, out);
            else
                BufIO<float>::store_raw(rd, voff, so, out);
            const bool count = tz >= zs && !solid;
            m2 += count ? o2.D : 0.0f;
            e2 = count ? fmaf(o2.vx, o2.vx, fmaf(o2.vy, o2.vy, fmaf(o2.vz, o2.vz, e2))) : e2;
        });
    } else if (tid < HALO0) {
        plane_loop<N>([&](int k, auto kc) {
            using I = PlaneIter<decltype(kc)::value, N, RING>;
            first_push(k, I{});
            if (I::phase < 2) return;
            middle(k, I{}, false);
        });
    } else {
        plane_loop<N>([&](int k, auto kc) {
            using I = PlaneIter<decltype(kc)::value, N, RING>;
            constexpr int j = I::j, j1 = (j + 1) % 3, jm = (j + 2) % 3;
            __builtin_amdgcn_sched_barrier(0);
            const f32x4 v = ring[j].v;
            push_halo<MASK>(v.x, v.y, v.z, v.w, MASK ? class_of(bw[j]) : 0, A, isY, sgn, hp[j1],
                            hz[j1], hp[j], hd1[j], hd2[j], hp[jm], hz[jm]);
            refill(k, I{});
            if (I::phase < 2) return;
            put_halo(X1, wslot1, isY, sgn, hp[jm], hz[jm], hd1[jm], hd2[jm]);
            __syncthreads();
            __syncthreads();
        });
    }

    double sums[4] = {(double)m1, 0.5 * (double)e1, (double)m2, 0.5 * (double)e2};
    block_sum<4>(sums);
    if (tid == 0) {
        r.partials[2 * (size_t)blockIdx.x] = sums[0];
        r.partials[2 * (size_t)blockIdx.x + 1] = sums[1];
        r.partials_b[2 * (size_t)blockIdx.x] = sums[2];
        r.partials_b[2 * (size_t)blockIdx.x + 1] = sums[3];
    }
    if (blockIdx.x == 0 && (r.prev_nblocks || r.prev_nblocks_b)) finish_previous_sums2(r);
}

// Chunk depth: the single-step kernel's, halved until it fits in nz.
int march2_nzc(const ProblemArgs &p)
{
    int c = p.march_nzc;
    while (c > 8 && c > p.nz) c /= 2;
    return c <= p.nz ? c : 0;
}

}  // namespace

bool march2_supported(const ProblemArgs &p)
{
    // halfway walls (moving or not) allowed; the per-step wall correction of
    // interpolated walls and link velocities needs one launch per step
    return march_supported(p) && !p.corr && !p.qd && !p.uwl && !p.split && !p.has_force &&
           p.march_nzc > 0 && p.nz >= 8;
}

unsigned march2_num_blocks(const ProblemArgs &p)
{
    if (!march2_supported(p)) return 0;
    const int c = march2_nzc(p);
    return (unsigned)((long long)(p.nx / TX) * (p.ny / TY) * ((p.nz + c - 1) / c));
}

template <bool MASK>
hipError_t launch_march2_t(const ProblemArgs &p, const float *src, float *dst,
                           const unsigned *bb_bits, const float4 *wallg, const ReduceArgs &r,
                           hipStream_t s)
{
    const unsigned nb = march2_num_blocks(p);
    switch (march2_nzc(p)) {
    case 8: k_fwd_march2<8, MASK><<<nb, NTHREADS, 0, s>>>(p, src, dst, bb_bits, wallg, r); break;
    case 16: k_fwd_march2<16, MASK><<<nb, NTHREADS, 0, s>>>(p, src, dst, bb_bits, wallg, r); break;
    case 32: k_fwd_march2<32, MASK><<<nb, NTHREADS, 0, s>>>(p, src, dst, bb_bits, wallg, r); break;
    case 64: k_fwd_march2<64, MASK><<<nb, NTHREADS, 0, s>>>(p, src, dst, bb_bits, wallg, r); break;
    case 128:
        k_fwd_march2<128, MASK><<<nb, NTHREADS, 0, s>>>(p, src, dst, bb_bits, wallg, r);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fwd_march2(const ProblemArgs &p, const float *src, float *dst,
                             const unsigned *bb_bits, const float4 *wallg, const ReduceArgs &r,
                             hipStream_t s)
{
    if (!march2_supported(p) || !r.partials_b) return hipErrorNotSupported;
    if (p.mask && !bb_bits) return hipErrorInvalidValue;  // the link sets come from k_classify
    return p.mask ? launch_march2_t<true>(p, src, dst, bb_bits, wallg, r, s)
                  : launch_march2_t<false>(p, src, dst, nullptr, nullptr, r, s);
}

}  // namespace lwacm
