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
// stores.  A body acceleration (Eq. force, uniform or node by node) enters
// that post-combine term as a rho u + rho g in one FMA.  Halfway bounce-back
// (Eqs. ACM2.0cbb-ACM2.0ccccbb) uses a precomputed per-node bit set of solid
// upstream links: a node sums its own bounced-back terms when it is pushed,
// and solid nodes push zeros and keep their state.
//
// Link terms are kept unweighted and summed with the exact integer weights
// 12, 2, 1 (= 36 w_i for rest, axis and diagonal links of D3Q19); the sums
// are divided by 36 once at the end (div36: no systematic rounding bias).
#include "lwacm_march_common.hpp"

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
// Planes per workgroup: a template parameter (ring and accumulator indices
// are compile-time constants), chosen per problem among kChunkDepths by
// march_choose_nzc().
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
                // link sets: only planes this chunk finalises (z0 <= pz < z1 <= nz)
                unsigned bits = 0u;
                if (MASK && cls == 1 && pz >= z0 && pz < z1)
                    bits = bb_bits[(long long)pz * plane + col];

                push_column<MASK>(dr, ux, uy, uz, cls, bits, A, a, A1, A0, Am, p.corr == nullptr);

                if (k < 2) return;  // planes below the chunk are halo only
                // ---- exchange the partials of plane pz - 1 through LDS
                if (NBUF == 1 && k > 2) __syncthreads();  // previous plane's reads done
                const Xchg<NSLOT> X{xp[k % NBUF], xd[k % NBUF]};
                put_slot(X, slot, Am);
                __syncthreads();
                const int tz = pz - 1;
                if (tz >= z1) return;  // padding iteration: nothing to finalise
                const NodeOut o = finalize<MASK, NSLOT, SX>(X, slot, Am, p, wallg,
                                                            (long long)tz * plane + col);
                const float D = o.D, vx = o.vx, vy = o.vy, vz = o.vz;
                if (!MASK || Am.cls < 2) {
                    const unsigned so = (unsigned)tz * plane_bytes;
                    if (std::is_same<T, __half>::value && p.fp16_sr) {
                        const U32x4 h = sr_words((uint32_t)((long long)tz * plane + col), p.sr_word);
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
                push_halo<MASK>(dr, ux, uy, uz, cls, A, role == HALO_Y, sgn, hp[j1], hz[j1], hp[j],
                                hd1[j], hd2[j], hp[jm], hz[jm]);
                if (k < 2) return;
                if (NBUF == 1 && k > 2) __syncthreads();
                if (active)
                    put_halo(Xchg<NSLOT>{xp[k % NBUF], xd[k % NBUF]}, slot, role == HALO_Y, sgn,
                             hp[jm], hz[jm], hd1[jm], hd2[jm]);
                __syncthreads();
            }
        });
    }

    double v[2] = {(double)mass, 0.5 * (double)energy};
    store_block_partials<2>(v, r.partials, blockIdx.x);
    if (blockIdx.x == 0 && r.prev_nblocks)
        finish_previous_sums(r.prev_partials, r.prev_nblocks, r.prev_out, r.prev_out2);
}

// The same step with the plane loop rolled (plane_loop: small code, so the
// instruction cache holds it) and every chunk NZC planes deep: a ragged last
// chunk is moved down to end at nz, its planes below zs written twice with
// the same bits and summed once.  Inside the loop every load and store is
// unconditional and a ring slot is refilled right after its last use, so the
// loads stay in flight across the back edge.  With walls, each node's 32-bit
// link set is loaded with its state on every plane (bit 0 marks a solid
// node), and a solid node stores back the value it loaded, so that its store
// too is unconditional; only the moving-wall sums are loaded conditionally,
// by the waves next to a moving wall.  Node for node the same operations as
// k_fwd_march (the column helpers are shared), so the same results.
// SPLIT: a separate omega_p for the density (no walls): the columns also
// push q = 36 w (Ap - A) rho (v . u) through eight more LDS arrays.
// FRC: body acceleration (Eq. force), 0 none, 1 uniform p.g, 2 node by node
// from p.g_field (loaded with the state).  The forcing adds rho(x, t) g(x) to
// the node's momentum; it enters the node's post-combine term a rho u through
// the addend of its FMA, where it meets a node-dependent product.
// THERM: the temperature lattice's step (Eq. ACM2.0t) in the same pass, from
// the same step-t velocities: each column also loads its T (p.T_in) with the
// state, pushes the temperature terms through the omega_p arrays and writes
// the new T (p.T_out): 4 + 4 bytes more per node instead of a pass of its own
// (with walls 8 more: the node's fixed-temperature wall links and their sum).
template <class T, int NZC, bool SR, bool MASK, bool SPLIT, int FRC, bool CORR, bool THERM>
__global__ __launch_bounds__(NTHREADS) void k_fwd_march_rolled(ProblemArgs p,
                                                               const T *__restrict__ src,
                                                               T *__restrict__ dst,
                                                               const unsigned *__restrict__ bb_bits,
                                                               const float4 *__restrict__ wallg,
                                                               ReduceArgs r)
{
    // two exchange buffers (by iteration parity) with one spare slot each:
    // idle halo lanes write there instead of branching
    __shared__ float2 xp[2][4][NSLOT + 1];
    __shared__ float xd[2][4][NSLOT + 1];
    constexpr bool QX = SPLIT || THERM;          // the q arrays are used
    constexpr int QS = QX ? NSLOT + 1 : 1;       // q slots (one spare, as above)
    __shared__ float xq[QX ? 2 : 1][8][QS];
    static_assert(!(SPLIT && MASK), "the separate omega_p runs without walls");
    static_assert(!THERM || (!CORR && !SPLIT && FRC == 0),
                  "the fused temperature step: halfway walls, no force or omega_p");
    const float dA = p.Ap - p.A;

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long n = p.n;
    const long long plane = (long long)nx * ny;

    const TileIdx ti = tile_of_block(nx, ny, TX, TY);
    const int zs = ti.zc * NZC;
    const int z0 = min(zs, nz - NZC);

    const int role = tid < NINT ? INTERIOR : (tid < NINT + kWave ? HALO_Y : HALO_X);
    int lx, ly;
    float sgn = 1.0f;
    bool active = true;
    if (role == INTERIOR) {
        lx = tid % TX;
        ly = tid / TX;
    } else if (role == HALO_Y) {
        const bool top = lane >= TX;
        lx = top ? lane - TX : lane;
        ly = top ? TY : -1;
        sgn = top ? -1.0f : 1.0f;
        active = lane < 2 * TX;
        if (!active) lx = 0;
    } else {
        const bool right = lane >= TY + 2;
        const int l = right ? lane - (TY + 2) : lane;
        lx = right ? TX : -1;
        ly = l - 1;
        sgn = right ? -1.0f : 1.0f;
        active = lane < 2 * (TY + 2);
        if (!active) ly = 0;
    }
    const int gx = wrap_index(ti.tile_x * TX + lx, nx);
    const int gy = wrap_index(ti.tile_y * TY + ly, ny);
    const unsigned col = (unsigned)(gy * nx + gx);
    const int slot = (ly + 1) * SX + (lx + 1);
    const int wslot = active ? slot : NSLOT;

    const float A = p.A;
    const float a = p.a;
    constexpr unsigned NB = BufIO<T>::kNodeBytes;
    const unsigned plane_bytes = (unsigned)(plane * (long long)NB);
    const unsigned long long sbytes = (unsigned long long)n * NB;
    const Rsrc rs = make_rsrc(src, sbytes);
    const Rsrc rd = make_rsrc(dst, sbytes);
    const unsigned voff = col * NB;
    const Rsrc rbits = make_rsrc(bb_bits, MASK ? (unsigned long long)n * 4u : 0ull);
    unsigned bw[3] = {0u, 0u, 0u};  // link sets of the ring's planes (MASK)
    // temperature in and out (THERM), and the T of the ring's planes
    const Rsrc rTi = make_rsrc(THERM ? p.T_in : nullptr, THERM ? (unsigned long long)n * 4u : 0ull);
    const Rsrc rTo = make_rsrc(THERM ? p.T_out : nullptr, THERM ? (unsigned long long)n * 4u : 0ull);
    unsigned tw[3] = {0u, 0u, 0u};
    // with walls, each node's links into fixed-temperature walls and the sum of
    // 36 w T_w over them (a table lwacm_set_thermal builds)
    constexpr bool TWALL = THERM && MASK;
    const Rsrc rTw = make_rsrc(TWALL ? (const void *)p.T_wall : nullptr,
                               TWALL ? (unsigned long long)n * 8u : 0ull);
    uint2 twb[3] = {{0u, 0u}, {0u, 0u}, {0u, 0u}};
    auto issue = [&](int j, Ring<T> &rg, int pz) {
        const unsigned pw = (unsigned)wrap_index(pz, nz);
        rg.v = BufIO<T>::load(rs, voff, pw * plane_bytes);
        if (MASK) bw[j] = __builtin_amdgcn_raw_buffer_load_b32(rbits, col * 4u, pw * (unsigned)(plane * 4), 0);
        if (THERM) tw[j] = __builtin_amdgcn_raw_buffer_load_b32(rTi, col * 4u, pw * (unsigned)(plane * 4), 0);
        if (TWALL)
            twb[j] = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(
                                                   rTw, col * 8u, pw * (unsigned)(plane * 8), 0));
    };
    // node-by-node acceleration (FRC 2): three FP32 fields, one resource each
    const unsigned long long gbytes = FRC == 2 ? (unsigned long long)n * 4u : 0ull;
    const Rsrc rgx = make_rsrc(FRC == 2 ? p.g_field : nullptr, gbytes);
    const Rsrc rgy = make_rsrc(FRC == 2 ? p.g_field + n : nullptr, gbytes);
    const Rsrc rgz = make_rsrc(FRC == 2 ? p.g_field + 2 * n : nullptr, gbytes);
    unsigned gq[3][3] = {{0u, 0u, 0u}, {0u, 0u, 0u}, {0u, 0u, 0u}};  // FP32 bits of g
    auto issue_g = [&](int j, int pz) {
        const unsigned so = (unsigned)wrap_index(pz, nz) * (unsigned)(plane * 4);
        gq[j][0] = __builtin_amdgcn_raw_buffer_load_b32(rgx, col * 4u, so, 0);
        gq[j][1] = __builtin_amdgcn_raw_buffer_load_b32(rgy, col * 4u, so, 0);
        gq[j][2] = __builtin_amdgcn_raw_buffer_load_b32(rgz, col * 4u, so, 0);
    };
    auto class_of = [](unsigned b) { return (b & 1u) ? 2 : (b ? 1 : 0); };
    // per-step wall correction (interpolated walls, link velocities): one
    // float4 per node next to a wall, loaded at the top of the iteration that
    // finalises its plane so that its latency hides behind the plane's work
    // CORR: interpolated walls or link velocities, the wall term from the
    // per-step correction (p.corr) in place of the bounce-back sums
    static_assert(!CORR || MASK, "the wall correction needs walls");
    constexpr bool corr = CORR;
    const Rsrc rcorr = make_rsrc(corr ? (const void *)p.corr : nullptr,
                                 corr ? (unsigned long long)n * 16u : 0ull);

    Ring<T> ring[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) issue(j, ring[j], z0 - 1 + j);
    // corrections of the ring's planes (slot = the plane's ring slot)
    f32x4 cwr[3] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
    if (FRC == 2 && role == INTERIOR)
#pragma unroll
        for (int j = 0; j < 3; ++j) issue_g(j, z0 - 1 + j);

    float mass = 0.0f, energy = 0.0f;
    constexpr int N = NZC + 2;  // planes z0 - 1 .. z1
    auto value = [&](const Ring<T> &rg, float &dr, float &ux, float &uy, float &uz) {
        dr = BufIO<T>::value(rg.v, 0, p.ld_scale[0]);
        ux = BufIO<T>::value(rg.v, 1, p.ld_scale[1]);
        uy = BufIO<T>::value(rg.v, 2, p.ld_scale[1]);
        uz = BufIO<T>::value(rg.v, 3, p.ld_scale[1]);
    };

    if (role == INTERIOR) {
        Acc acc[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[j] = Acc{};
        plane_loop<N>([&](int k, auto kc) {
            using I = PlaneIter<decltype(kc)::value, N, 3>;
            constexpr int j = I::j;
            __builtin_amdgcn_sched_barrier(0);
            float dr, ux, uy, uz;
            value(ring[j], dr, ux, uy, uz);
            const unsigned b = bw[j];
            Acc &Am = acc[(j + 2) % 3];  // target plane pz - 1 (finalised now)
            // the correction of plane pz - 1, loaded in the previous iteration
            const f32x4 cw = cwr[(j + 2) % 3];
            push_column<MASK>(dr, ux, uy, uz, MASK ? class_of(b) : 0, b, A, a, acc[(j + 1) % 3],
                              acc[j], Am, !corr);
            if (SPLIT) push_split_column(1.0f + dr, ux, uy, uz, dA, acc[(j + 1) % 3], acc[j], Am);
            if (THERM)
                push_temp_column<MASK>(__builtin_bit_cast(float, tw[j]), ux, uy, uz, p.t_h,
                                       acc[(j + 1) % 3], acc[j], Am, MASK ? class_of(b) : 0, b,
                                       twb[j]);
            if (FRC) {  // post-combine a rho u plus the forcing rho g
                const float rho = 1.0f + dr, arho = a * rho;
                const float gx = FRC == 2 ? __builtin_bit_cast(float, gq[j][0]) : p.g[0];
                const float gy = FRC == 2 ? __builtin_bit_cast(float, gq[j][1]) : p.g[1];
                const float gz = FRC == 2 ? __builtin_bit_cast(float, gq[j][2]) : p.g[2];
                acc[j].post[0] = fmaf(arho, ux, rho * gx);
                acc[j].post[1] = fmaf(arho, uy, rho * gy);
                acc[j].post[2] = fmaf(arho, uz, rho * gz);
            }
            if constexpr (CORR) {
                // the correction of plane pz (its link set is this
                // iteration's), finalised in the next iteration: issued before
                // this iteration's ring refill, so waiting for it then waits
                // for no load that is not due by then.  Two slots of cwr are
                // live at a time.  Lanes away from the walls ask for an offset
                // past the end of the buffer: zeros, no memory access.
                cwr[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                if (__builtin_amdgcn_ballot_w64(b > 1u) != 0ull) {
                    const unsigned node = (unsigned)wrap_index(z0 - 1 + k, nz) * (unsigned)plane + col;
                    cwr[j] = BufIO<float>::load(rcorr, b > 1u ? node * 16u : 0xfffffff0u, 0u);
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // the ring slot's last use is above
            if (I::refill) {
                issue(j, ring[j], z0 + 2 + k);
                if (FRC == 2) issue_g(j, z0 + 2 + k);
            }
            if (I::phase < 2) return;
            const Xchg<NSLOT + 1> X{xp[k & 1], xd[k & 1]};
            put_slot(X, slot, Am);
            if constexpr (QX) put_slot_split(XchgQ<QS>{xq[k & 1]}, slot, Am);
            __syncthreads();
            const int tz = z0 - 2 + k;
            float qsum = 0.0f;
            if constexpr (SPLIT) qsum = Am.qd + gather_split<QS, SX>(XchgQ<QS>{xq[k & 1]}, slot);
            const NodeOut o = finalize<MASK, NSLOT + 1, SX, SPLIT>(X, slot, Am, p, wallg,
                                                                   (long long)tz * plane + col,
                                                                   qsum, corr ? &cw : nullptr);
            const unsigned so = (unsigned)tz * plane_bytes;
            typename BufIO<T>::Raw out;
            if (SR) {  // FP16 storage, stochastic rounding (a template parameter: one path)
                const U32x4 h = sr_words((uint32_t)((long long)tz * plane + col), p.sr_word);
                out = BufIO<T>::pack_sr(o.D, o.vx, o.vy, o.vz, p.st_scale, h);
            } else {
                out = BufIO<T>::pack(o.D, o.vx, o.vy, o.vz, p.st_scale);
            }
            const bool solid = MASK && Am.cls >= 2;
            if (MASK) {
                // a solid node keeps its state, which both buffers hold
                // (lwacm_set_state and lwacm_load_state write both): its
                // store goes past the end of the buffer (n * NB <= 2^32 - 16
                // bytes), where the hardware drops it; the store itself stays
                // unconditional
                BufIO<T>::store_raw(rd, solid ? 0xfffffff0u : voff + so, 0u, out);
            } else {
                BufIO<T>::store_raw(rd, voff, so, out);
            }
            if constexpr (THERM) {
                // T(x, t + 1) = (2 - 2/omega_t) T(x) + the incoming terms / 36;
                // a solid node keeps its T (written, so both buffers hold it)
                const float Tsum = Am.qd + gather_split<QS, SX>(XchgQ<QS>{xq[k & 1]}, slot);
                const float Tn = solid ? Am.tx : fmaf(p.t_kap, Am.tx, div36(Tsum));
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, Tn), rTo,
                                                      col * 4u, (unsigned)tz * (unsigned)(plane * 4),
                                                      0);
                store_data_guard();
            }
            const bool count = tz >= zs && !solid;
            mass += count ? o.D : 0.0f;
            energy = count ? fmaf(o.vx, o.vx, fmaf(o.vy, o.vy, fmaf(o.vz, o.vz, energy))) : energy;
        });
    } else {
        float hp[3] = {0.0f, 0.0f, 0.0f}, hz[3] = {0.0f, 0.0f, 0.0f};
        float hd1[3] = {0.0f, 0.0f, 0.0f}, hd2[3] = {0.0f, 0.0f, 0.0f};
        float hq[3] = {0.0f, 0.0f, 0.0f}, hq1[3] = {0.0f, 0.0f, 0.0f}, hq2[3] = {0.0f, 0.0f, 0.0f};
        const bool isY = role == HALO_Y;
        plane_loop<N>([&](int k, auto kc) {
            using I = PlaneIter<decltype(kc)::value, N, 3>;
            constexpr int j = I::j, j1 = (j + 1) % 3, jm = (j + 2) % 3;
            __builtin_amdgcn_sched_barrier(0);
            float dr, ux, uy, uz;
            value(ring[j], dr, ux, uy, uz);
            push_halo<MASK>(dr, ux, uy, uz, MASK ? class_of(bw[j]) : 0, A, isY, sgn, hp[j1],
                            hz[j1], hp[j], hd1[j], hd2[j], hp[jm], hz[jm]);
            if (SPLIT)
                push_split_halo(1.0f + dr, ux, uy, uz, dA, isY, sgn, hq[j1], hq[j], hq1[j], hq2[j],
                                hq[jm]);
            if (THERM)
                push_temp_halo(__builtin_bit_cast(float, tw[j]), ux, uy, uz, p.t_h, isY, sgn, hq[j1],
                               hq[j], hq1[j], hq2[j], hq[jm], MASK && class_of(bw[j]) >= 2);
            __builtin_amdgcn_sched_barrier(0);
            if (I::refill) issue(j, ring[j], z0 + 2 + k);
            if (I::phase < 2) return;
            put_halo(Xchg<NSLOT + 1>{xp[k & 1], xd[k & 1]}, wslot, isY, sgn, hp[jm], hz[jm],
                     hd1[jm], hd2[jm]);
            if constexpr (QX)
                put_halo_split(XchgQ<QS>{xq[k & 1]}, wslot, isY, sgn, hq[jm], hq1[jm], hq2[jm]);
            __syncthreads();
        });
    }

    double v[2] = {(double)mass, 0.5 * (double)energy};
    store_block_partials<2>(v, r.partials, blockIdx.x);
    if (blockIdx.x == 0 && r.prev_nblocks)
        finish_previous_sums(r.prev_partials, r.prev_nblocks, r.prev_out, r.prev_out2);
}

// Chunk depth of the rolled kernel: the problem's, halved while deeper than
// nz (0: nz < 8, the unrolled kernel runs).
int rolled_nzc(const ProblemArgs &p)
{
    int c = p.march_nzc;
    while (c > 8 && c > p.nz) c /= 2;
    return c <= p.nz ? c : 0;
}

// Node classes and solid-upstream bit sets for the bounce-back of the march
// kernel: class 0 fluid with only fluid upstream nodes, 1 fluid with at
// least one solid upstream node (bit i set when x - v_i is solid), 2 solid
// (bit set 1: bit 0 alone, so the bit set also tells the class).
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
            bits[idx] = 1u;  // bit 0 (the rest link, never a bounce-back link): solid
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

template <class T, bool SR, bool MASK, bool SPLIT = false, int FRC = 0, bool CORR = false,
          bool THERM = false>
void launch_rolled(int c, unsigned nb, hipStream_t s, const ProblemArgs &p, const T *a, T *b,
                   const unsigned *bits, const float4 *wallg, const ReduceArgs &r)
{
    switch (c) {
    case 8: k_fwd_march_rolled<T, 8, SR, MASK, SPLIT, FRC, CORR, THERM><<<nb, NTHREADS, 0, s>>>(p, a, b, bits, wallg, r); break;
    case 16: k_fwd_march_rolled<T, 16, SR, MASK, SPLIT, FRC, CORR, THERM><<<nb, NTHREADS, 0, s>>>(p, a, b, bits, wallg, r); break;
    case 32: k_fwd_march_rolled<T, 32, SR, MASK, SPLIT, FRC, CORR, THERM><<<nb, NTHREADS, 0, s>>>(p, a, b, bits, wallg, r); break;
    case 64: k_fwd_march_rolled<T, 64, SR, MASK, SPLIT, FRC, CORR, THERM><<<nb, NTHREADS, 0, s>>>(p, a, b, bits, wallg, r); break;
    default: k_fwd_march_rolled<T, 128, SR, MASK, SPLIT, FRC, CORR, THERM><<<nb, NTHREADS, 0, s>>>(p, a, b, bits, wallg, r); break;
    }
}

// forced problems (march_supported: nz >= 8, no separate omega_p)
template <class T, bool SR, bool MASK, bool CORR = false>
void launch_rolled_forced(int c, unsigned nb, hipStream_t s, const ProblemArgs &p, const T *a,
                          T *b, const unsigned *bits, const float4 *wallg, const ReduceArgs &r)
{
    if (p.g_field)
        launch_rolled<T, SR, MASK, false, 2, CORR>(c, nb, s, p, a, b, bits, wallg, r);
    else
        launch_rolled<T, SR, MASK, false, 1, CORR>(c, nb, s, p, a, b, bits, wallg, r);
}

// walls: halfway bounce-back in the kernel, or the per-step wall correction
template <class T, bool SR>
void launch_rolled_walls(int c, unsigned nb, hipStream_t s, const ProblemArgs &p, const T *a,
                         T *b, const unsigned *bits, const float4 *wallg, const ReduceArgs &r)
{
    if (p.has_force) {
        if (p.corr) launch_rolled_forced<T, SR, true, true>(c, nb, s, p, a, b, bits, wallg, r);
        else launch_rolled_forced<T, SR, true, false>(c, nb, s, p, a, b, bits, wallg, r);
    } else {
        if (p.corr) launch_rolled<T, SR, true, false, 0, true>(c, nb, s, p, a, b, bits, wallg, r);
        else launch_rolled<T, SR, true>(c, nb, s, p, a, b, bits, wallg, r);
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
    const int c = rolled_nzc(p);
    const bool sr = std::is_same<T, __half>::value && p.fp16_sr;
    if (p.T_in) {  // with the temperature step (march_thermal_supported)
        if constexpr (std::is_same<T, __half>::value) {
            if (sr) {
                if (p.mask) launch_rolled<T, true, true, false, 0, false, true>(c, nb, s, p, a, b, bits, wallg, r);
                else launch_rolled<T, true, false, false, 0, false, true>(c, nb, s, p, a, b, bits, wallg, r);
                return hipGetLastError();
            }
        }
        if (p.mask) launch_rolled<T, false, true, false, 0, false, true>(c, nb, s, p, a, b, bits, wallg, r);
        else launch_rolled<T, false, false, false, 0, false, true>(c, nb, s, p, a, b, bits, wallg, r);
        return hipGetLastError();
    }
    if (c == 0) {  // nz < 8: the unrolled kernel with a 32-plane chunk
        if (p.mask)
            k_fwd_march<T, true, 32><<<nb, NTHREADS, 0, s>>>(p, a, b, cls, bits, wallg, r);
        else
            k_fwd_march<T, false, 32><<<nb, NTHREADS, 0, s>>>(p, a, b, cls, bits, wallg, r);
    } else if (p.mask) {
        if (sr) launch_rolled_walls<T, true>(c, nb, s, p, a, b, bits, wallg, r);
        else launch_rolled_walls<T, false>(c, nb, s, p, a, b, bits, wallg, r);
    } else if (p.has_force) {
        if (sr) launch_rolled_forced<T, true, false>(c, nb, s, p, a, b, bits, wallg, r);
        else launch_rolled_forced<T, false, false>(c, nb, s, p, a, b, bits, wallg, r);
    } else if (p.split) {  // separate omega_p (no walls, nz >= 8: march_supported)
        if (sr) launch_rolled<T, true, false, true>(c, nb, s, p, a, b, bits, wallg, r);
        else launch_rolled<T, false, false, true>(c, nb, s, p, a, b, bits, wallg, r);
    } else {
        if (sr) launch_rolled<T, true, false>(c, nb, s, p, a, b, bits, wallg, r);
        else launch_rolled<T, false, false>(c, nb, s, p, a, b, bits, wallg, r);
    }
    return hipGetLastError();
}

}  // namespace

bool march_supported(const ProblemArgs &p)
{
    // 32-bit byte offsets inside a state buffer: n * 16 bytes < 4 GiB
    // a separate omega_p only on the rolled kernel without walls; forcing only
    // on the rolled kernel and not together with a separate omega_p;
    // interpolated walls and link-by-link wall velocities only with the
    // per-step wall correction (p.corr)
    const bool split_ok = !p.split || (!p.mask && p.nz >= 8);
    const bool force_ok = !p.has_force || (!p.split && p.nz >= 8);
    return p.Q == 19 && force_ok && split_ok && ((!p.qd && !p.uwl) || p.corr) && p.nx >= TX && p.ny >= TY && p.nx % TX == 0 &&
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
    const int c = rolled_nzc(p);  // the kernel dispatch() launches
    return (unsigned)march_blocks_for(p, c > 0 ? c : 32);
}

hipError_t launch_classify(const ProblemArgs &p, uint8_t *cls, unsigned *bits, float4 *wallg,
                           hipStream_t s)
{
    long long nb = (p.n + 255) / 256;
    if (nb > 4096) nb = 4096;
    k_classify<<<(unsigned)nb, 256, 0, s>>>(p, cls, bits, wallg);
    return hipGetLastError();
}

bool march_thermal_supported(const ProblemArgs &p)
{
    // halfway walls need the fixed-temperature wall table (p.T_wall)
    return march_supported(p) && (!p.mask || p.T_wall) && !p.split && !p.has_force && !p.corr &&
           !p.qd && !p.uwl && rolled_nzc(p) > 0;
}

hipError_t launch_fwd_march(const ProblemArgs &p, int storage, const void *src, void *dst,
                            const uint8_t *cls, const unsigned *bits, const float4 *wallg,
                            const ReduceArgs &r, hipStream_t s)
{
    if (!march_supported(p) || (p.mask && (!cls || !bits))) return hipErrorNotSupported;
    if (p.T_in && (!p.T_out || !march_thermal_supported(p))) return hipErrorNotSupported;
    return storage ? dispatch<__half>(p, src, dst, cls, bits, wallg, r, s)
                   : dispatch<float>(p, src, dst, cls, bits, wallg, r, s);
}

}  // namespace lwacm
