// lwacm_march.hip -- D3Q19 LW-ACM forward step as a z-marching tile kernel.
//
// Design (gfx950).  A workgroup owns a TX x TY tile of (x, y) columns and a
// chunk of NZC planes; every thread owns one column and walks up the chunk.
// For each plane it loads the node's state once (three planes in flight in
// a register ring), evaluates the node's own pre-combined link terms of
// Eq. ACM2.0b for all 19 links, and pushes them towards the columns that
// consume them.  Links are grouped by their (v_x, v_y) direction: the three
// links sharing a direction (v_z = -1, 0, +1) reach the same neighbouring
// column on three consecutive planes, so each column sums them in registers
// while marching and exchanges only two numbers per direction (density part
// and z-momentum part; the x/y momentum parts follow from the direction) plus
// one number per in-plane diagonal: 12 floats per node through LDS, instead
// of gathering 18 neighbour states.  A ring of halo columns around the tile
// is computed by extra threads in their own waves.  The receiving column
// adds the exchanged terms, its own (v_x, v_y) = (0, 0) links and the
// post-combine term a rho u (Eqs. ACM2.0b), normalises, and stores.  Forced
// problems (Eq. force) run on the generic kernel, which adds the forcing
// inside each link term where its FP32 rounding does not bias long runs.  Halfway bounce-back (Eqs. ACM2.0cbb-ACM2.0ccccbb)
// is applied at the receiving node from a precomputed per-node bit set of
// solid upstream links; solid nodes push zeros and are never written.
//
// Link terms are kept unweighted and summed with the exact integer weights
// 12, 2, 1 (= 36 w_i for rest, axis and diagonal links of D3Q19); the sums
// are divided by 36 once at the end (div36: no systematic rounding bias).
#include "lwacm_device.hpp"
#include "lwacm_internal.hpp"

namespace lwacm {

namespace {

constexpr int TX = 32;   // tile width (x, contiguous in memory)
constexpr int TY = 16;   // tile height (y)
constexpr int NZC = 32;  // planes per workgroup
constexpr int NINT = TX * TY;                 // interior columns
constexpr int NHALO = 2 * (TX + 2) + 2 * TY;  // ring of halo columns
constexpr int NTHREADS = ((NINT + NHALO + kWave - 1) / kWave) * kWave;
constexpr int SX = TX + 2;                    // LDS row pitch
constexpr int SPLANE = SX * (TY + 2);         // floats per exchanged quantity
constexpr int NQ = 12;                        // exchanged quantities per node

// Exchanged quantities (per sending column, per target plane):
enum : int {
    Q_PE = 0,  // density part of the three links with (vx,vy) = (+1, 0)
    Q_ZE,      // their z-momentum part
    Q_PW, Q_ZW,   // (-1, 0)
    Q_PN, Q_ZN,   // ( 0,+1)
    Q_PS, Q_ZS,   // ( 0,-1)
    Q_NE,      // link (+1,+1,0)
    Q_NW,      // link (-1,+1,0)
    Q_SE,      // link (+1,-1,0)
    Q_SW       // link (-1,-1,0)
};

// Per target plane accumulator of one column.
struct Acc {
    float pe, ze, pw, zw, pn, zn, ps, zs;  // direction partials (weights folded)
    float ne, nw, se, sw;                  // in-plane diagonals
    float d, jz;                           // own column: rest + (0,0,+-1) links
    float post[3];                         // a rho u of the node itself
    float lnk[19];                         // own link terms (bounce-back only)
    unsigned bits;                         // solid upstream links (bounce-back only)
    int cls;                               // 0 fluid, 1 fluid next to a wall, 2 solid
};

template <class T>
struct Ring {
    T v[4];
    uint8_t cls;
};

// Upstream-solid bit of link i in the per-node bit set (link indexing of
// lwacm_device.hpp); bit 0 is unused.
__device__ __forceinline__ bool has_bit(unsigned bits, int i) { return (bits >> i) & 1u; }

template <class T, bool MASK>
__global__ __launch_bounds__(NTHREADS) void k_fwd_march(ProblemArgs p, const T *__restrict__ src,
                                                        T *__restrict__ dst,
                                                        const uint8_t *__restrict__ cls_arr,
                                                        const unsigned *__restrict__ bb_bits,
                                                        ReduceArgs r)
{
    __shared__ float xch[2][NQ * SPLANE];

    const int tid = threadIdx.x;
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
    const int nzc = z1 - z0;

    // My column, in tile coordinates [-1, TX] x [-1, TY].
    int lx, ly;
    bool interior = tid < NINT;
    bool active = tid < NINT + NHALO;
    if (interior) {
        lx = tid % TX;
        ly = tid / TX;
    } else {
        const int h = tid - NINT;
        if (h < TX + 2) {
            ly = -1;
            lx = h - 1;
        } else if (h < 2 * (TX + 2)) {
            ly = TY;
            lx = h - (TX + 2) - 1;
        } else if (h < 2 * (TX + 2) + TY) {
            lx = -1;
            ly = h - 2 * (TX + 2);
        } else if (h < NHALO) {
            lx = TX;
            ly = h - 2 * (TX + 2) - TY;
        } else {
            lx = 0;  // padding lanes: valid address, never written to LDS
            ly = 0;
        }
    }
    int gx = tile_x * TX + lx;
    int gy = tile_y * TY + ly;
    gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
    gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
    const long long col = (long long)gy * nx + gx;
    const int slot = (ly + 1) * SX + (lx + 1);

    const float A = p.A;
    const float a = p.a;

    auto node_at_plane = [&](int pz) -> long long {
        pz = pz < 0 ? pz + nz : (pz >= nz ? pz - nz : pz);
        return (long long)pz * plane + col;
    };
    auto issue = [&](Ring<T> &rg, int pz) {
        const long long idx = node_at_plane(pz);
        rg.v[0] = src[idx];
        rg.v[1] = src[n + idx];
        rg.v[2] = src[2 * n + idx];
        rg.v[3] = src[3 * n + idx];
        if (MASK) rg.cls = cls_arr[idx];
    };

    Ring<T> ring[3];
    Acc acc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        acc[j] = Acc{};
        ring[j].cls = 0;
    }
    const int niter = nzc + 2;
    issue(ring[0], z0 - 1);
    issue(ring[1], z0);
    issue(ring[2], z0 + 1);

    float mass = 0.0f, energy = 0.0f;

    for (int k0 = 0; k0 < niter; k0 += 3) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int k = k0 + j;
            if (k >= niter) break;
            const int pz = z0 - 1 + k;  // source plane of this iteration
            Acc &A1 = acc[(j + 1) % 3];  // target plane pz + 1
            Acc &A0 = acc[j];            // target plane pz
            Acc &Am = acc[(j + 2) % 3];  // target plane pz - 1 (finalised now)

            // ---- consume the ring slot of plane pz, refill it with pz + 3
            const float dr = Storage<T>::load(ring[j].v, 0, p.ld_scale[0]);
            const float ux = Storage<T>::load(ring[j].v, 1, p.ld_scale[1]);
            const float uy = Storage<T>::load(ring[j].v, 2, p.ld_scale[1]);
            const float uz = Storage<T>::load(ring[j].v, 3, p.ld_scale[1]);
            const int cls = MASK ? (int)ring[j].cls : 0;
            if (k + 3 < niter) issue(ring[j], pz + 3);

            // ---- own link terms of plane pz, unweighted, in +-c pairs:
            // L(+-c) = E0 + 4.5 rho c^2 +- A rho c with E0 = drho - 1.5 rho |u|^2
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
                const float m = fmaf(r45 * c, c, E0);
                const float q = rA * c;
                lp = m + q;
                lm = m - q;
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

            // ---- links with v_z = +1 start the accumulator of plane pz + 1
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
            // ---- links with v_z = 0 complete the in-plane part of plane pz
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
                if (cls == 1) A0.bits = bb_bits[node_at_plane(pz)];
                A0.lnk[0] = E0;
                A0.lnk[1] = Lpx;  A0.lnk[2] = Lmx;  A0.lnk[3] = Lpy;  A0.lnk[4] = Lmy;
                A0.lnk[5] = Lpp0; A0.lnk[6] = Lmm0; A0.lnk[7] = Lpm0; A0.lnk[8] = Lmp0;
                A0.lnk[9] = Lpz;  A0.lnk[10] = Lp0p; A0.lnk[11] = Lm0p; A0.lnk[12] = L0pp;
                A0.lnk[13] = L0mp; A0.lnk[14] = Lmz; A0.lnk[15] = Lm0m; A0.lnk[16] = Lp0m;
                A0.lnk[17] = L0mm; A0.lnk[18] = L0pm;
            }
            // ---- links with v_z = -1 finish plane pz - 1
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

            if (k < 2) continue;  // planes below the chunk are halo only

            // ---- exchange the partials of plane pz - 1 through LDS
            float *X = xch[k & 1];
            if (active) {
                X[Q_PE * SPLANE + slot] = Am.pe;
                X[Q_ZE * SPLANE + slot] = Am.ze;
                X[Q_PW * SPLANE + slot] = Am.pw;
                X[Q_ZW * SPLANE + slot] = Am.zw;
                X[Q_PN * SPLANE + slot] = Am.pn;
                X[Q_ZN * SPLANE + slot] = Am.zn;
                X[Q_PS * SPLANE + slot] = Am.ps;
                X[Q_ZS * SPLANE + slot] = Am.zs;
                X[Q_NE * SPLANE + slot] = Am.ne;
                X[Q_NW * SPLANE + slot] = Am.nw;
                X[Q_SE * SPLANE + slot] = Am.se;
                X[Q_SW * SPLANE + slot] = Am.sw;
            }
            __syncthreads();
            if (!interior) continue;
            const float pE = X[Q_PE * SPLANE + slot - 1];
            const float zE = X[Q_ZE * SPLANE + slot - 1];
            const float pW = X[Q_PW * SPLANE + slot + 1];
            const float zW = X[Q_ZW * SPLANE + slot + 1];
            const float pN = X[Q_PN * SPLANE + slot - SX];
            const float zN = X[Q_ZN * SPLANE + slot - SX];
            const float pS = X[Q_PS * SPLANE + slot + SX];
            const float zS = X[Q_ZS * SPLANE + slot + SX];
            const float dNE = X[Q_NE * SPLANE + slot - SX - 1];
            const float dNW = X[Q_NW * SPLANE + slot - SX + 1];
            const float dSE = X[Q_SE * SPLANE + slot + SX - 1];
            const float dSW = X[Q_SW * SPLANE + slot + SX + 1];

            float D36 = Am.d + ((pE + pW) + (pN + pS)) + ((dNE + dNW) + (dSE + dSW));
            float Jx = (pE - pW) + ((dNE - dNW) + (dSE - dSW));
            float Jy = (pN - pS) + ((dNE + dNW) - (dSE + dSW));
            float Jz = Am.jz + ((zE + zW) + (zN + zS));
            if (MASK && Am.bits != 0u) {
                // halfway bounce-back: a solid upstream node x - v_i pushed
                // nothing; the node's own term of the opposite link returns
                // along i, plus the moving-wall term of Eq. ACM2.0ccccbb.
                const int tz = pz - 1;
#pragma unroll
                for (int i = 1; i < 19; ++i) {
                    if (has_bit(Am.bits, i)) {
                        const int cx = link_cx(i), cy = link_cy(i), cz = link_cz(i);
                        int ux_ = gx - cx, uy_ = gy - cy, uz_ = tz - cz;
                        ux_ = ux_ < 0 ? ux_ + nx : (ux_ >= nx ? ux_ - nx : ux_);
                        uy_ = uy_ < 0 ? uy_ + ny : (uy_ >= ny ? uy_ - ny : uy_);
                        uz_ = uz_ < 0 ? uz_ + nz : (uz_ >= nz ? uz_ - nz : uz_);
                        const int m = p.mask[((long long)uz_ * ny + uy_) * nx + ux_];
                        const float wt = cx * p.wall_term[m][0] + cy * p.wall_term[m][1] +
                                         cz * p.wall_term[m][2];
                        const float wi36 = (i <= 4 || i == 9 || i == 14) ? 2.0f : 1.0f;
                        const float s = wi36 * (Am.lnk[link_opp(i)] + wt);
                        D36 += s;
                        Jx = fmaf((float)cx, s, Jx);
                        Jy = fmaf((float)cy, s, Jy);
                        Jz = fmaf((float)cz, s, Jz);
                    }
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
                const long long idx = (long long)(pz - 1) * plane + col;
                Storage<T>::store(dst, idx, D, p.st_scale[0]);
                Storage<T>::store(dst, n + idx, vx, p.st_scale[1]);
                Storage<T>::store(dst, 2 * n + idx, vy, p.st_scale[1]);
                Storage<T>::store(dst, 3 * n + idx, vz, p.st_scale[1]);
                mass += D;
                energy = fmaf(vx, vx, fmaf(vy, vy, fmaf(vz, vz, energy)));
            }
        }
    }

    double v[2] = {(double)mass, 0.5 * (double)energy};
    double tot[2];
    if (grid_sum_last_block<2>(v, r.partials, r.counter, gridDim.x, blockIdx.x, tot) &&
        threadIdx.x == 0) {
        r.out[0] = tot[0];
        r.out[1] = tot[1];
        if (r.out2) {
            r.out2[0] = tot[0];
            r.out2[1] = tot[1];
        }
    }
}

// Node classes and solid-upstream bit sets for the bounce-back of the march
// kernel: class 0 fluid with only fluid upstream nodes, 1 fluid with at
// least one solid upstream node (bit i set when x - v_i is solid), 2 solid.
__global__ __launch_bounds__(256) void k_classify(ProblemArgs p, uint8_t *cls, unsigned *bits)
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
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            int ux = x - link_cx(i), uy = y - link_cy(i), uz = z - link_cz(i);
            ux = ux < 0 ? ux + p.nx : (ux >= p.nx ? ux - p.nx : ux);
            uy = uy < 0 ? uy + p.ny : (uy >= p.ny ? uy - p.ny : uy);
            uz = uz < 0 ? uz + p.nz : (uz >= p.nz ? uz - p.nz : uz);
            if (p.mask[((long long)uz * p.ny + uy) * p.nx + ux] != 0) bb |= 1u << i;
        }
        cls[idx] = bb ? 1 : 0;
        bits[idx] = bb;
    }
}

template <class T>
hipError_t dispatch(const ProblemArgs &p, const void *src, void *dst, const uint8_t *cls,
                    const unsigned *bits, const ReduceArgs &r, hipStream_t s)
{
    const unsigned nb = march_num_blocks(p);
    const T *a = static_cast<const T *>(src);
    T *b = static_cast<T *>(dst);
    if (p.mask)
        k_fwd_march<T, true><<<nb, NTHREADS, 0, s>>>(p, a, b, cls, bits, r);
    else
        k_fwd_march<T, false><<<nb, NTHREADS, 0, s>>>(p, a, b, cls, bits, r);
    return hipGetLastError();
}

}  // namespace

bool march_supported(const ProblemArgs &p)
{
    return p.Q == 19 && !p.has_force && p.nx >= TX && p.ny >= TY && p.nx % TX == 0 &&
           p.ny % TY == 0 && p.nz >= 1 && (long long)p.nx * p.ny < (1LL << 31);
}

unsigned march_num_blocks(const ProblemArgs &p)
{
    if (!march_supported(p)) return 0;
    const long long tiles = (long long)(p.nx / TX) * (p.ny / TY);
    const long long chunks = (p.nz + NZC - 1) / NZC;
    return (unsigned)(tiles * chunks);
}

hipError_t launch_classify(const ProblemArgs &p, uint8_t *cls, unsigned *bits, hipStream_t s)
{
    long long nb = (p.n + 255) / 256;
    if (nb > 4096) nb = 4096;
    k_classify<<<(unsigned)nb, 256, 0, s>>>(p, cls, bits);
    return hipGetLastError();
}

hipError_t launch_fwd_march(const ProblemArgs &p, int storage, const void *src, void *dst,
                            const uint8_t *cls, const unsigned *bits, const ReduceArgs &r,
                            hipStream_t s)
{
    if (!march_supported(p) || (p.mask && (!cls || !bits))) return hipErrorNotSupported;
    return storage ? dispatch<__half>(p, src, dst, cls, bits, r, s)
                   : dispatch<float>(p, src, dst, cls, bits, r, s);
}

}  // namespace lwacm
