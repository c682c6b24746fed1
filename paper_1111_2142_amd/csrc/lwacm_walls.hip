// lwacm_walls.hip -- the fluid nodes next to a wall, and what is done on
// them alone: the list itself, the per-step correction that carries the
// interpolated bounce-back of Eq. ACM2.0cc and the link-by-link wall motion
// of Eq. ACM2.0move into the D3Q19 tile kernel, and the momentum-exchange
// force and torque of Eqs. MEA3-MEA5 (the set S of Eq. MEA4: the links from
// these nodes into a body).
//
// List.  A fluid node x belongs to it when some x + v_j (equivalently some
// x - v_i: the link set is symmetric) is solid.  Built once per context in
// node order by three launches (count per block of 256 nodes, one-block
// exclusive scan of the counts, scatter), so the order, and every sum taken
// over the list in a fixed grid, is reproducible.
//
// Correction.  The link data that stay fixed with the walls (q of each wall
// link, and whether the q < 1/2 rule finds a fluid second node) are packed
// once per context, link-major, so a step reads them contiguously.  For
// every incoming link i whose upstream node x - v_i is solid, the halfway
// rule (Eq. ACM2.0ccbb) returns the node's own term of the opposite link ib;
// the interpolated rule replaces it by 2q L_ib(x) + (1 - 2q) L_ib(x - v_ib)
// (q < 1/2, where x - v_ib is fluid) or L_ib(x)/(2q) + (1 - 1/(2q)) L_i(x)
// (q >= 1/2), and scales the moving-wall term (2/omega - 1) 2 f^(e,o)(rho0,
// u_w) by 1/(2q) for q >= 1/2 (Eq. ACM2.0move).  Per node this kernel sums
// these terms, moving wall included, with the integer weights 36 w_i into
// (1, v_i): one float4 that the tile kernel adds before normalisation in
// place of its own bounce-back sums, which it skips for such problems.  The
// forcing term is not in it: the tile kernel adds rho g as a whole.
#include "lwacm_device.hpp"
#include "lwacm_internal.hpp"
#include "lwacm_march_common.hpp"
#include "lwacm_walls.hpp"

namespace lwacm {

namespace {

constexpr unsigned kListBlock = 256;

__device__ __forceinline__ int wrap1(int a, int n)
{
    return a < 0 ? a + n : (a >= n ? a - n : a);
}

// Does fluid node idx have a solid node among its Q - 1 link neighbours?
template <int Q>
__device__ __forceinline__ bool next_to_wall(const ProblemArgs &p, long long idx)
{
    if (p.mask[idx] != 0) return false;
    const long long t = idx / p.nx;
    const int x = (int)(idx - t * p.nx);
    const int z = (int)(t / p.ny);
    const int y = (int)(t - (long long)z * p.ny);
    bool any = false;
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        const long long nb = ((long long)wrap1(z + link_cz(j), p.nz) * p.ny +
                              wrap1(y + link_cy(j), p.ny)) * p.nx + wrap1(x + link_cx(j), p.nx);
        any = any || p.mask[nb] != 0;
    }
    return any;
}

template <int Q>
__global__ __launch_bounds__(kListBlock) void k_list_count(ProblemArgs p, unsigned *counts)
{
    const long long idx = (long long)blockIdx.x * kListBlock + threadIdx.x;
    const bool in = idx < p.n && next_to_wall<Q>(p, idx);
    const int c = __syncthreads_count(in);
    if (threadIdx.x == 0) counts[blockIdx.x] = (unsigned)c;
}

// Exclusive scan of nb counts in place, total in *total.  One block: each
// thread adds a contiguous run of counts, the runs' sums are scanned in LDS,
// then each thread writes its run's offsets.
constexpr unsigned kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_list_scan(unsigned *counts, unsigned nb,
                                                            unsigned long long *total)
{
    __shared__ unsigned long long part[kScanThreads];
    const unsigned per = (nb + kScanThreads - 1) / kScanThreads;
    const unsigned b0 = threadIdx.x * per;
    const unsigned b1 = min(nb, b0 + per);
    unsigned long long s = 0;
    for (unsigned b = b0; b < b1; ++b) s += counts[b];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the run sums
    for (unsigned off = 1; off < kScanThreads; off <<= 1) {
        const unsigned long long v = threadIdx.x >= off ? part[threadIdx.x - off] : 0ull;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    unsigned long long run = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
    for (unsigned b = b0; b < b1; ++b) {
        const unsigned c = counts[b];
        counts[b] = (unsigned)run;
        run += c;
    }
    if (threadIdx.x == kScanThreads - 1) *total = part[kScanThreads - 1];
}

template <int Q>
__global__ __launch_bounds__(kListBlock) void k_list_scatter(ProblemArgs p, const unsigned *offsets,
                                                             unsigned *list)
{
    __shared__ unsigned wave_count[kListBlock / kWave];
    const long long idx = (long long)blockIdx.x * kListBlock + threadIdx.x;
    const bool in = idx < p.n && next_to_wall<Q>(p, idx);
    const unsigned long long ball = __builtin_amdgcn_ballot_w64(in);
    const unsigned lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const unsigned below = (unsigned)__builtin_popcountll(ball & ((1ull << lane) - 1ull));
    if (lane == 0) wave_count[wave] = (unsigned)__builtin_popcountll(ball);
    __syncthreads();
    unsigned base = offsets[blockIdx.x];
    for (unsigned w = 0; w < wave; ++w) base += wave_count[w];
    if (in) list[base + below] = (unsigned)idx;
}

template <class T>
__device__ __forceinline__ void load_node(const T *s, long long idx, const ProblemArgs &p,
                                          float &dr, float (&u)[3])
{
    float v[4];
    NodeState<T, 4>::load(s, idx, p.ld_scale, v);
    dr = v[0];
    u[0] = v[1];
    u[1] = v[2];
    u[2] = v[3];
}

__device__ __forceinline__ float vdot19(int i, const float (&u)[3])
{
    return (float)link_cx(i) * u[0] + (float)link_cy(i) * u[1] + (float)link_cz(i) * u[2];
}

// Link data of the listed nodes that stays fixed with the walls, packed
// once: the link-wall distance of every incoming link i whose upstream node
// x - v_i is solid (q of the outgoing link opp(i), link-major: qc[(i - 1) *
// nlist + k], 1/2 without d_q), and a bit per link that the q < 1/2 rule
// takes the fluid node x - v_opp(i) = x + v_i (else it falls back to the
// halfway term), and the node's set of solid upstream links (bit i: x - v_i
// solid), so that a step reads nothing per node but the state.
__global__ __launch_bounds__(256) void k_wall_pack(ProblemArgs p, const unsigned *__restrict__ list,
                                                   unsigned nlist, float *__restrict__ qc,
                                                   unsigned *__restrict__ second,
                                                   unsigned *__restrict__ wbits)
{
    const long long n = p.n;
    for (unsigned k = blockIdx.x * blockDim.x + threadIdx.x; k < nlist;
         k += gridDim.x * blockDim.x) {
        const long long idx = list[k];
        const long long t = idx / p.nx;
        const int x = (int)(idx - t * p.nx);
        const int z = (int)(t / p.ny);
        const int y = (int)(t - (long long)z * p.ny);
        unsigned sec = 0u, bb = 0u;
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            const int cx = link_cx(i), cy = link_cy(i), cz = link_cz(i);
            const long long up = ((long long)wrap1(z - cz, p.nz) * p.ny + wrap1(y - cy, p.ny)) * p.nx +
                                 wrap1(x - cx, p.nx);
            float qv = 0.5f;
            if (p.mask[up] != 0) bb |= 1u << i;
            if (p.mask[up] != 0 && p.qd) {
                qv = p.qd[(long long)link_opp(i) * n + idx];
                const long long dn = ((long long)wrap1(z + cz, p.nz) * p.ny + wrap1(y + cy, p.ny)) *
                                         p.nx + wrap1(x + cx, p.nx);
                if (qv < 0.5f && p.mask[dn] == 0) sec |= 1u << i;
            }
            qc[(long long)(i - 1) * nlist + k] = qv;
        }
        second[k] = sec;
        wbits[k] = bb;
    }
}

// Four lanes per listed node: lane s of a node's group takes the links
// i = 1 + s, 5 + s, 9 + s, 13 + s, 17 + s (up to 18), so a node's wall links
// spread over four lanes and each lane keeps few loads in flight.  A lane
// issues the loads of all its links (q of each wall link, the second node of
// each link the q < 1/2 rule takes) before it uses any, as buffer loads whose
// offset lies past the end of the buffer where a link does not need them
// (such a load returns zeros and touches no memory).  The four partial sums
// are added across the group in a fixed order (xor 1, then xor 2), and the
// group's first lane stores the node's correction.
constexpr int kLanesPerNode = 4;
constexpr int kLinksPerLane = 5;

// Link i's velocity components and opposite, from packed constants (the
// link index is a run-time value here): cx + 1, cy + 1, cz + 1 in two bits
// each, the opposite in five.
__device__ __forceinline__ void link_of(int i, int &cx, int &cy, int &cz, int &ib)
{
    constexpr unsigned long long kx = []() {
        unsigned long long v = 0;
        for (int j = 0; j < 19; ++j) v |= (unsigned long long)(link_cx(j) + 1) << (2 * j);
        return v;
    }();
    constexpr unsigned long long ky = []() {
        unsigned long long v = 0;
        for (int j = 0; j < 19; ++j) v |= (unsigned long long)(link_cy(j) + 1) << (2 * j);
        return v;
    }();
    constexpr unsigned long long kz = []() {
        unsigned long long v = 0;
        for (int j = 0; j < 19; ++j) v |= (unsigned long long)(link_cz(j) + 1) << (2 * j);
        return v;
    }();
    constexpr unsigned long long ko_lo = []() {  // links 0..11
        unsigned long long v = 0;
        for (int j = 0; j < 12; ++j) v |= (unsigned long long)link_opp(j) << (5 * j);
        return v;
    }();
    constexpr unsigned long long ko_hi = []() {  // links 12..18
        unsigned long long v = 0;
        for (int j = 12; j < 19; ++j) v |= (unsigned long long)link_opp(j) << (5 * (j - 12));
        return v;
    }();
    cx = (int)((kx >> (2 * i)) & 3u) - 1;
    cy = (int)((ky >> (2 * i)) & 3u) - 1;
    cz = (int)((kz >> (2 * i)) & 3u) - 1;
    ib = (int)(((i < 12 ? ko_lo >> (5 * i) : ko_hi >> (5 * (i - 12)))) & 31u);
}

template <class T>
__global__ __launch_bounds__(256) void k_wall_correction(ProblemArgs p, const T *__restrict__ src,
                                                         const unsigned *__restrict__ list,
                                                         unsigned nlist,
                                                         const unsigned *__restrict__ bits,
                                                         const float *__restrict__ qc,
                                                         const unsigned *__restrict__ second,
                                                         int table_moving, float4 *__restrict__ corr)
{
    constexpr unsigned NB = BufIO<T>::kNodeBytes;
    constexpr unsigned OOB = 0xfffffff0u;  // past the end of every buffer here
    // 32-bit node arithmetic: the tile kernels run problems of n < 2^28 nodes
    const unsigned n = (unsigned)p.n, nx = (unsigned)p.nx, ny = (unsigned)p.ny;
    const unsigned plane = nx * ny;
    const Rsrc rs = make_rsrc(src, (unsigned long long)n * NB);
    const Rsrc rq = make_rsrc(qc, 18ull * nlist * 4u);
    const unsigned total = nlist * (unsigned)kLanesPerNode;
    const unsigned stride = gridDim.x * blockDim.x;  // a multiple of 4: groups stay aligned
    for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
        const unsigned k = g / kLanesPerNode;
        const int sub = (int)(g % kLanesPerNode);
        const unsigned idx = list[k];
        const unsigned bb = bits[k];  // bit i: x - v_i solid (packed per entry)
        const unsigned sec = second[k];
        const unsigned t = idx / nx;
        const int x = (int)(idx - t * nx);
        const int z = (int)(t / ny);
        const int y = (int)(t - (unsigned)z * ny);
        const unsigned xo[3] = {(unsigned)wrap1(x - 1, p.nx), (unsigned)x, (unsigned)wrap1(x + 1, p.nx)};
        const unsigned yo[3] = {(unsigned)wrap1(y - 1, p.ny) * nx, (unsigned)y * nx,
                                (unsigned)wrap1(y + 1, p.ny) * nx};
        const unsigned zo[3] = {(unsigned)wrap1(z - 1, p.nz) * plane, (unsigned)z * plane,
                                (unsigned)wrap1(z + 1, p.nz) * plane};
        const typename BufIO<T>::Raw own = BufIO<T>::load(rs, idx * NB, 0u);
        float qv[kLinksPerLane];
        typename BufIO<T>::Raw zr[kLinksPerLane];
#pragma unroll
        for (int s = 0; s < kLinksPerLane; ++s) {
            const int i = 1 + sub + kLanesPerNode * s;
            int cx, cy, cz, ib;
            link_of(i < 19 ? i : 0, cx, cy, cz, ib);
            const bool set = i < 19 && ((bb >> i) & 1u);
            const bool two = i < 19 && ((sec >> i) & 1u);
            qv[s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                  rq, set ? ((unsigned)(i - 1) * nlist + k) * 4u : OOB,
                                                  0u, 0));
            const unsigned dn = zo[1 + cz] + yo[1 + cy] + xo[1 + cx];  // x + v_i
            zr[s] = BufIO<T>::load(rs, two ? dn * NB : OOB, 0u);
        }
        const float dr = BufIO<T>::value(own, 0, p.ld_scale[0]);
        const float u[3] = {BufIO<T>::value(own, 1, p.ld_scale[1]),
                            BufIO<T>::value(own, 2, p.ld_scale[1]),
                            BufIO<T>::value(own, 3, p.ld_scale[1])};
        const float rho = 1.0f + dr;
        const float B = -1.5f * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f;
#pragma unroll
        for (int s = 0; s < kLinksPerLane; ++s) {
            const int i = 1 + sub + kLanesPerNode * s;
            int cx, cy, cz, ib;
            link_of(i < 19 ? i : 0, cx, cy, cz, ib);
            const bool set = i < 19 && ((bb >> i) & 1u);
            const float c = cx * u[0] + cy * u[1] + cz * u[2];  // v_i . u
            const float hw = link_term_unweighted(dr, rho, -c, B, p.A);
            float sb = hw, wsc = 1.0f;
            if (i < 19 && ((sec >> i) & 1u)) {
                // q < 1/2 with the fluid node x - v_ib = x + v_i
                const float dz = BufIO<T>::value(zr[s], 0, p.ld_scale[0]);
                const float uz[3] = {BufIO<T>::value(zr[s], 1, p.ld_scale[1]),
                                     BufIO<T>::value(zr[s], 2, p.ld_scale[1]),
                                     BufIO<T>::value(zr[s], 3, p.ld_scale[1])};
                const float Bz = -1.5f * (uz[0] * uz[0] + uz[1] * uz[1] + uz[2] * uz[2]);
                const float cz2 = cx * uz[0] + cy * uz[1] + cz * uz[2];
                const float sz = link_term_unweighted(dz, 1.0f + dz, -cz2, Bz, p.A);
                sb = fmaf(2.0f * qv[s], hw, (1.0f - 2.0f * qv[s]) * sz);
            } else if (qv[s] >= 0.5f) {
                const float si = link_term_unweighted(dr, rho, c, B, p.A);
                const float h = 0.5f / qv[s];
                sb = fmaf(h, hw, (1.0f - h) * si);
                wsc = h;
            }
            // the wall's velocity: per link when given so, else the id table's
            float uw[3] = {0.0f, 0.0f, 0.0f};
            if (p.uwl) {
                if (set)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc)
                        uw[cc] = p.wall_scale * p.uwl[((unsigned long long)ib * 3u + (unsigned)cc) * n + idx];
            } else if (table_moving && set) {
                const int m = p.mask[zo[1 - cz] + yo[1 - cy] + xo[1 - cx]];  // x - v_i
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) uw[cc] = p.wall_term[m][cc];
            }
            const float w36 = (i <= 4 || i == 9 || i == 14) ? 2.0f : 1.0f;
            const float d = set ? w36 * fmaf(wsc, cx * uw[0] + cy * uw[1] + cz * uw[2], sb) : 0.0f;
            c0 += d;
            c1 = fmaf((float)cx, d, c1);
            c2 = fmaf((float)cy, d, c2);
            c3 = fmaf((float)cz, d, c3);
        }
        // the group's four partial sums, added in a fixed order
        c0 += __shfl_xor(c0, 1);
        c1 += __shfl_xor(c1, 1);
        c2 += __shfl_xor(c2, 1);
        c3 += __shfl_xor(c3, 1);
        c0 += __shfl_xor(c0, 2);
        c1 += __shfl_xor(c1, 2);
        c2 += __shfl_xor(c2, 2);
        c3 += __shfl_xor(c3, 2);
        if (sub == 0) corr[idx] = make_float4(c0, c1, c2, c3);
    }
}

}  // namespace

size_t wall_list_count_blocks(long long n)
{
    return (size_t)((n + kListBlock - 1) / kListBlock);
}

hipError_t launch_wall_list_count(const ProblemArgs &p, unsigned *counts,
                                  unsigned long long *d_total, hipStream_t s)
{
    const size_t nb = wall_list_count_blocks(p.n);
    if (!p.mask || nb == 0 || nb > 0xffffffffull) return hipErrorInvalidValue;
    if (p.Q == 19)
        k_list_count<19><<<(unsigned)nb, kListBlock, 0, s>>>(p, counts);
    else
        k_list_count<9><<<(unsigned)nb, kListBlock, 0, s>>>(p, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_list_scan<<<1, kScanThreads, 0, s>>>(counts, (unsigned)nb, d_total);
    return hipGetLastError();
}

hipError_t launch_wall_list_scatter(const ProblemArgs &p, const unsigned *offsets,
                                    unsigned *list, hipStream_t s)
{
    const size_t nb = wall_list_count_blocks(p.n);
    if (!p.mask || nb == 0) return hipErrorInvalidValue;
    if (p.Q == 19)
        k_list_scatter<19><<<(unsigned)nb, kListBlock, 0, s>>>(p, offsets, list);
    else
        k_list_scatter<9><<<(unsigned)nb, kListBlock, 0, s>>>(p, offsets, list);
    return hipGetLastError();
}

hipError_t launch_wall_pack(const ProblemArgs &p, const unsigned *list, unsigned nlist, float *qc,
                            unsigned *second, unsigned *wbits, hipStream_t s)
{
    if (p.Q != 19 || !p.mask) return hipErrorInvalidValue;
    if (nlist == 0) return hipSuccess;
    unsigned nb = (nlist + 255) / 256;
    if (nb > 4096) nb = 4096;
    k_wall_pack<<<nb, 256, 0, s>>>(p, list, nlist, qc, second, wbits);
    return hipGetLastError();
}

hipError_t launch_wall_correction(const ProblemArgs &p, int storage, const void *src,
                                  const WallLinks &w, float4 *corr, hipStream_t s)
{
    if (p.Q != 19 || !p.mask || !corr || !w.bits || !w.qc || !w.second) return hipErrorInvalidValue;
    if (w.nlist == 0) return hipSuccess;
    if (w.nlist > 0xffffffffu / kLanesPerNode) return hipErrorInvalidValue;
    unsigned nb = (w.nlist * kLanesPerNode + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (storage)
        k_wall_correction<__half><<<nb, 256, 0, s>>>(p, static_cast<const __half *>(src), w.list,
                                                      w.nlist, w.bits, w.qc, w.second,
                                                      w.table_moving, corr);
    else
        k_wall_correction<float><<<nb, 256, 0, s>>>(p, static_cast<const float *>(src), w.list,
                                                     w.nlist, w.bits, w.qc, w.second,
                                                     w.table_moving, corr);
    return hipGetLastError();
}

}  // namespace lwacm
