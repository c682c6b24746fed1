// lwacm_api.hip -- the C ABI declared in include/lwacm.h: argument checks,
// context and scratch management, buffer toggling and kernel dispatch.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "lwacm.h"
#include "lwacm_internal.hpp"
#include "lwacm_thermal.hpp"
#include "lwacm_force.hpp"
#include "lwacm_walls.hpp"

using lwacm::ProblemArgs;
using lwacm::ReduceArgs;

struct lwacm_ctx {
    ProblemArgs p;
    int lattice;
    int storage;
    int variant;  // requested LWACM_KERNEL_*
    bool force;
    double omega;
    double omega_p;  // relaxation of the density update (== omega: single relaxation)
    double a_exact;  // the a used by the kernels (1 - quantised h), as a double
    double rho0;
    void *buf[2];
    int cur;
    float wall_u[lwacm::kMaxWallIds][3];
    int n_wall_ids;
    int k_rho, k_u;
    uint32_t sr_seed;
    hipStream_t stream;
    double *d_partials;
    size_t n_partial_blocks;
    double *d_diag;     // [2] mass deviation, energy of the last step's output
    double *d_scratch;  // [2] for lwacm_moments
    unsigned *d_scan;   // [2] mask scan
    uint8_t *d_cls;     // node classes for the march kernel (masked problems)
    unsigned *d_bits;   // solid-upstream link bits for the march kernel
    float4 *d_wallg;    // moving-wall geometry sums for the march kernel (moving walls only)
    double *d_hist;
    int hist_cap;
    long long steps;
    bool diag_valid;
    unsigned long long n_fluid;
    // temperature lattice (lwacm_set_thermal): two caller-owned buffers
    bool thermal;
    int thermal_qt;  // temperature lattice (lwacm_set_thermal_lattice): 0 = the flow's
    uint2 *d_twall;  // fixed-temperature wall links per node (fused step with walls)
    float *T_buf[2];
    int tcur;
    lwacm::ThermalArgs targs;
    double *d_force;  // wall-force partials (allocated on first use)
    // reverse sweeps (lwacm_adjoint_sweep): the steps' block partials and
    // totals, allocated on first use and grown as needed (doubles)
    double *d_sweep;
    size_t sweep_cap;
    double *h_force;  // pinned host memory the wall-force sum kernel writes its six results to
    // fluid nodes next to a wall, in node order (built on first use)
    unsigned *d_wlist;
    unsigned n_wlist;
    bool wlist_built;
    float4 *d_corr;   // per-step wall correction of the tile kernels (interpolated walls)
    float *d_wqc;     // packed q of the listed nodes' wall links (18 per node, link-major)
    unsigned *d_wsec; // per listed node: links whose q < 1/2 rule takes the second node
    unsigned *d_wbits; // per listed node: its solid upstream links
    bool semi_implicit;  // pressure from the updated velocity (Eq. FDcompact_si)
};

namespace {

int dev_err(hipError_t e)
{
    return e == hipSuccess ? LWACM_OK : LWACM_EDEVICE;
}

// h = 2/omega - 1 rounded to a multiple of the finest power of two q for
// which 1 - h and 3 h are both FP32 numbers, so that a = 1 - h and A = 3 h
// hold exactly and a + A/3 = 1 (the link terms then conserve momentum to
// rounding; a mismatch of ~1e-8 would act like a source term every step).
// The quantum follows the FP32 spacing of 3 h and of 1 - h: 2^-24 or 2^-23
// for 1 <= omega < 2, coarser for omega < 1 where h > 1.  h moves by at most
// q / 2, a relative change of nu = h/6 of at most q / (2 h).
double quantised_h(double omega)
{
    const double h = 2.0 / omega - 1.0;
    for (int e = -40; e <= 8; ++e) {
        const double q = ldexp(1.0, e);
        const double hq = nearbyint(h / q) * q;
        if ((double)(float)(1.0 - hq) == 1.0 - hq && (double)(float)(3.0 * hq) == 3.0 * hq)
            return hq;
    }
    return h;  // not reached for 0 < omega < 2
}

void set_wall_terms(lwacm_ctx *c)
{
    const float a = c->p.a;
    const double hp = c->p.Ap / 3.0;  // 2/omega_p - 1 (exact: Ap = 3 hp in FP32)
    for (int m = 0; m < lwacm::kMaxWallIds; ++m)
        for (int k = 0; k < 3; ++k) {
            const double uw = (m < c->n_wall_ids) ? c->wall_u[m][k] : 0.0;
            c->p.wall_da[m][k] = (float)(6.0 * c->rho0 * uw);
            c->p.wall_term[m][k] = (float)((1.0 - a) * 6.0 * c->rho0 * uw);
            c->p.wall_term_p[m][k] = (float)(hp * 6.0 * c->rho0 * uw);
            c->p.wall_u[m][k] = (float)uw;
        }
    c->p.wall_scale = (float)((1.0 - a) * 6.0 * c->rho0);
    c->p.wall6rho0 = (float)(6.0 * c->rho0);
}

void set_scales(lwacm_ctx *c)
{
    if (c->storage == LWACM_FP16_DEV) {
        c->p.st_scale[0] = ldexpf(1.0f, c->k_rho);
        c->p.st_scale[1] = ldexpf(1.0f, c->k_u);
        c->p.ld_scale[0] = ldexpf(1.0f, -c->k_rho);
        c->p.ld_scale[1] = ldexpf(1.0f, -c->k_u);
    } else {
        c->p.st_scale[0] = c->p.st_scale[1] = 1.0f;
        c->p.ld_scale[0] = c->p.ld_scale[1] = 1.0f;
    }
}

ReduceArgs reduce_args(lwacm_ctx *c, double *out, double *out2)
{
    ReduceArgs r;
    r.partials = c->d_partials;
    r.prev_partials = nullptr;
    r.prev_nblocks = 0;
    r.prev_out = r.prev_out2 = nullptr;
    r.partials_b = nullptr;
    r.prev_partials_b = nullptr;
    r.prev_nblocks_b = 0;
    r.prev_out_b = r.prev_out2_b = nullptr;
    r.out = out;
    r.out2 = out2;
    r.accumulate = 0;
    r.out_scale = 1.0;
    return r;
}

size_t state_bytes(const lwacm_ctx *c)
{
    return (size_t)(c->p.D + 1) * (size_t)c->p.n * (c->storage == LWACM_FP32 ? 4 : 2);
}

// Several D2Q9 steps per launch in LDS (lwacm_d2q9_multi.hip): FP32, no
// history (it sums only a launch's last step), variant AUTO.
bool use_multi(const lwacm_ctx *c)
{
    return c->variant == LWACM_KERNEL_AUTO && c->storage == LWACM_FP32 && !c->thermal &&
           !c->semi_implicit && !c->d_hist && lwacm::d2q9_multi_supported(c->p) &&
           lwacm::d2q9_multi_num_blocks(c->p) <= c->n_partial_blocks;
}

bool use_march(const lwacm_ctx *c)
{
    if (c->variant == LWACM_KERNEL_GENERIC || c->semi_implicit) return false;
    return lwacm::march_supported(c->p);
}

// Two steps per launch: FP32 state, AUTO or MARCH2 selection.
bool use_march2(const lwacm_ctx *c)
{
    if (c->variant != LWACM_KERNEL_AUTO && c->variant != LWACM_KERNEL_MARCH2) return false;
    return c->storage == LWACM_FP32 && !c->thermal && lwacm::march2_supported(c->p);
}

double *hist_slot(lwacm_ctx *c, long long step)
{
    return c->d_hist ? c->d_hist + 2 * (size_t)(step % c->hist_cap) : nullptr;
}

void free_scratch(lwacm_ctx *c)
{
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_diag) (void)hipFree(c->d_diag);
    if (c->d_scratch) (void)hipFree(c->d_scratch);
    if (c->d_scan) (void)hipFree(c->d_scan);
    if (c->d_cls) (void)hipFree(c->d_cls);
    if (c->d_bits) (void)hipFree(c->d_bits);
    if (c->d_wallg) (void)hipFree(c->d_wallg);
    if (c->d_force) (void)hipFree(c->d_force);
    if (c->d_sweep) (void)hipFree(c->d_sweep);
    c->d_sweep = nullptr;
    c->sweep_cap = 0;
    if (c->h_force) (void)hipHostFree(c->h_force);
    c->h_force = nullptr;
    if (c->d_wlist) (void)hipFree(c->d_wlist);
    if (c->d_corr) (void)hipFree(c->d_corr);
    if (c->d_wqc) (void)hipFree(c->d_wqc);
    if (c->d_wsec) (void)hipFree(c->d_wsec);
    if (c->d_wbits) (void)hipFree(c->d_wbits);
    c->d_wbits = nullptr;
    if (c->d_twall) (void)hipFree(c->d_twall);
    c->d_twall = nullptr;
    c->p.T_wall = nullptr;
    c->d_wqc = nullptr;
    c->d_wsec = nullptr;
    c->d_wlist = nullptr;
    c->d_corr = nullptr;
    c->p.corr = nullptr;
    c->wlist_built = false;
    c->d_force = nullptr;
    c->d_cls = nullptr;
    c->d_bits = nullptr;
    c->d_wallg = nullptr;
    c->d_partials = nullptr;
    c->d_diag = c->d_scratch = nullptr;
    c->d_scan = nullptr;
}

// The list of fluid nodes next to a wall (lwacm_walls.hip), built once:
// counts per block, their scan, the total read back (one synchronisation),
// then the scatter.  Masked problems with fewer than 2^32 nodes.
int ensure_wall_list(lwacm_ctx *c)
{
    if (c->wlist_built) return LWACM_OK;
    if (!c->p.mask || c->p.n >= (1LL << 32)) return LWACM_EUNSUPPORTED;
    const size_t nb = lwacm::wall_list_count_blocks(c->p.n);
    unsigned *counts = nullptr;
    unsigned long long *d_total = nullptr, total = 0;
    hipError_t e = hipMalloc(&counts, nb * sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc(&d_total, sizeof(unsigned long long));
    if (e != hipSuccess) {
        if (counts) (void)hipFree(counts);
        return LWACM_ENOMEM;
    }
    e = lwacm::launch_wall_list_count(c->p, counts, d_total, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&total, d_total, sizeof(total), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMalloc(&c->d_wlist, (total ? total : 1) * sizeof(unsigned));
    if (e == hipSuccess) e = lwacm::launch_wall_list_scatter(c->p, counts, c->d_wlist, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(counts);
    (void)hipFree(d_total);
    if (e != hipSuccess) {
        if (c->d_wlist) (void)hipFree(c->d_wlist);
        c->d_wlist = nullptr;
        return LWACM_EDEVICE;
    }
    c->n_wlist = (unsigned)total;
    c->wlist_built = true;
    return LWACM_OK;
}

// Interpolated walls or link velocities on the D3Q19 tile kernels: the wall
// list and one float4 per node for the per-step correction.  Returns OK and
// leaves p.corr unset where the tile kernels cannot take the problem (the
// generic kernel then runs it).
int enable_wall_correction(lwacm_ctx *c)
{
    ProblemArgs g = c->p;  // the tile kernels' own conditions, walls aside
    g.qd = nullptr;
    g.uwl = nullptr;
    g.corr = nullptr;
    if (!c->p.mask || !c->d_bits || !lwacm::march_supported(g)) return LWACM_OK;
    const int rc = ensure_wall_list(c);
    if (rc != LWACM_OK) return rc == LWACM_EUNSUPPORTED ? LWACM_OK : rc;
    // the correction kernel addresses the packed q (18 per listed node) and
    // the link velocities (57 fields) with 32-bit byte offsets
    if (72ull * c->n_wlist >= (1ull << 32) || (c->p.uwl && 228ull * c->p.n >= (1ull << 32)))
        return LWACM_OK;
    if (!c->d_corr) {
        const size_t nl = c->n_wlist ? c->n_wlist : 1;
        if (hipMalloc(&c->d_corr, (size_t)c->p.n * sizeof(float4)) != hipSuccess ||
            hipMalloc(&c->d_wqc, 18 * nl * sizeof(float)) != hipSuccess ||
            hipMalloc(&c->d_wsec, nl * sizeof(unsigned)) != hipSuccess ||
            hipMalloc(&c->d_wbits, nl * sizeof(unsigned)) != hipSuccess) {
            if (c->d_corr) (void)hipFree(c->d_corr);
            if (c->d_wqc) (void)hipFree(c->d_wqc);
            if (c->d_wsec) (void)hipFree(c->d_wsec);
            c->d_corr = nullptr;
            c->d_wqc = nullptr;
            c->d_wsec = nullptr;
            c->d_wbits = nullptr;
            return LWACM_ENOMEM;
        }
        // q, the second-node choice and the link sets are fixed with the
        // walls: packed once
        if (lwacm::launch_wall_pack(c->p, c->d_wlist, c->n_wlist, c->d_wqc, c->d_wsec,
                                    c->d_wbits, c->stream) != hipSuccess)
            return LWACM_EDEVICE;
    }
    c->p.corr = c->d_corr;
    return LWACM_OK;
}

lwacm::WallLinks wall_links(const lwacm_ctx *c)
{
    lwacm::WallLinks w;
    w.list = c->d_wlist;
    w.nlist = c->n_wlist;
    w.bits = c->d_wbits;
    w.qc = c->d_wqc;
    w.second = c->d_wsec;
    w.table_moving = 0;
    for (int m = 1; m < c->n_wall_ids; ++m)
        for (int k = 0; k < 3; ++k) w.table_moving |= c->wall_u[m][k] != 0.0f;
    return w;
}

}  // namespace

// Fixed scratch of lwacm_step_static: the per-block FP64 partial sums of the
// forward steps (four sets of two doubles per block: a launch of one or two
// steps and the launch before it whose second passes it finishes) and two
// doubles for the mass and energy when the caller passes no d_diag.  Each
// device holds its own copy for the life of the process; host code reaches
// it only through the address hipGetSymbolAddress returns on that device.
constexpr size_t kStaticMaxBlocks = 8192;
constexpr size_t kStaticScratchDoubles = 8 * kStaticMaxBlocks + 2;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {

constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;
double *g_static_scratch[kStaticMaxDevices];

// Device address of this device's copy of `scratch`, looked up once per device.
int static_scratch(double **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LWACM_EDEVICE;
    if (dev < 0 || dev >= kStaticMaxDevices) return LWACM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return LWACM_EDEVICE;
        g_static_scratch[dev] = static_cast<double *>(ptr);
    }
    *out = g_static_scratch[dev];
    return LWACM_OK;
}

}  // namespace

extern "C" {

size_t lwacm_state_bytes(int lattice, int nx, int ny, int nz, int storage)
{
    if ((lattice != LWACM_D2Q9 && lattice != LWACM_D3Q19) || nx < 1 || ny < 1 || nz < 1) return 0;
    if (lattice == LWACM_D2Q9 && nz != 1) return 0;
    if (storage != LWACM_FP32 && storage != LWACM_FP16_DEV) return 0;
    const size_t fields = (lattice == LWACM_D2Q9) ? 3 : 4;
    return fields * (size_t)nx * (size_t)ny * (size_t)nz * (storage == LWACM_FP32 ? 4 : 2);
}

const char *lwacm_strerror(int code)
{
    switch (code) {
    case LWACM_OK: return "success";
    case LWACM_EINVAL: return "invalid argument";
    case LWACM_ENOMEM: return "out of device memory for library scratch";
    case LWACM_EDEVICE: return "HIP runtime or kernel launch error";
    case LWACM_ENONFINITE: return "non-finite mass or kinetic energy (unstable run)";
    case LWACM_EUNSUPPORTED: return "not supported by the library";
    case LWACM_ESCRATCH: return "problem too large for the fixed scratch of lwacm_step_static";
    case LWACM_WOMEGA:
        return "success, with a warning: relaxation frequency below 1 (the method is stable "
               "for 1 <= omega < 2)";
    default: return "unknown error code";
    }
}

int lwacm_init(lwacm_ctx **out, int lattice, int nx, int ny, int nz, double omega, int storage,
               void *d_state_a, void *d_state_b, const uint8_t *d_mask, const float *h_wall_u,
               int n_wall_ids, const float *d_q, const float *h_g, hipStream_t stream)
{
    if (!out) return LWACM_EINVAL;
    *out = nullptr;
    if (lwacm_state_bytes(lattice, nx, ny, nz, storage) == 0) return LWACM_EINVAL;
    if (!(omega > 0.0 && omega < 2.0)) return LWACM_EINVAL;
    if (!d_state_a || !d_state_b || d_state_a == d_state_b) return LWACM_EINVAL;
    if (h_wall_u && (n_wall_ids < 1 || n_wall_ids > lwacm::kMaxWallIds)) return LWACM_EINVAL;

    lwacm_ctx *c = new (std::nothrow) lwacm_ctx;
    if (!c) return LWACM_ENOMEM;
    memset(c, 0, sizeof(*c));
    c->lattice = lattice;
    c->storage = storage;
    c->variant = LWACM_KERNEL_AUTO;
    c->omega = omega;
    c->rho0 = 1.0;
    c->buf[0] = d_state_a;
    c->buf[1] = d_state_b;
    c->stream = stream;
    c->k_rho = c->k_u = 14;
    c->sr_seed = 0;
    c->p.fp16_sr = 1;
    ProblemArgs &p = c->p;
    p.Q = lattice;
    p.D = lattice == LWACM_D2Q9 ? 2 : 3;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.n = (long long)nx * ny * nz;
    // a = 1 - h and A = 3 h from the quantised h = 2/omega - 1
    {
        const double hq = quantised_h(omega);
        p.a = (float)(1.0 - hq);
        p.A = (float)(3.0 * hq);
        p.Ap = p.A;
        p.split = 0;
        c->a_exact = 1.0 - hq;
        c->omega_p = omega;
    }
    p.mask = d_mask;
    p.qd = d_q;
    if (h_g) {
        for (int k = 0; k < p.D; ++k) p.g[k] = h_g[k];
        c->force = true;
        p.has_force = 1;
    }
    if (h_wall_u) {
        c->n_wall_ids = n_wall_ids;
        for (int m = 0; m < n_wall_ids; ++m)
            for (int k = 0; k < 3; ++k) c->wall_u[m][k] = h_wall_u[3 * m + k];
    }
    set_scales(c);
    set_wall_terms(c);

    // the tile kernels' chunk depth and block counts of the unforced problem
    // (a force, or a field set later, keeps the same tiling)
    ProblemArgs unforced = p;
    unforced.has_force = 0;
    unforced.qd = nullptr;  // interpolated walls run on the tiles with the wall correction
    if (lwacm::march_supported(unforced)) {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 256;
        p.march_nzc = lwacm::march_choose_nzc(p, ncu);
    }
    unforced.march_nzc = p.march_nzc;
    size_t nb = lwacm::kGenericMaxBlocks;
    const size_t mb = lwacm::march_num_blocks(unforced);
    if (mb > nb) nb = mb;
    const size_t ab = lwacm::adj_march_num_blocks(unforced);
    if (ab > nb) nb = ab;
    const size_t fb = lwacm::march2_num_blocks(unforced);
    if (fb > nb) nb = fb;
    const size_t rb = lwacm::adj_march2_num_blocks(unforced);
    if (rb > nb) nb = rb;
    c->n_partial_blocks = nb;
    // four partial sets of 2 doubles per block: a forward launch (one or two
    // steps) defers its second reduction passes into the next launch, so the
    // sets of two consecutive launches are live at once
    hipError_t e = hipMalloc(&c->d_partials, 8 * nb * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->d_diag, 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->d_scratch, 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->d_scan, 2 * sizeof(unsigned));
    if (e != hipSuccess) {
        free_scratch(c);
        delete c;
        return LWACM_ENOMEM;
    }
    e = hipMemsetAsync(c->d_diag, 0, 2 * sizeof(double), stream);

    c->n_fluid = (unsigned long long)p.n;
    if (e == hipSuccess && d_mask) {
        e = hipMemsetAsync(c->d_scan, 0, 2 * sizeof(unsigned), stream);
        if (e == hipSuccess) e = lwacm::launch_mask_scan(p, c->d_scan, stream);
        unsigned scan[2] = {0, 0};
        if (e == hipSuccess)
            e = hipMemcpyAsync(scan, c->d_scan, sizeof(scan), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) {
            const unsigned limit = h_wall_u ? (unsigned)n_wall_ids : 2u;
            if (scan[0] >= limit) {
                free_scratch(c);
                delete c;
                return LWACM_EINVAL;
            }
            c->n_fluid = scan[1];
        }
        if (e == hipSuccess &&
            (lwacm::march_supported(unforced) || lwacm::adj_march_supported(unforced))) {
            bool moving = false;
            for (int m = 1; m < lwacm::kMaxWallIds; ++m)
                for (int k = 0; k < 3; ++k) moving = moving || p.wall_u[m][k] != 0.0f;
            e = hipMalloc(&c->d_cls, (size_t)p.n);
            if (e == hipSuccess) e = hipMalloc(&c->d_bits, (size_t)p.n * sizeof(unsigned));
            if (e == hipSuccess && moving)
                e = hipMalloc(&c->d_wallg, (size_t)p.n * sizeof(float4));
            if (e != hipSuccess) {
                free_scratch(c);
                delete c;
                return LWACM_ENOMEM;
            }
            e = lwacm::launch_classify(p, c->d_cls, c->d_bits, c->d_wallg, stream);
        }
    }
    if (e != hipSuccess) {
        free_scratch(c);
        delete c;
        return LWACM_EDEVICE;
    }
    if (d_q && d_mask) {
        const int rc = enable_wall_correction(c);
        if (rc != LWACM_OK) {
            free_scratch(c);
            delete c;
            return rc;
        }
    }
    *out = c;
    return omega < 1.0 ? LWACM_WOMEGA : LWACM_OK;
}

int lwacm_coefficients(double omega, float *a, float *A)
{
    if (!a || !A || !(omega > 0.0 && omega < 2.0)) return LWACM_EINVAL;
    const double hq = quantised_h(omega);
    *a = (float)(1.0 - hq);
    *A = (float)(3.0 * hq);
    return omega < 1.0 ? LWACM_WOMEGA : LWACM_OK;
}

int lwacm_set_fp16_scales(lwacm_ctx *c, int k_rho, int k_u)
{
    if (!c || k_rho < 0 || k_rho > 24 || k_u < 0 || k_u > 24) return LWACM_EINVAL;
    c->k_rho = k_rho;
    c->k_u = k_u;
    set_scales(c);
    return LWACM_OK;
}

int lwacm_set_fp16_rounding(lwacm_ctx *c, int mode, uint32_t seed)
{
    if (!c || (mode != LWACM_ROUND_NEAREST && mode != LWACM_ROUND_STOCHASTIC)) return LWACM_EINVAL;
    c->p.fp16_sr = mode == LWACM_ROUND_STOCHASTIC;
    c->sr_seed = seed;
    return LWACM_OK;
}

int lwacm_set_march_chunk(lwacm_ctx *c, int planes)
{
    if (!c || (planes != 32 && planes != 64 && planes != 128)) return LWACM_EINVAL;
    if (!lwacm::march_supported(c->p)) return LWACM_EUNSUPPORTED;
    const int keep = c->p.march_nzc;
    c->p.march_nzc = planes;
    if (lwacm::march_num_blocks(c->p) > c->n_partial_blocks ||
        lwacm::march2_num_blocks(c->p) > c->n_partial_blocks) {  // reduction scratch too small
        c->p.march_nzc = keep;
        return LWACM_EUNSUPPORTED;
    }
    return LWACM_OK;
}

int lwacm_set_force_field(lwacm_ctx *c, const float *d_g)
{
    if (!c) return LWACM_EINVAL;
    c->p.g_field = d_g;
    c->p.has_force = (c->force || d_g) ? 1 : 0;
    return LWACM_OK;
}

int lwacm_set_omega_p(lwacm_ctx *c, double omega_p)
{
    if (!c || !(omega_p > 0.0 && omega_p < 2.0)) return LWACM_EINVAL;
    const float Ap = (float)(3.0 * quantised_h(omega_p));
    // not with interpolated walls, wall velocities given link by link or the
    // semi-implicit pressure update
    if ((c->p.qd || c->p.uwl || c->semi_implicit) && Ap != c->p.A) return LWACM_EUNSUPPORTED;
    c->omega_p = omega_p;
    c->p.Ap = Ap;
    c->p.split = c->p.Ap != c->p.A;
    set_wall_terms(c);
    return omega_p < 1.0 ? LWACM_WOMEGA : LWACM_OK;
}

int lwacm_set_semi_implicit(lwacm_ctx *c, int on)
{
    if (!c) return LWACM_EINVAL;
    if (on && (c->storage != LWACM_FP32 || c->p.split || c->p.qd || c->p.uwl ||
               c->variant == LWACM_KERNEL_MARCH || c->variant == LWACM_KERNEL_MARCH2))
        return LWACM_EUNSUPPORTED;
    c->semi_implicit = on != 0;
    return LWACM_OK;
}

int lwacm_set_wall_velocity_links(lwacm_ctx *c, const float *d_uw)
{
    if (!c || (d_uw && !c->p.mask)) return LWACM_EINVAL;
    if (d_uw && (c->p.split || c->semi_implicit)) return LWACM_EUNSUPPORTED;
    c->p.uwl = d_uw;
    if (d_uw) {
        if (228ull * c->p.n >= (1ull << 32)) {  // beyond the correction kernel's offsets
            c->p.corr = nullptr;
            return LWACM_OK;
        }
        return enable_wall_correction(c);
    }
    if (!c->p.qd) c->p.corr = nullptr;  // back to the halfway rule and the id table
    return LWACM_OK;
}

int lwacm_set_thermal(lwacm_ctx *c, double omega_t, float *d_T_a, float *d_T_b,
                      const float *h_wall_T, int n_wall_T)
{
    if (!c) return LWACM_EINVAL;
    if (!d_T_a && !d_T_b) {
        c->thermal = false;
        return LWACM_OK;
    }
    if (!d_T_a || !d_T_b || d_T_a == d_T_b || !(omega_t > 0.0 && omega_t < 2.0))
        return LWACM_EINVAL;
    if (n_wall_T < 0 || n_wall_T > lwacm::kMaxThermalWallIds || (n_wall_T > 0 && !h_wall_T))
        return LWACM_EINVAL;
    if (c->variant == LWACM_KERNEL_MARCH2) return LWACM_EUNSUPPORTED;
    lwacm::ThermalArgs &t = c->targs;
    t.st_half = c->storage != LWACM_FP32;  // refreshed with the scales at every launch
    t.ld_scale[0] = c->p.ld_scale[0];
    t.ld_scale[1] = c->p.ld_scale[1];
    t.Q = c->p.Q;
    t.QT = c->thermal_qt ? c->thermal_qt : c->p.Q;
    t.nx = c->p.nx;
    t.ny = c->p.ny;
    t.nz = c->p.nz;
    t.kap = (float)(2.0 - 2.0 / omega_t);
    t.h = (float)(2.0 / omega_t - 1.0);
    t.mask = c->p.mask;
    for (int m = 0; m < lwacm::kMaxThermalWallIds; ++m)
        t.wall_T[m] = m < n_wall_T ? h_wall_T[m] : __builtin_nanf("");
    // walls on a D3Q19 flow: the table of fixed-temperature wall links that
    // the flow kernel's fused temperature step reads
    if (c->p.mask && c->p.Q == 19) {
        if (!c->d_twall &&
            hipMalloc(&c->d_twall, sizeof(uint2) * (size_t)c->p.n) != hipSuccess) {
            c->d_twall = nullptr;
            return LWACM_ENOMEM;
        }
        if (lwacm::launch_thermal_wall_table(t, c->d_twall, c->stream) != hipSuccess)
            return LWACM_EDEVICE;
        c->p.T_wall = c->d_twall;
    }
    c->T_buf[0] = d_T_a;
    c->T_buf[1] = d_T_b;
    c->tcur = 0;
    c->thermal = true;
    return omega_t < 1.0 ? LWACM_WOMEGA : LWACM_OK;
}

int lwacm_adjoint_thermal_step(lwacm_ctx *c, const void *d_state_t, const float *d_T_t,
                               const float *d_lamT_in, float *d_lamT_out, float *d_mu,
                               int final_t0)
{
    if (!c || !d_state_t || !d_T_t || !d_lamT_in || !d_lamT_out || !d_mu) return LWACM_EINVAL;
    if (d_lamT_in == d_lamT_out || !c->thermal) return LWACM_EINVAL;
    lwacm::ThermalAdjArgs a;
    a.t = c->targs;
    a.t.state = d_state_t;
    a.t.st_half = c->storage != LWACM_FP32;
    a.t.ld_scale[0] = c->p.ld_scale[0];
    a.t.ld_scale[1] = c->p.ld_scale[1];
    a.t.T_in = d_T_t;
    a.t.T_out = nullptr;
    a.lam_in = d_lamT_in;
    a.lam_out = d_lamT_out;
    a.mu = d_mu;
    a.final_t0 = final_t0 != 0;
    return lwacm::launch_thermal_adjoint(a, c->stream) == hipSuccess ? LWACM_OK : LWACM_EDEVICE;
}

int lwacm_set_thermal_lattice(lwacm_ctx *c, int q_t)
{
    if (!c) return LWACM_EINVAL;
    const int axis = c->p.Q == 9 ? 5 : 7;
    if (q_t != 0 && q_t != c->p.Q && q_t != axis) return LWACM_EINVAL;
    c->thermal_qt = q_t == c->p.Q ? 0 : q_t;
    c->targs.QT = q_t ? q_t : c->p.Q;
    return LWACM_OK;
}

int lwacm_wall_force(lwacm_ctx *c, int wall_id, const double *h_center, double *h_out)
{
    if (!c || !h_out || !c->p.mask || wall_id < 1 || wall_id > 255) return LWACM_EINVAL;
    if (c->storage != LWACM_FP32) return LWACM_EUNSUPPORTED;
    // momentum exchange as the paper states it covers bodies at rest
    if (wall_id < c->n_wall_ids)
        for (int k = 0; k < 3; ++k)
            if (c->wall_u[wall_id][k] != 0.0f) return LWACM_EUNSUPPORTED;
    if (!c->d_force) {
        // the result goes straight to pinned host memory: no copy after the sum
        if (hipMalloc(&c->d_force, sizeof(double) * 6 * (lwacm::kForceMaxBlocks + 1)) != hipSuccess ||
            hipHostMalloc(&c->h_force, 6 * sizeof(double), hipHostMallocMapped) != hipSuccess) {
            if (c->d_force) (void)hipFree(c->d_force);
            c->d_force = nullptr;
            c->h_force = nullptr;
            return LWACM_ENOMEM;
        }
    }
    lwacm::ForceArgs f;
    f.Q = c->p.Q;
    f.nx = c->p.nx;
    f.ny = c->p.ny;
    f.nz = c->p.nz;
    f.A = c->p.A;
    f.state = static_cast<const float *>(c->buf[c->cur]);
    f.mask = c->p.mask;
    f.qd = c->p.qd;
    f.wall_id = wall_id;
    for (int k = 0; k < 3; ++k) f.xc[k] = h_center ? h_center[k] : 0.0;
    f.partials = c->d_force + 6;
    double *d_out = nullptr;
    if (hipHostGetDevicePointer((void **)&d_out, c->h_force, 0) != hipSuccess || !d_out)
        return LWACM_EDEVICE;
    f.out = d_out;
    f.list = nullptr;
    f.nlist = 0;
    long long items = (long long)c->p.nx * c->p.ny * c->p.nz;
    const int lrc = ensure_wall_list(c);
    if (lrc == LWACM_OK) {
        // only the fluid nodes next to a wall carry links into one
        f.list = c->d_wlist;
        f.nlist = c->n_wlist;
        items = c->n_wlist;
    } else if (lrc != LWACM_EUNSUPPORTED) {
        return lrc;
    }
    long long nb = (items + lwacm::kForceBlock - 1) / lwacm::kForceBlock;
    if (nb < 1) nb = 1;
    if (nb > (long long)lwacm::kForceMaxBlocks) nb = lwacm::kForceMaxBlocks;
    if (lwacm::launch_wall_force(f, (unsigned)nb, c->stream) != hipSuccess) return LWACM_EDEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LWACM_EDEVICE;
    for (int k = 0; k < 6; ++k) h_out[k] = c->h_force[k];
    return LWACM_OK;
}

int lwacm_temperature(lwacm_ctx *c, float **d_T)
{
    if (!c || !d_T || !c->thermal) return LWACM_EINVAL;
    *d_T = c->T_buf[c->tcur];
    return LWACM_OK;
}

int lwacm_set_variant(lwacm_ctx *c, int variant)
{
    if (!c) return LWACM_EINVAL;
    if (variant == LWACM_KERNEL_AUTO || variant == LWACM_KERNEL_GENERIC) {
        c->variant = variant;
        return LWACM_OK;
    }
    if (variant == LWACM_KERNEL_MARCH2) {
        if (c->storage != LWACM_FP32 || c->thermal || c->semi_implicit ||
            !lwacm::march2_supported(c->p))
            return LWACM_EUNSUPPORTED;
        c->variant = variant;
        return LWACM_OK;
    }
    if (variant == LWACM_KERNEL_MARCH) {
        if (c->semi_implicit || !lwacm::march_supported(c->p)) return LWACM_EUNSUPPORTED;
        c->variant = variant;
        return LWACM_OK;
    }
    return LWACM_EINVAL;
}

int lwacm_set_state(lwacm_ctx *c, const float *d_drho, const float *d_u)
{
    if (!c || !d_drho || !d_u) return LWACM_EINVAL;
    set_scales(c);
    hipError_t e = lwacm::launch_set_state(c->p, c->storage, d_drho, d_u, c->buf[c->cur], c->stream);
    if (e != hipSuccess) return LWACM_EDEVICE;
    // both buffers hold the state: a step leaves solid nodes as they are
    e = hipMemcpyAsync(c->buf[c->cur ^ 1], c->buf[c->cur], state_bytes(c),
                       hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return LWACM_EDEVICE;
    // rho0 = mean fluid density of the stored state (moving-wall term)
    ReduceArgs r = reduce_args(c, c->d_scratch, nullptr);
    e = lwacm::launch_moments(c->p, c->storage, c->buf[c->cur], nullptr, nullptr, r,
                              lwacm::generic_grid(c->p.n), c->stream);
    double h[2] = {0.0, 0.0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, c->d_scratch, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return LWACM_EDEVICE;
    if (!isfinite(h[0]) || !isfinite(h[1])) return LWACM_ENONFINITE;
    c->rho0 = c->n_fluid ? 1.0 + h[0] / (double)c->n_fluid : 1.0;
    set_wall_terms(c);
    c->steps = 0;
    c->diag_valid = false;
    return LWACM_OK;
}

int lwacm_step(lwacm_ctx *c, int nsteps)
{
    if (!c || nsteps < 0) return LWACM_EINVAL;
    const bool march = use_march(c);
    const bool fuse = march && use_march2(c);
    const bool multi = !march && use_multi(c);
    const unsigned nb1 = march ? lwacm::march_num_blocks(c->p)
                               : (multi ? lwacm::d2q9_multi_num_blocks(c->p)
                                        : lwacm::generic_grid(c->p.n));
    const unsigned nb2 = fuse ? lwacm::march2_num_blocks(c->p) : 0u;
    const size_t set = 2 * c->n_partial_blocks;  // doubles per partial set
    // Steps whose partials are stored but not yet added up (oldest first): the
    // next launch's block 0 adds them, or the final passes after the loop.
    struct Pending {
        double *partials, *out, *out2;
        unsigned nblocks;
    } pend[2];
    int npend = 0;
    int s = 0;
    for (int launch = 0; s < nsteps; ++launch) {
        // an odd step count starts with one single step, then pairs; the
        // multi-step D2Q9 kernel takes up to kMultiSteps steps at a time
        const bool two = fuse && (nsteps - s) % 2 == 0;
        const int kk = multi ? (nsteps - s < lwacm::kMultiSteps ? nsteps - s : lwacm::kMultiSteps)
                             : (two ? 2 : 1);
        double *part = c->d_partials + 2 * set * (size_t)(launch & 1);
        ReduceArgs r = reduce_args(c, c->d_diag, hist_slot(c, c->steps + 1));
        r.partials = part;
        if (two) r.partials_b = part + set;
        if (npend > 0) {
            r.prev_partials = pend[0].partials;
            r.prev_nblocks = pend[0].nblocks;
            r.prev_out = pend[0].out;
            r.prev_out2 = pend[0].out2;
        }
        if (npend > 1) {
            r.prev_partials_b = pend[1].partials;
            r.prev_nblocks_b = pend[1].nblocks;
            r.prev_out_b = pend[1].out;
            r.prev_out2_b = pend[1].out2;
        }
        const void *src = c->buf[c->cur];
        void *dst = c->buf[c->cur ^ 1];
        c->p.sr_word = (uint32_t)(c->steps + 1) ^ c->sr_seed;
        hipError_t e;
        // T advances with the flow velocity of the same time: in the flow's own
        // tile kernel where it can, else by a kernel of its own that reads the
        // state this step's flow kernel reads, before that kernel runs
        ProblemArgs pl = c->p;
        const bool tfuse = c->thermal && march && !two && c->targs.QT == c->p.Q &&
                           lwacm::march_thermal_supported(c->p);
        if (tfuse) {
            pl.T_in = c->T_buf[c->tcur];
            pl.T_out = c->T_buf[c->tcur ^ 1];
            pl.t_h = c->targs.h;
            pl.t_kap = c->targs.kap;
            c->tcur ^= 1;
        } else if (c->thermal) {
            lwacm::ThermalArgs t = c->targs;
            t.state = src;
            t.st_half = c->storage != LWACM_FP32;
            t.ld_scale[0] = c->p.ld_scale[0];
            t.ld_scale[1] = c->p.ld_scale[1];
            t.T_in = c->T_buf[c->tcur];
            t.T_out = c->T_buf[c->tcur ^ 1];
            if (lwacm::launch_thermal_step(t, c->stream) != hipSuccess) return LWACM_EDEVICE;
            c->tcur ^= 1;
        }
        if (march && !two && c->p.corr &&
            lwacm::launch_wall_correction(c->p, c->storage, src, wall_links(c), c->d_corr,
                                          c->stream) != hipSuccess)
            return LWACM_EDEVICE;
        if (two)
            e = lwacm::launch_fwd_march2(c->p, static_cast<const float *>(src),
                                         static_cast<float *>(dst), c->d_bits, c->d_wallg, r,
                                         c->stream);
        else if (march)
            e = lwacm::launch_fwd_march(pl, c->storage, src, dst, c->d_cls, c->d_bits,
                                        c->d_wallg, r, c->stream);
        else if (multi)
            e = lwacm::launch_fwd_d2q9_multi(c->p, static_cast<const float *>(src),
                                             static_cast<float *>(dst), kk, r, c->stream);
        else
            e = lwacm::launch_fwd_generic(c->p, c->storage, c->p.has_force != 0, src, dst, r, nb1,
                                          c->stream);
        if (e == hipSuccess && c->semi_implicit) {
            // the density again, from the old density and the new velocity;
            // its sums replace the explicit pass's in the same partial set
            ReduceArgs r2 = reduce_args(c, r.out, r.out2);
            r2.partials = r.partials;
            e = lwacm::launch_density_si(c->p, static_cast<const float *>(src),
                                         static_cast<float *>(dst), r2, nb1, c->stream);
        }
        if (e != hipSuccess) return LWACM_EDEVICE;
        const unsigned nb = two ? nb2 : nb1;
        npend = 0;
        pend[npend++] = {r.partials, r.out, r.out2, nb};
        if (two) pend[npend++] = {r.partials_b, c->d_diag, hist_slot(c, c->steps + 2), nb};
        c->cur ^= 1;
        c->steps += kk;
        s += kk;
        c->diag_valid = true;
    }
    // the last launch's sums: mass/energy and history complete when the call's work is
    for (int i = 0; i < npend; ++i) {
        ReduceArgs r = reduce_args(c, pend[i].out, pend[i].out2);
        r.partials = pend[i].partials;
        if (lwacm::launch_reduce(r, 2, pend[i].nblocks, c->stream) != hipSuccess)
            return LWACM_EDEVICE;
    }
    return LWACM_OK;
}

int lwacm_diagnostics(lwacm_ctx *c, double *h_mass, double *h_energy)
{
    if (!c || !h_mass || !h_energy) return LWACM_EINVAL;
    if (!c->diag_valid) return LWACM_EINVAL;
    double h[2];
    hipError_t e = hipMemcpyAsync(h, c->d_diag, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return LWACM_EDEVICE;
    *h_mass = (double)c->n_fluid + h[0];
    *h_energy = h[1];
    return (isfinite(h[0]) && isfinite(h[1])) ? LWACM_OK : LWACM_ENONFINITE;
}

int lwacm_set_diag_history(lwacm_ctx *c, double *d_hist, int capacity)
{
    if (!c || (d_hist && capacity < 1)) return LWACM_EINVAL;
    c->d_hist = d_hist;
    c->hist_cap = d_hist ? capacity : 0;
    return LWACM_OK;
}

int lwacm_moments(lwacm_ctx *c, float *d_drho, float *d_u, double *h_mass, double *h_energy)
{
    if (!c) return LWACM_EINVAL;
    ReduceArgs r = reduce_args(c, c->d_scratch, nullptr);
    hipError_t e = lwacm::launch_moments(c->p, c->storage, c->buf[c->cur], d_drho, d_u, r,
                                         lwacm::generic_grid(c->p.n), c->stream);
    if (e != hipSuccess) return LWACM_EDEVICE;
    if (!h_mass && !h_energy) return LWACM_OK;
    double h[2];
    e = hipMemcpyAsync(h, c->d_scratch, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return LWACM_EDEVICE;
    if (h_mass) *h_mass = (double)c->n_fluid + h[0];
    if (h_energy) *h_energy = h[1];
    return (isfinite(h[0]) && isfinite(h[1])) ? LWACM_OK : LWACM_ENONFINITE;
}

int lwacm_save_state(lwacm_ctx *c, void *d_dst)
{
    if (!c || !d_dst) return LWACM_EINVAL;
    const size_t bytes = lwacm_state_bytes(c->lattice, c->p.nx, c->p.ny, c->p.nz, c->storage);
    return dev_err(hipMemcpyAsync(d_dst, c->buf[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream));
}

int lwacm_load_state(lwacm_ctx *c, const void *d_src, long long step)
{
    if (!c || !d_src || step < 0) return LWACM_EINVAL;
    const size_t bytes = lwacm_state_bytes(c->lattice, c->p.nx, c->p.ny, c->p.nz, c->storage);
    hipError_t e = hipMemcpyAsync(c->buf[c->cur], d_src, bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->buf[c->cur ^ 1], d_src, bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return LWACM_EDEVICE;
    c->steps = step;
    c->diag_valid = false;
    return LWACM_OK;
}

const void *lwacm_current_state(lwacm_ctx *c)
{
    return c ? c->buf[c->cur] : nullptr;
}

long long lwacm_step_count(lwacm_ctx *c)
{
    return c ? c->steps : -1;
}

int lwacm_adjoint_seed(lwacm_ctx *c, const void *d_state_T, const float *d_lambda_T, float *d_mu)
{
    if (!c || !d_state_T || !d_lambda_T || !d_mu || (const void *)d_lambda_T == (const void *)d_mu)
        return LWACM_EINVAL;
    return dev_err(lwacm::launch_adj_seed(c->p, c->storage, d_state_T, d_lambda_T, d_mu, c->stream));
}

int lwacm_adjoint_step(lwacm_ctx *c, const void *d_state_t, const float *d_mu_in, float *d_mu_out,
                       double *d_dL_domega, int final_t0)
{
    if (!c || !d_state_t || !d_mu_in || !d_mu_out || !d_dL_domega || d_mu_in == d_mu_out)
        return LWACM_EINVAL;
    // no reverse step for omega_p != omega, a node-by-node acceleration or
    // interpolated bounce-back
    if (c->p.split || c->p.g_field || c->p.qd || c->p.uwl || c->semi_implicit)
        return LWACM_EUNSUPPORTED;
    ReduceArgs r = reduce_args(c, d_dL_domega, nullptr);
    r.accumulate = 1;
    r.out_scale = 2.0 / (c->omega * c->omega);  // da/domega for a = 2 - 2/omega
    if (c->variant != LWACM_KERNEL_GENERIC && lwacm::adj_march_supported(c->p))
        return dev_err(lwacm::launch_adj_march(c->p, c->storage, d_state_t, d_mu_in, d_mu_out,
                                               c->d_bits, c->d_wallg, final_t0, r, c->stream));
    return dev_err(lwacm::launch_adj_generic(c->p, c->storage, d_state_t, d_mu_in, d_mu_out,
                                             final_t0, r, lwacm::generic_grid(c->p.n), c->stream));
}

int lwacm_adjoint_step2(lwacm_ctx *c, const void *d_state_t, const void *d_state_tm1,
                        const float *d_mu_in, float *d_mu_out, double *d_dL_domega, int final_t0)
{
    if (!c || !d_state_t || !d_state_tm1 || !d_mu_in || !d_mu_out || !d_dL_domega ||
        d_mu_in == d_mu_out)
        return LWACM_EINVAL;
    if ((c->variant != LWACM_KERNEL_AUTO && c->variant != LWACM_KERNEL_MARCH2) ||
        !lwacm::adj_march2_supported(c->p) || c->p.split || c->p.g_field || c->p.qd || c->p.uwl ||
        c->semi_implicit)
        return LWACM_EUNSUPPORTED;
    ReduceArgs r = reduce_args(c, d_dL_domega, nullptr);
    r.accumulate = 1;
    r.out_scale = 2.0 / (c->omega * c->omega);  // da/domega for a = 2 - 2/omega
    r.partials_b = c->d_partials + c->n_partial_blocks;
    return dev_err(lwacm::launch_adj_march2(c->p, c->storage, d_state_t, d_state_tm1, d_mu_in,
                                            d_mu_out, final_t0, r, c->stream));
}

int lwacm_forward_states(lwacm_ctx *c, const void *d_state0, long long t0, int nsteps,
                         void *d_states)
{
    if (!c || !d_state0 || !d_states || nsteps < 0 || t0 < 0) return LWACM_EINVAL;
    if (c->thermal) return LWACM_EUNSUPPORTED;
    const size_t sb = state_bytes(c);
    const char *lo = static_cast<const char *>(d_states);
    const char *s0 = static_cast<const char *>(d_state0);
    if (s0 + sb > lo && s0 < lo + (size_t)nsteps * sb) return LWACM_EINVAL;  // overlap
    const bool march = use_march(c);
    const bool multi = !march && use_multi(c);
    const unsigned nb1 = march ? lwacm::march_num_blocks(c->p)
                               : (multi ? lwacm::d2q9_multi_num_blocks(c->p)
                                        : lwacm::generic_grid(c->p.n));
    // The masked tile kernels leave solid nodes unwritten (the context's two
    // buffers both hold them): the slots get them from d_state0 first.
    if (march && c->p.mask)
        for (int k = 0; k < nsteps; ++k)
            if (hipMemcpyAsync(static_cast<char *>(d_states) + (size_t)k * sb, d_state0, sb,
                               hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
                return LWACM_EDEVICE;
    // block partials go to the scratch; no second pass (no diagnostics)
    ReduceArgs r = reduce_args(c, nullptr, nullptr);
    if (multi) {  // D2Q9: up to kMultiSteps steps per launch, each step's state out
        for (int k = 0; k < nsteps;) {
            const int kk = nsteps - k < lwacm::kMultiSteps ? nsteps - k : lwacm::kMultiSteps;
            const void *src = k == 0 ? d_state0 : static_cast<const void *>(lo + (size_t)(k - 1) * sb);
            if (lwacm::launch_fwd_d2q9_multi(c->p, static_cast<const float *>(src), nullptr, kk, r,
                                             c->stream,
                                             reinterpret_cast<float *>(
                                                 static_cast<char *>(d_states) + (size_t)k * sb),
                                             sb / 4) != hipSuccess)
                return LWACM_EDEVICE;
            k += kk;
        }
        return LWACM_OK;
    }
    for (int k = 0; k < nsteps; ++k) {
        const void *src = k == 0 ? d_state0 : static_cast<const void *>(lo + (size_t)(k - 1) * sb);
        void *dst = static_cast<char *>(d_states) + (size_t)k * sb;
        ProblemArgs pl = c->p;
        pl.sr_word = (uint32_t)(t0 + k + 1) ^ c->sr_seed;  // as lwacm_step draws for step t0 + k
        hipError_t e = hipSuccess;
        if (march && pl.corr)
            e = lwacm::launch_wall_correction(pl, c->storage, src, wall_links(c), c->d_corr,
                                              c->stream);
        if (e == hipSuccess) {
            if (march)
                e = lwacm::launch_fwd_march(pl, c->storage, src, dst, c->d_cls, c->d_bits,
                                            c->d_wallg, r, c->stream);
            else if (multi)
                e = lwacm::launch_fwd_d2q9_multi(pl, static_cast<const float *>(src),
                                                 static_cast<float *>(dst), 1, r, c->stream);
            else
                e = lwacm::launch_fwd_generic(pl, c->storage, pl.has_force != 0, src, dst, r, nb1,
                                              c->stream);
        }
        if (e == hipSuccess && c->semi_implicit)
            e = lwacm::launch_density_si(pl, static_cast<const float *>(src),
                                         static_cast<float *>(dst), r, nb1, c->stream);
        if (e != hipSuccess) return LWACM_EDEVICE;
    }
    return LWACM_OK;
}

int lwacm_adjoint_sweep(lwacm_ctx *c, const void *d_states, long long t0, int nsteps,
                        float *d_mu, float *d_mu_tmp, double *d_dL_domega)
{
    if (!c || !d_states || !d_mu || !d_mu_tmp || !d_dL_domega || d_mu == d_mu_tmp ||
        nsteps < 0 || t0 < 0)
        return LWACM_EINVAL;
    if (c->p.split || c->p.g_field || c->p.qd || c->p.uwl || c->semi_implicit)
        return LWACM_EUNSUPPORTED;
    if (nsteps == 0) return LWACM_OK;
    const size_t sb = state_bytes(c);
    const char *st = static_cast<const char *>(d_states);
    const size_t stride = c->n_partial_blocks;  // doubles per slice
    const size_t need = (size_t)nsteps * (stride + 1);
    if (need > c->sweep_cap) {
        if (c->d_sweep) (void)hipFree(c->d_sweep);
        c->d_sweep = nullptr;
        c->sweep_cap = 0;
        if (hipMalloc(&c->d_sweep, need * sizeof(double)) != hipSuccess) return LWACM_ENOMEM;
        c->sweep_cap = need;
    }
    // zero slices: each launch fills its own blocks' entries only
    if (hipMemsetAsync(c->d_sweep, 0, (size_t)nsteps * stride * sizeof(double), c->stream) !=
        hipSuccess)
        return LWACM_EDEVICE;
    const bool two_ok = (c->variant == LWACM_KERNEL_AUTO || c->variant == LWACM_KERNEL_MARCH2) &&
                        lwacm::adj_march2_supported(c->p);
    const bool tile = c->variant != LWACM_KERNEL_GENERIC && lwacm::adj_march_supported(c->p);
    // D2Q9: up to kMultiSteps reverse steps per launch in LDS
    const bool multi = c->variant == LWACM_KERNEL_AUTO && c->storage == LWACM_FP32 &&
                       lwacm::d2q9_multi_supported(c->p) &&
                       lwacm::d2q9_multi_num_blocks(c->p) <= c->n_partial_blocks;
    float *mu_in = d_mu, *mu_out = d_mu_tmp;
    unsigned slice = 0;
    long long t = t0 + nsteps - 1;
    while (t >= t0) {
        ReduceArgs r = reduce_args(c, nullptr, nullptr);  // partials only, added below
        r.partials = c->d_sweep + (size_t)slice * stride;
        hipError_t e;
        if (multi) {
            const int k = (int)(t - t0 + 1 < lwacm::kMultiSteps ? t - t0 + 1 : lwacm::kMultiSteps);
            e = lwacm::launch_adj_d2q9_multi(c->p, reinterpret_cast<const float *>(st), sb / 4,
                                             (int)(t - t0), k, t - k + 1 == 0, mu_in, mu_out,
                                             c->d_sweep, stride, slice, c->stream);
            slice += (unsigned)k;
            t -= k;
        } else if (two_ok && t - 1 >= t0) {
            r.partials_b = r.partials + stride;
            e = lwacm::launch_adj_march2(c->p, c->storage, st + (size_t)(t - t0) * sb,
                                         st + (size_t)(t - 1 - t0) * sb, mu_in, mu_out,
                                         t - 1 == 0, r, c->stream);
            slice += 2;
            t -= 2;
        } else {
            if (tile)
                e = lwacm::launch_adj_march(c->p, c->storage, st + (size_t)(t - t0) * sb, mu_in,
                                            mu_out, c->d_bits, c->d_wallg, t == 0, r, c->stream);
            else
                e = lwacm::launch_adj_generic(c->p, c->storage, st + (size_t)(t - t0) * sb,
                                              mu_in, mu_out, t == 0, r,
                                              lwacm::generic_grid(c->p.n), c->stream);
            slice += 1;
            t -= 1;
        }
        if (e != hipSuccess) return LWACM_EDEVICE;
        float *tmp = mu_in;
        mu_in = mu_out;
        mu_out = tmp;
    }
    // the steps' dL/domega, added in the order separate calls add them
    if (lwacm::launch_reduce_slices(c->d_sweep, stride, (unsigned)stride, slice,
                                    c->d_sweep + (size_t)nsteps * stride,
                                    2.0 / (c->omega * c->omega), d_dL_domega,
                                    c->stream) != hipSuccess)
        return LWACM_EDEVICE;
    if (mu_in != d_mu &&
        hipMemcpyAsync(d_mu, mu_in, (size_t)(c->p.D + 1) * (size_t)c->p.n * sizeof(float),
                       hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return LWACM_EDEVICE;
    return LWACM_OK;
}

void lwacm_destroy(lwacm_ctx *c)
{
    if (!c) return;
    free_scratch(c);
    delete c;
}

int lwacm_step_static(int lattice, int nx, int ny, int nz, double omega, float *d_state_a,
                      float *d_state_b, int nsteps, double *d_diag, float **h_state_out,
                      hipStream_t stream)
{
    if (lwacm_state_bytes(lattice, nx, ny, nz, LWACM_FP32) == 0 || nsteps < 0) return LWACM_EINVAL;
    if (!(omega > 0.0 && omega < 2.0)) return LWACM_EINVAL;
    if (!d_state_a || !d_state_b || d_state_a == d_state_b) return LWACM_EINVAL;
    // a context on the stack: the problem of lwacm_init without mask, walls
    // or force, in FP32 storage, with the kernels lwacm_step chooses for it
    lwacm_ctx c;
    memset(&c, 0, sizeof(c));
    c.lattice = lattice;
    c.storage = LWACM_FP32;
    c.variant = LWACM_KERNEL_AUTO;
    c.omega = omega;
    c.omega_p = omega;
    c.rho0 = 1.0;
    c.buf[0] = d_state_a;
    c.buf[1] = d_state_b;
    c.stream = stream;
    ProblemArgs &p = c.p;
    p.Q = lattice;
    p.D = lattice == LWACM_D2Q9 ? 2 : 3;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.n = (long long)nx * ny * nz;
    const double hq = quantised_h(omega);
    p.a = (float)(1.0 - hq);
    p.A = (float)(3.0 * hq);
    p.Ap = p.A;
    c.a_exact = 1.0 - hq;
    set_scales(&c);
    set_wall_terms(&c);
    if (lwacm::march_supported(p)) {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 256;
        p.march_nzc = lwacm::march_choose_nzc(p, ncu);
    }
    // the partial sets of the kernels lwacm_step may launch must fit the scratch
    size_t nb = lwacm::generic_grid(p.n);
    const size_t mb = lwacm::march_num_blocks(p);
    if (mb > nb) nb = mb;
    const size_t fb = lwacm::march2_num_blocks(p);
    if (fb > nb) nb = fb;
    if (nb > kStaticMaxBlocks) return LWACM_ESCRATCH;
    double *base = nullptr;
    const int rc = static_scratch(&base);
    if (rc != LWACM_OK) return rc;
    c.d_partials = base;
    c.n_partial_blocks = nb;
    c.d_diag = d_diag ? d_diag : base + 8 * kStaticMaxBlocks;
    c.n_fluid = (unsigned long long)p.n;
    const int code = lwacm_step(&c, nsteps);
    if (code == LWACM_OK && h_state_out) *h_state_out = static_cast<float *>(c.buf[c.cur]);
    return (code == LWACM_OK && omega < 1.0) ? LWACM_WOMEGA : code;
}

}  // extern "C"
