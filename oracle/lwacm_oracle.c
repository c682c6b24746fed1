/*
 * lwacm_oracle.c -- plain FP64 CPU oracle of the LW-ACM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  It shares no
 * code, header, table or constant with the HIP library: lattices, equilibria
 * and the update are written out again here, directly from the paper, in the
 * paper's own (population) form and in double precision, with no fusion,
 * blocking or algebraic simplification.
 *
 * What it computes (Asinari, Ohwada, Chiavazzo, Di Rienzo, "Link-wise
 * artificial compressibility method", arXiv:1111.2142):
 *   - lattices D2Q9 and D3Q19 with their weights (Appendix A, Eqs.
 *     d2q9_equilibrium_compact, weight_factors, weight_factors_3d);
 *   - the equilibrium f^(e) (Eq. d2q9_equilibrium_compact, "formally
 *     identical" for D3Q19) and its odd part f^(e,o), taken literally as
 *     half the difference of f^(e) at +u and -u (Eq. feqo);
 *   - the link-wise update, Eq. ACM2.0: every population at x is the
 *     upstream equilibrium plus (2 - 2/omega) times the odd-part difference
 *     between x and the upstream node;
 *   - the forcing step, Eq. force: the odd part evaluated at (rho(x,t), g) is
 *     added to every population; g uniform, or a field given node by node
 *     (the space- and time-dependent acceleration of Section "Generalized
 *     Taylor-Green vortex flow");
 *   - halfway bounce-back for a solid upstream node, Eqs. ACM2.0cbb to
 *     ACM2.0cccbb2, with the moving-wall correction of Eqs. ACM2.0movebb
 *     and ACM2.0ccccbb, (2/omega - 1) * 2 f^(e,o)(rho0, u_w); and, with
 *     link-wall distances q, the interpolated bounce-back of Eq. ACM2.0cc
 *     with the moving-wall term of Eq. ACM2.0move (factor 2 or 1/q in place
 *     of 2);
 *   - new moments rho = sum f_i, rho u = sum v_i f_i (Section 2.1);
 *   - a separate relaxation omega_p for the continuity equation (Section
 *     "finite-difference formulation", item 3; Appendix E): the density is
 *     the zeroth moment of the populations of Eq. ACM2.0 evaluated with
 *     omega_p in place of omega (in the link update, the bounce-back and
 *     the moving-wall correction alike), the momentum their first moment
 *     with omega, and u = momentum / density;
 *   - diagnostics: mass sum(rho) and kinetic energy 1/2 sum |u|^2 over
 *     fluid nodes (the energy of Section 3.1.1, in lattice units);
 *   - FP16 storage with stochastic rounding (not part of the paper: a
 *     storage format of the GPU library): the real value is rounded up to
 *     the next FP16 magnitude when its fractional position between the two
 *     neighbouring FP16 magnitudes, cut to 13 bits, plus a uniform 13-bit
 *     variate reaches 1; the variate comes from the pcg2d hash (Jarzynski
 *     and Olano, "Hash Functions for GPU Rendering", JCGT 9(3), 2020) of
 *     (node index, t ^ seed);
 *   - force and torque on a wall by momentum exchange (Eqs. MEA3, MEA4,
 *     MEA5), for halfway and interpolated walls at rest;
 *   - the thermal extension (Appendix "Asymptotic analysis for energy
 *     equation", Eqs. ACM2.0t and feqe): a temperature lattice, the flow's
 *     own or the smaller D2Q5 / D3Q7 (the appendix allows Q_t != Q),
 *     advected by the flow velocity, with an equilibrium whose moments are
 *     the ones the appendix states (on D2Q5 / D3Q7 all but the O(eps^2)
 *     u u part, which those lattices cannot carry), its even part taken
 *     literally as the mean at +u and -u, and adiabatic or fixed-temperature
 *     halfway walls (the oracle's reading; the paper has no thermal wall rule);
 *   - the vector-Jacobian product of one step (reverse mode), obtained by
 *     the chain rule through the same population form.  The paper has no
 *     adjoint; the oracle's reading is "exact derivative of the step above",
 *     pinned by central finite differences in the tests.
 *
 * Layout: structure of arrays, node index ((z*ny)+y)*nx+x, every axis
 * periodic; walls are solid mask nodes (mask != 0), mask value m >= 1 selects
 * wall velocity wall_u[3*m .. 3*m+2] (all zero when wall_u is NULL).
 * Solid nodes are never updated: their state is copied through.
 * The state is (rho, u) in double precision; u has D components (SoA).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXQ 19

typedef struct {
    int q;          /* number of links */
    int d;          /* dimension */
    int v[MAXQ][3]; /* link velocities */
    double w[MAXQ]; /* weights */
    int opp[MAXQ];  /* BB(i): the link opposite to i */
    int lin;        /* temperature lattices D2Q5, D3Q7: linear equilibrium */
} lattice_t;

/* D2Q9 in the order of Appendix A: rest, the four axis links, the four
 * diagonals, with weights 4/9, 1/9, 1/36 (Eq. weight_factors). */
static const int D2Q9_V[9][2] = {
    {0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};

/* D3Q19: rest, six axis links, twelve face diagonals (Appendix A names only
 * the groups; the order inside a group is this oracle's own choice).
 * Weights 1/3, 1/18, 1/36 (Eq. weight_factors_3d). */
static const int D3Q19_V[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static int make_lattice(int q, lattice_t *L)
{
    memset(L, 0, sizeof(*L));
    if (q == 9) {
        L->q = 9;
        L->d = 2;
        for (int i = 0; i < 9; ++i) {
            L->v[i][0] = D2Q9_V[i][0];
            L->v[i][1] = D2Q9_V[i][1];
            L->v[i][2] = 0;
            L->w[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
    } else if (q == 19) {
        L->q = 19;
        L->d = 3;
        for (int i = 0; i < 19; ++i) {
            for (int k = 0; k < 3; ++k) L->v[i][k] = D3Q19_V[i][k];
            L->w[i] = (i == 0) ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
    } else {
        return -1;
    }
    /* BB(i): found by search for the link with velocity -v_i. */
    for (int i = 0; i < L->q; ++i) {
        L->opp[i] = -1;
        for (int j = 0; j < L->q; ++j)
            if (L->v[j][0] == -L->v[i][0] && L->v[j][1] == -L->v[i][1] &&
                L->v[j][2] == -L->v[i][2])
                L->opp[i] = j;
        if (L->opp[i] < 0) return -1;
    }
    return 0;
}

/* ---- equilibrium and odd part, Eqs. d2q9_equilibrium_compact and feqo ---- */

static double vdot(const lattice_t *L, int i, const double u[3])
{
    return L->v[i][0] * u[0] + L->v[i][1] * u[1] + L->v[i][2] * u[2];
}

static double feq(const lattice_t *L, int i, double rho, const double u[3])
{
    double c = vdot(L, i, u);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->w[i] * rho * (1.0 + 3.0 * c + 4.5 * c * c - 1.5 * uu);
}

static double feo(const lattice_t *L, int i, double rho, const double u[3])
{
    double mu[3] = {-u[0], -u[1], -u[2]};
    return 0.5 * (feq(L, i, rho, u) - feq(L, i, rho, mu));
}

/* Partial derivatives of f^(e) with respect to rho and to u (componentwise),
 * differentiated term by term from Eq. d2q9_equilibrium_compact. */
static void dfeq(const lattice_t *L, int i, double rho, const double u[3], double *d_rho,
                 double d_u[3])
{
    double c = vdot(L, i, u);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    *d_rho = L->w[i] * (1.0 + 3.0 * c + 4.5 * c * c - 1.5 * uu);
    for (int k = 0; k < 3; ++k)
        d_u[k] = L->w[i] * rho * (3.0 * L->v[i][k] + 9.0 * c * L->v[i][k] - 3.0 * u[k]);
}

/* Derivatives of f^(e,o)(rho,u) = 1/2 [f^(e)(rho,u) - f^(e)(rho,-u)] by the
 * chain rule through the definition (the -u argument flips the sign of the
 * u-derivative of the second term). */
static void dfeo(const lattice_t *L, int i, double rho, const double u[3], double *d_rho,
                 double d_u[3])
{
    double mu[3] = {-u[0], -u[1], -u[2]};
    double ap, am, bp[3], bm[3];
    dfeq(L, i, rho, u, &ap, bp);
    dfeq(L, i, rho, mu, &am, bm);
    *d_rho = 0.5 * (ap - am);
    for (int k = 0; k < 3; ++k) d_u[k] = 0.5 * (bp[k] + bm[k]);
}

/* ---- grid helpers ---- */

static long node_index(int nx, int ny, int x, int y, int z)
{
    return ((long)z * ny + y) * nx + x;
}

static int wrap(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

/* Upstream neighbour x - v_i with periodic wrap in every axis. */
static long upstream(const lattice_t *L, int nx, int ny, int nz, int x, int y, int z, int i)
{
    return node_index(nx, ny, wrap(x - L->v[i][0], nx), wrap(y - L->v[i][1], ny),
                      wrap(z - L->v[i][2], nz));
}

static void load_u(const lattice_t *L, long n, long idx, const double *u, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    for (int k = 0; k < L->d; ++k) out[k] = u[k * n + idx];
}

static void wall_velocity(const double *wall_u, int n_ids, int m, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    if (wall_u && m >= 0 && m < n_ids)
        for (int k = 0; k < 3; ++k) out[k] = wall_u[3 * m + k];
}

/* Populations f_i(x, t+1), i = 0..q-1, of one fluid node x (Eq. ACM2.0 with
 * the forcing of Eq. force and the bounce-back / moving-wall rules). */
static void node_populations(const lattice_t *L, int nx, int ny, int nz, double omega,
                             const uint8_t *mask, const double *wall_u, int n_ids,
                             const double g[3], double rho0, const double *rho,
                             const double *u, int x, int y, int z, double f[MAXQ],
                             const double *qd, const double *uwl)
{
    long n = (long)nx * ny * nz;
    long ix = node_index(nx, ny, x, y, z);
    double a = 2.0 * (omega - 1.0) / omega;
    double ux[3];
    load_u(L, n, ix, u, ux);
    double rx = rho[ix];
    for (int i = 0; i < L->q; ++i) {
        long iy = upstream(L, nx, ny, nz, x, y, z, i);
        if (!mask || mask[iy] == 0) {
            double uy[3];
            load_u(L, n, iy, u, uy);
            double ry = rho[iy];
            f[i] = feq(L, i, ry, uy) + a * (feo(L, i, rx, ux) - feo(L, i, ry, uy));
        } else {
            /* The upstream node is solid: the population leaving x along
             * BB(i) = ib is reflected back halfway (Eq. ACM2.0ccbb), then
             * post-combined (Eq. ACM2.0cccbb) and corrected for the wall
             * motion (Eq. ACM2.0ccccbb). */
            int ib = L->opp[i];
            double uw[3];
            if (uwl) {
                /* the velocity of the wall where the link x -> x + v_ib
                 * crosses it, given per link (a wall whose velocity varies
                 * along it, e.g. a rotating cylinder) */
                uw[0] = uw[1] = uw[2] = 0.0;
                for (int k = 0; k < L->d; ++k) uw[k] = uwl[((long)ib * L->d + k) * n + ix];
            } else {
                wall_velocity(wall_u, n_ids, mask[iy], uw);
            }
            double fstar = feq(L, ib, rx, ux) - a * feo(L, ib, rx, ux);
            /* Interpolated bounce-back (Eq. ACM2.0cc) when the wall cuts the
             * link x -> x + v_ib at the fraction q of its length (qd, link ib
             * of node x; NULL: q = 1/2, the halfway rule above), and the
             * moving-wall term scaled as in Eq. ACM2.0move: 2 for q < 1/2,
             * 1/q for q >= 1/2.  For q < 1/2 the rule also takes the
             * pre-combined population of the node x - v_ib = x + v_i; when
             * that node is solid as well, the halfway rule is used. */
            double wscale = 2.0;
            if (qd) {
                double q = qd[(long)ib * n + ix];
                if (q < 0.5) {
                    long iz = upstream(L, nx, ny, nz, x, y, z, ib); /* x - v_ib */
                    if (!mask || mask[iz] == 0) {
                        double uz[3];
                        load_u(L, n, iz, u, uz);
                        double rz = rho[iz];
                        double fz = feq(L, ib, rz, uz) - a * feo(L, ib, rz, uz);
                        fstar = 2.0 * q * fstar + (1.0 - 2.0 * q) * fz;
                    }
                } else {
                    double fi = feq(L, i, rx, ux) - a * feo(L, i, rx, ux);
                    fstar = fstar / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * fi;
                    wscale = 1.0 / q;
                }
            }
            f[i] = fstar + a * feo(L, i, rx, ux) + (2.0 / omega - 1.0) * wscale * feo(L, i, rho0, uw);
        }
        if (g) f[i] += feo(L, i, rx, g);
    }
}

/* Number of threads the parallel loops below use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the parallel loops (timing of the oracle). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int make_thermal_lattice(int qt, lattice_t *L);

/* D, velocities, weights and opposite links of lattice q: the flow lattices
 * 9 and 19, and the temperature-only lattices 5 and 7. */
int oracle_lattice_info(int q, int *d, int *v_out, double *w_out, int *opp_out)
{
    lattice_t L;
    if (make_thermal_lattice(q, &L)) return -1;
    *d = L.d;
    for (int i = 0; i < L.q; ++i) {
        for (int k = 0; k < 3; ++k) v_out[3 * i + k] = L.v[i][k];
        w_out[i] = L.w[i];
        opp_out[i] = L.opp[i];
    }
    return 0;
}

/* One LW-ACM time step.  rho_out/u_out must not alias rho_in/u_in
 * (two arrays toggled, Section 2.4). */
int oracle_step(int q, int nx, int ny, int nz, double omega, const uint8_t *mask,
                const double *wall_u, int n_ids, const double *g_in, double rho0,
                const double *rho_in, const double *u_in, double *rho_out, double *u_out)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1)) return -1;
    long n = (long)nx * ny * nz;
    double g[3] = {0, 0, 0};
    if (g_in)
        for (int k = 0; k < L.d; ++k) g[k] = g_in[k];
    const double *gp = g_in ? g : NULL;

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                if (mask && mask[ix] != 0) {
                    rho_out[ix] = rho_in[ix];
                    for (int k = 0; k < L.d; ++k) u_out[k * n + ix] = u_in[k * n + ix];
                    continue;
                }
                double f[MAXQ];
                node_populations(&L, nx, ny, nz, omega, mask, wall_u, n_ids, gp, rho0, rho_in,
                                 u_in, x, y, z, f, NULL, NULL);
                double r = 0.0, j[3] = {0, 0, 0};
                for (int i = 0; i < L.q; ++i) {
                    r += f[i];
                    for (int k = 0; k < 3; ++k) j[k] += L.v[i][k] * f[i];
                }
                rho_out[ix] = r;
                for (int k = 0; k < L.d; ++k) u_out[k * n + ix] = j[k] / r;
            }
    return 0;
}

/* One step with link-wall distances (interpolated bounce-back, Section
 * "Moving complex boundaries", Eqs. ACM2.0cc and ACM2.0move).  qd holds q
 * fields of n values (SoA): qd[j * n + x] is the fraction of the link from
 * the fluid node x to x + v_j at which the wall cuts it, read where x + v_j
 * is solid; NULL gives the halfway rule (q = 1/2) of oracle_step.  uwl, if
 * not NULL, gives the wall velocity link by link in place of the per-id
 * table: D * q fields of n values, uwl[(j * D + k) * n + x] the component k
 * of the velocity of the wall where the link x -> x + v_j crosses it (read
 * where x + v_j is solid).  It enters the moving-wall term of Eq. ACM2.0move
 * as the table's velocity does. */
int oracle_step_qw(int q, int nx, int ny, int nz, double omega, const uint8_t *mask,
                   const double *wall_u, int n_ids, const double *g_in, double rho0,
                   const double *qd, const double *uwl, const double *rho_in,
                   const double *u_in, double *rho_out, double *u_out)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1)) return -1;
    long n = (long)nx * ny * nz;
    double g[3] = {0, 0, 0};
    if (g_in)
        for (int k = 0; k < L.d; ++k) g[k] = g_in[k];
    const double *gp = g_in ? g : NULL;

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                if (mask && mask[ix] != 0) {
                    rho_out[ix] = rho_in[ix];
                    for (int k = 0; k < L.d; ++k) u_out[k * n + ix] = u_in[k * n + ix];
                    continue;
                }
                double f[MAXQ];
                node_populations(&L, nx, ny, nz, omega, mask, wall_u, n_ids, gp, rho0, rho_in,
                                 u_in, x, y, z, f, qd, uwl);
                double r = 0.0, j[3] = {0, 0, 0};
                for (int i = 0; i < L.q; ++i) {
                    r += f[i];
                    for (int k = 0; k < 3; ++k) j[k] += L.v[i][k] * f[i];
                }
                rho_out[ix] = r;
                for (int k = 0; k < L.d; ++k) u_out[k * n + ix] = j[k] / r;
            }
    return 0;
}

/* oracle_step_qw with the wall velocities of the per-id table. */
int oracle_step_q(int q, int nx, int ny, int nz, double omega, const uint8_t *mask,
                  const double *wall_u, int n_ids, const double *g_in, double rho0,
                  const double *qd, const double *rho_in, const double *u_in, double *rho_out,
                  double *u_out)
{
    return oracle_step_qw(q, nx, ny, nz, omega, mask, wall_u, n_ids, g_in, rho0, qd, NULL,
                          rho_in, u_in, rho_out, u_out);
}

/* One step with a body acceleration that varies from node to node (Section
 * "Generalized Taylor-Green vortex flow": a space- and time-dependent
 * external acceleration).  g_field holds D fields of n values (SoA): the
 * acceleration of node x for this step, entering Eq. force with rho(x, t)
 * as the uniform g does. */
int oracle_step_field(int q, int nx, int ny, int nz, double omega, const uint8_t *mask,
                      const double *wall_u, int n_ids, const double *g_field, double rho0,
                      const double *rho_in, const double *u_in, double *rho_out, double *u_out)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1) || !g_field) return -1;
    long n = (long)nx * ny * nz;

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                if (mask && mask[ix] != 0) {
                    rho_out[ix] = rho_in[ix];
                    for (int k = 0; k < L.d; ++k) u_out[k * n + ix] = u_in[k * n + ix];
                    continue;
                }
                double g[3] = {0, 0, 0};
                for (int k = 0; k < L.d; ++k) g[k] = g_field[k * n + ix];
                double f[MAXQ];
                node_populations(&L, nx, ny, nz, omega, mask, wall_u, n_ids, g, rho0, rho_in,
                                 u_in, x, y, z, f, NULL, NULL);
                double r = 0.0, j[3] = {0, 0, 0};
                for (int i = 0; i < L.q; ++i) {
                    r += f[i];
                    for (int k = 0; k < 3; ++k) j[k] += L.v[i][k] * f[i];
                }
                rho_out[ix] = r;
                for (int k = 0; k < L.d; ++k) u_out[k * n + ix] = j[k] / r;
            }
    return 0;
}

/* One step with the semi-implicit pressure update (Section "The main
 * algorithm: Finite difference formulation", item 2, Eq. FDcompact_si): the
 * velocity of the step comes from the explicit update as in oracle_step (or
 * oracle_step_field when g_field is given); the density (pressure p = rho/3)
 * is then the zeroth moment of the Eq. ACM2.0 populations evaluated with the
 * already updated velocity field and the old density, f_p(u+, v+, p): the
 * same function of the stencil's values, with u+ in place of u.  Forcing
 * adds nothing to the density (its odd part sums to zero over the links).
 * Solid nodes keep their values. */
int oracle_step_si(int q, int nx, int ny, int nz, double omega, const uint8_t *mask,
                   const double *wall_u, int n_ids, const double *g_in, const double *g_field,
                   double rho0, const double *rho_in, const double *u_in, double *rho_out,
                   double *u_out)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1)) return -1;
    int rc = g_field ? oracle_step_field(q, nx, ny, nz, omega, mask, wall_u, n_ids, g_field, rho0,
                                         rho_in, u_in, rho_out, u_out)
                     : oracle_step(q, nx, ny, nz, omega, mask, wall_u, n_ids, g_in, rho0, rho_in,
                                   u_in, rho_out, u_out);
    if (rc) return rc;
    /* the pressure from the old density and the new velocity: reads rho_in
     * and u_out only, so rho_out can be written in place */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                if (mask && mask[ix] != 0) continue;
                double f[MAXQ];
                node_populations(&L, nx, ny, nz, omega, mask, wall_u, n_ids, NULL, rho0, rho_in,
                                 u_out, x, y, z, f, NULL, NULL);
                double r = 0.0;
                for (int i = 0; i < L.q; ++i) r += f[i];
                rho_out[ix] = r;
            }
    return 0;
}

/* One step with a separate relaxation omega_p for the density (the
 * continuity equation) and omega for the momentum; omega_p == omega is the
 * step of oracle_step.  The populations are evaluated twice, once with each
 * relaxation: rho = sum f_i(omega_p), rho u = sum v_i f_i(omega). */
int oracle_step_split(int q, int nx, int ny, int nz, double omega, double omega_p,
                      const uint8_t *mask, const double *wall_u, int n_ids, const double *g_in,
                      double rho0, const double *rho_in, const double *u_in, double *rho_out,
                      double *u_out)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1)) return -1;
    if (!(omega_p > 0.0 && omega_p < 2.0)) return -1;
    long n = (long)nx * ny * nz;
    double g[3] = {0, 0, 0};
    if (g_in)
        for (int k = 0; k < L.d; ++k) g[k] = g_in[k];
    const double *gp = g_in ? g : NULL;

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                if (mask && mask[ix] != 0) {
                    rho_out[ix] = rho_in[ix];
                    for (int k = 0; k < L.d; ++k) u_out[k * n + ix] = u_in[k * n + ix];
                    continue;
                }
                double f[MAXQ], fp[MAXQ];
                node_populations(&L, nx, ny, nz, omega, mask, wall_u, n_ids, gp, rho0, rho_in,
                                 u_in, x, y, z, f, NULL, NULL);
                node_populations(&L, nx, ny, nz, omega_p, mask, wall_u, n_ids, gp, rho0, rho_in,
                                 u_in, x, y, z, fp, NULL, NULL);
                double r = 0.0, j[3] = {0, 0, 0};
                for (int i = 0; i < L.q; ++i) {
                    r += fp[i];
                    for (int k = 0; k < 3; ++k) j[k] += L.v[i][k] * f[i];
                }
                rho_out[ix] = r;
                for (int k = 0; k < L.d; ++k) u_out[k * n + ix] = j[k] / r;
            }
    return 0;
}

/* The same update for a list of nodes only (for spot checks of large grids
 * the full-grid loop would be too slow for).  rho_sel/u_sel receive the new
 * state of node idx[k] at position k (u_sel: D values per node). */
int oracle_step_nodes(int q, int nx, int ny, int nz, double omega, const uint8_t *mask,
                      const double *wall_u, int n_ids, const double *g_in, double rho0,
                      const double *rho_in, const double *u_in, const long *idx, long count,
                      double *rho_sel, double *u_sel)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1)) return -1;
    long n = (long)nx * ny * nz;
    double g[3] = {0, 0, 0};
    if (g_in)
        for (int k = 0; k < L.d; ++k) g[k] = g_in[k];
    const double *gp = g_in ? g : NULL;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < count; ++k) {
        long ix = idx[k];
        if (ix < 0 || ix >= n) continue;
        if (mask && mask[ix] != 0) {
            rho_sel[k] = rho_in[ix];
            for (int c = 0; c < L.d; ++c) u_sel[k * L.d + c] = u_in[c * n + ix];
            continue;
        }
        int x = (int)(ix % nx), y = (int)((ix / nx) % ny), z = (int)(ix / ((long)nx * ny));
        double f[MAXQ];
        node_populations(&L, nx, ny, nz, omega, mask, wall_u, n_ids, gp, rho0, rho_in, u_in, x,
                         y, z, f, NULL, NULL);
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < L.q; ++i) {
            r += f[i];
            for (int c = 0; c < 3; ++c) j[c] += L.v[i][c] * f[i];
        }
        rho_sel[k] = r;
        for (int c = 0; c < L.d; ++c) u_sel[k * L.d + c] = j[c] / r;
    }
    return 0;
}

/* ---- FP16 storage with stochastic rounding ---- */

/* pcg2d of Jarzynski and Olano (JCGT 2020): a linear congruential step on
 * each of the two words, then two rounds of "each word adds the other times
 * the LCG multiplier" followed by an xor-shift by 16.  All arithmetic is
 * modulo 2^32.  The map is a bijection of the 64-bit input, so distinct
 * (node, step) counters give distinct output pairs. */
static void pcg2d(uint32_t v[2])
{
    v[0] = v[0] * 1664525u + 1013904223u;
    v[1] = v[1] * 1664525u + 1013904223u;
    for (int round = 0; round < 2; ++round) {
        v[0] += v[1] * 1664525u;
        v[1] += v[0] * 1664525u;
        v[0] ^= v[0] >> 16;
        v[1] ^= v[1] >> 16;
    }
}

/* The random words of the fields of node idx at step word w = t ^ seed:
 * (a, b) = pcg2d(idx, w) and field f draws from word f of
 * (a, b, a << 13, b << 13); the rounding reads only a word's top 13 bits,
 * so the four fields take disjoint bits of a and b. */
static void sr_words(uint32_t idx, uint32_t w, uint32_t out[4])
{
    uint32_t v[2] = {idx, w};
    pcg2d(v);
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[0] << 13;
    out[3] = v[1] << 13;
}

/* Stochastic rounding of the real y to an IEEE half value with random word r.
 * Between the neighbouring half magnitudes lo <= |y| < lo + s (spacing s =
 * 2^(e - 10) for |y| in [2^e, 2^(e+1)), e >= -14; s = 2^-24 below 2^-14),
 * write (|y| - lo)/s = F / 2^13 + rest with F an integer in [0, 2^13) and
 * 0 <= rest < 2^-13 (rest is 0 in the normal range, where an FP32 value has
 * 13 bits below the half spacing); |y| goes to lo + s when
 * F + (r >> 19) >= 2^13.  The variate thus has 13 bits in both ranges and
 * the position is cut to 13 bits: the rounding of gfx950's stochastic
 * FP32 -> FP16 conversion.  Magnitudes above the largest half, 65504,
 * become infinite. */
double oracle_round_fp16_sr(double y, uint32_t r)
{
    double a = fabs(y);
    if (a == 0.0 || isnan(a)) return y;
    double sp;
    if (a < ldexp(1.0, -14)) {
        sp = ldexp(1.0, -24);
    } else {
        int e;
        frexp(a, &e); /* a = m 2^e, m in [1/2, 1): a lies in [2^(e-1), 2^e) */
        sp = ldexp(1.0, e - 1 - 10);
    }
    double lo = floor(a / sp) * sp;
    double F = floor((a - lo) / sp * 8192.0);
    double res = (F + (double)(r >> 19) >= 8192.0) ? lo + sp : lo;
    if (res > 65504.0) res = INFINITY;
    return copysign(res, y);
}

/* Round a state the way the FP16 storage stores the output of step t:
 * rho - 1 scaled by 2^k_rho and each u component scaled by 2^k_u are rounded
 * stochastically, field f of node idx = (z ny + y) nx + x with word f of
 * sr_words(idx, t ^ seed), and scaled back.  In place. */
int oracle_store_fp16_sr(int q, int nx, int ny, int nz, uint32_t t, uint32_t seed, int k_rho,
                         int k_u, double *rho, double *u)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    long n = (long)nx * ny * nz;
    double s_rho = ldexp(1.0, k_rho), s_u = ldexp(1.0, k_u);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                uint32_t h[4];
                sr_words((uint32_t)ix, t ^ seed, h);
                rho[ix] = 1.0 + oracle_round_fp16_sr((rho[ix] - 1.0) * s_rho, h[0]) / s_rho;
                for (int k = 0; k < L.d; ++k)
                    u[k * n + ix] = oracle_round_fp16_sr(u[k * n + ix] * s_u, h[k + 1]) / s_u;
            }
    return 0;
}

/* The four field words of node idx at step word w (for the tests of the
 * generator itself). */
void oracle_sr_words(uint32_t idx, uint32_t w, uint32_t *out)
{
    sr_words(idx, w, out);
}

/* Mass sum(rho) and energy 1/2 sum |u|^2 over fluid nodes. */
int oracle_diagnostics(int q, int nx, int ny, int nz, const uint8_t *mask, const double *rho,
                       const double *u, double *mass, double *energy)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    long n = (long)nx * ny * nz;
    double m = 0.0, e = 0.0;
    for (long ix = 0; ix < n; ++ix) {
        if (mask && mask[ix] != 0) continue;
        m += rho[ix];
        double s = 0.0;
        for (int k = 0; k < L.d; ++k) s += u[k * n + ix] * u[k * n + ix];
        e += 0.5 * s;
    }
    *mass = m;
    *energy = e;
    return 0;
}

/*
 * Reverse mode of one step.  Given the state (rho_t, u_t) entering the step
 * and the cotangents (lam_rho1, lam_u1) of the step's outputs, return the
 * cotangents (lam_rho0, lam_u0) of the inputs and dL/domega of this step.
 *
 * Pass 1, per fluid target x: the cotangent of every population,
 *   fbar_i = dL/d rho+ + dL/d u+ . (v_i - u+) / rho+,
 * then every term of f_i that depends on x itself (post-combine, bounce-back,
 * forcing) is accumulated into x's own input cotangent, and d f_i / d a into
 * a per-node array.  The forcing term enters every f_i (Eq. force), so its
 * rho(x,t)-derivative is carried by fbar_i like the other local terms.
 * Pass 2, per fluid source y: the terms f^(e)_i(y) - a f^(e,o)_i(y) that
 * stream to the fluid target y + v_i.
 * Cotangents of solid nodes are zero (their state never influences a fluid
 * update: bounce-back reads only the fluid node's own state).
 */
int oracle_vjp(int q, int nx, int ny, int nz, double omega, const uint8_t *mask,
               const double *wall_u, int n_ids, const double *g_in, double rho0,
               const double *rho_t, const double *u_t, const double *lam_rho1,
               const double *lam_u1, double *lam_rho0, double *lam_u0, double *dL_domega)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1)) return -1;
    long n = (long)nx * ny * nz;
    double a = 2.0 * (omega - 1.0) / omega;
    double g[3] = {0, 0, 0};
    if (g_in)
        for (int k = 0; k < L.d; ++k) g[k] = g_in[k];
    const double *gp = g_in ? g : NULL;

    double *fbar = (double *)calloc((size_t)L.q * n, sizeof(double));
    double *da = (double *)calloc((size_t)n, sizeof(double));
    if (!fbar || !da) {
        free(fbar);
        free(da);
        return -2;
    }

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                lam_rho0[ix] = 0.0;
                for (int k = 0; k < L.d; ++k) lam_u0[k * n + ix] = 0.0;
                if (mask && mask[ix] != 0) continue;
                double f[MAXQ];
                node_populations(&L, nx, ny, nz, omega, mask, wall_u, n_ids, gp, rho0, rho_t,
                                 u_t, x, y, z, f, NULL, NULL);
                double r = 0.0, j[3] = {0, 0, 0};
                for (int i = 0; i < L.q; ++i) {
                    r += f[i];
                    for (int k = 0; k < 3; ++k) j[k] += L.v[i][k] * f[i];
                }
                double up[3] = {j[0] / r, j[1] / r, j[2] / r};
                double lr = lam_rho1[ix];
                double lu[3] = {0, 0, 0};
                for (int k = 0; k < L.d; ++k) lu[k] = lam_u1[k * n + ix];

                double ux[3];
                load_u(&L, n, ix, u_t, ux);
                double rx = rho_t[ix];
                double acc_r = 0.0, acc_u[3] = {0, 0, 0}, acc_a = 0.0;
                for (int i = 0; i < L.q; ++i) {
                    double fb = lr;
                    for (int k = 0; k < 3; ++k) fb += lu[k] * (L.v[i][k] - up[k]) / r;
                    fbar[(size_t)i * n + ix] = fb;

                    double dr, du[3];
                    /* post-combine term a f^(e,o)_i(x) (present for both cases) */
                    dfeo(&L, i, rx, ux, &dr, du);
                    acc_r += fb * a * dr;
                    for (int k = 0; k < 3; ++k) acc_u[k] += fb * a * du[k];
                    acc_a += fb * feo(&L, i, rx, ux);

                    long iy = upstream(&L, nx, ny, nz, x, y, z, i);
                    if (!mask || mask[iy] == 0) {
                        double uy[3];
                        load_u(&L, n, iy, u_t, uy);
                        acc_a -= fb * feo(&L, i, rho_t[iy], uy);
                    } else {
                        int ib = L.opp[i];
                        double uw[3];
                        wall_velocity(wall_u, n_ids, mask[iy], uw);
                        double er, eu[3], orr, ou[3];
                        dfeq(&L, ib, rx, ux, &er, eu);
                        dfeo(&L, ib, rx, ux, &orr, ou);
                        acc_r += fb * (er - a * orr);
                        for (int k = 0; k < 3; ++k) acc_u[k] += fb * (eu[k] - a * ou[k]);
                        /* d/da of [-a f^(e,o)_ib(x) + (2/omega - 1) 2 f^(e,o)_i(rho0,uw)]
                         * with 2/omega - 1 = 1 - a */
                        acc_a += fb * (-feo(&L, ib, rx, ux) - 2.0 * feo(&L, i, rho0, uw));
                    }
                    if (gp) {
                        /* forcing term f^(e,o)_i(rho(x,t), g): linear in rho(x,t) */
                        double gr, gu[3];
                        dfeo(&L, i, rx, g, &gr, gu);
                        acc_r += fb * gr;
                    }
                }
                lam_rho0[ix] += acc_r;
                for (int k = 0; k < L.d; ++k) lam_u0[k * n + ix] += acc_u[k];
                da[ix] = acc_a;
            }

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long iy = node_index(nx, ny, x, y, z);
                if (mask && mask[iy] != 0) continue;
                double uy[3];
                load_u(&L, n, iy, u_t, uy);
                double ry = rho_t[iy];
                double acc_r = 0.0, acc_u[3] = {0, 0, 0};
                for (int i = 0; i < L.q; ++i) {
                    long ixt = node_index(nx, ny, wrap(x + L.v[i][0], nx), wrap(y + L.v[i][1], ny),
                                          wrap(z + L.v[i][2], nz));
                    if (mask && mask[ixt] != 0) continue;
                    double fb = fbar[(size_t)i * n + ixt];
                    double er, eu[3], orr, ou[3];
                    dfeq(&L, i, ry, uy, &er, eu);
                    dfeo(&L, i, ry, uy, &orr, ou);
                    acc_r += fb * (er - a * orr);
                    for (int k = 0; k < 3; ++k) acc_u[k] += fb * (eu[k] - a * ou[k]);
                }
                lam_rho0[iy] += acc_r;
                for (int k = 0; k < L.d; ++k) lam_u0[k * n + iy] += acc_u[k];
            }

    double s = 0.0;
    for (long ix = 0; ix < n; ++ix) s += da[ix];
    *dL_domega = s * 2.0 / (omega * omega); /* a = 2 - 2/omega, da/domega = 2/omega^2 */
    free(fbar);
    free(da);
    return 0;
}

/* ---- thermal LW-ACM: a temperature lattice advected by the flow ----
 *
 * Appendix "Asymptotic analysis for energy equation", Eqs. ACM2.0t and
 * feqe.  The temperature lattice is the flow's (Q_t = Q) or, as the appendix
 * allows (Q_t != Q), the rest link and the axis links alone: D2Q5 under a
 * D2Q9 flow, D3Q7 under a D3Q19 flow.  Its only state is T at every node.
 * The velocity u in its equilibria is the flow velocity at the same node and
 * time (the flow is not influenced by T).
 */

/* Temperature lattices: D2Q9 and D3Q19 as the flow's; D2Q5 (rest and the
 * four axis links of D2Q9, weights 1/3, 1/6) and D3Q7 (rest and the six
 * axis links of D3Q19, weights 0, 1/6).  The second moment T/3 I that the
 * appendix requires fixes the axis weight at 1/6 (sum_i w_i v_i v_i =
 * 2 w_axis I), and the weights sum to one; D3Q7 then has no rest weight. */
static int make_thermal_lattice(int qt, lattice_t *L)
{
    if (qt == 9 || qt == 19) return make_lattice(qt, L);
    if (qt != 5 && qt != 7) return -1;
    if (make_lattice(qt == 5 ? 9 : 19, L)) return -1;
    lattice_t A = *L;
    int k = 0;
    for (int i = 0; i < A.q; ++i) {
        int nz = (A.v[i][0] != 0) + (A.v[i][1] != 0) + (A.v[i][2] != 0);
        if (nz > 1) continue; /* keep the rest and the axis links, in order */
        for (int c = 0; c < 3; ++c) L->v[k][c] = A.v[i][c];
        L->w[k] = (nz == 0) ? (qt == 5 ? 1.0 / 3.0 : 0.0) : 1.0 / 6.0;
        ++k;
    }
    if (k != qt) return -1;
    L->q = qt;
    L->lin = 1;
    for (int i = 0; i < L->q; ++i) {
        L->opp[i] = -1;
        for (int j = 0; j < L->q; ++j)
            if (L->v[j][0] == -L->v[i][0] && L->v[j][1] == -L->v[i][1] &&
                L->v[j][2] == -L->v[i][2])
                L->opp[i] = j;
        if (L->opp[i] < 0) return -1;
    }
    return 0;
}

/* g_i^(e)(T, u): the function of T and u whose moments are the ones the
 * appendix requires -- sum_i g = T, sum_i v_i g = T u and
 * sum_i v_i v_i g = u u + T/3 I -- written with the lattice's weights as
 * w_i [T (1 + 3 v_i.u) + 4.5 (v_i.u)^2 - 1.5 |u|^2] on D2Q9 and D3Q19.
 * D2Q5 and D3Q7 cannot carry the u u part (their v_i v_i have no
 * off-diagonal components, and no quadratic term has both the diagonal
 * u_a^2 and a zero sum); under the appendix's diffusive scaling (Eq.
 * scaling2t) that part is O(eps^2), so on those lattices the equilibrium is
 * the linear one, w_i T (1 + 3 v_i.u), with the moments T, T u and T/3 I. */
static double geq(const lattice_t *L, int i, double T, const double u[3])
{
    double c = vdot(L, i, u);
    if (L->lin) return L->w[i] * T * (1.0 + 3.0 * c);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->w[i] * (T * (1.0 + 3.0 * c) + 4.5 * c * c - 1.5 * uu);
}

/* Even part, Eq. feqe: the mean of g^(e) at +u and at -u. */
static double gee(const lattice_t *L, int i, double T, const double u[3])
{
    double mu[3] = {-u[0], -u[1], -u[2]};
    return 0.5 * (geq(L, i, T, u) + geq(L, i, T, mu));
}

/* g^(e)_i(T, u) and g^(e,e)_i(T, u) for i = 0..q-1 of the temperature
 * lattice q (5, 7, 9 or 19; pinned in the tests against the moments the
 * appendix requires). */
int oracle_thermal_equilibrium(int q, double T, const double *u_in, double *g_out,
                               double *gee_out)
{
    lattice_t L;
    if (make_thermal_lattice(q, &L)) return -1;
    double u[3] = {0, 0, 0};
    for (int k = 0; k < L.d; ++k) u[k] = u_in[k];
    for (int i = 0; i < L.q; ++i) {
        g_out[i] = geq(&L, i, T, u);
        gee_out[i] = gee(&L, i, T, u);
    }
    return 0;
}

/*
 * One step of the temperature lattice, Eq. ACM2.0t:
 *   g_i(x, t+1) = g^(e)_i(x - v_i) + (2 - 2/omega_t) (g^(e,e)_i(x) - g^(e,e)_i(x - v_i)),
 *   T(x, t+1)   = sum_i g_i(x, t+1),
 * on the temperature lattice q (5, 7, 9 or 19; D2Q5 and D2Q9 need nz = 1),
 * with T(., t) from T_in and u(., t) the flow velocity (D fields, SoA).
 *
 * Walls (the paper gives no thermal wall rule; this is the oracle's reading,
 * built like the flow's halfway rule): where x - v_i is solid, the term
 * g^(e)_ib(x) - (2 - 2/omega_t) g^(e,e)_ib(x) that x sends along ib = BB(i)
 * into the wall comes back along i, with its sign kept for an adiabatic wall
 * (bounce-back: no flux of T through the wall), or with its sign reversed
 * plus (2/omega_t - 1) * 2 w_i T_w for a wall held at temperature T_w
 * (anti-bounce-back, the same factor as the flow's moving-wall term); the
 * own term (2 - 2/omega_t) g^(e,e)_i(x) is added as in the interior.
 * wall_T[m] is the temperature of the walls with mask id m (0 <= m < n_ids);
 * NaN, an id >= n_ids or wall_T == NULL mean adiabatic.  Solid nodes keep
 * their T.
 */
int oracle_thermal_step(int q, int nx, int ny, int nz, double omega_t, const uint8_t *mask,
                        const double *wall_T, int n_ids, const double *T_in, const double *u,
                        double *T_out)
{
    lattice_t L;
    if (make_thermal_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1)) return -1;
    if (!(omega_t > 0.0 && omega_t < 2.0)) return -1;
    long n = (long)nx * ny * nz;
    double k = 2.0 * (omega_t - 1.0) / omega_t;

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                if (mask && mask[ix] != 0) {
                    T_out[ix] = T_in[ix];
                    continue;
                }
                double ux[3];
                load_u(&L, n, ix, u, ux);
                double Tx = T_in[ix];
                double sum = 0.0;
                for (int i = 0; i < L.q; ++i) {
                    long iy = upstream(&L, nx, ny, nz, x, y, z, i);
                    double gi;
                    if (!mask || mask[iy] == 0) {
                        double uy[3];
                        load_u(&L, n, iy, u, uy);
                        double Ty = T_in[iy];
                        gi = geq(&L, i, Ty, uy) + k * (gee(&L, i, Tx, ux) - gee(&L, i, Ty, uy));
                    } else {
                        int ib = L.opp[i];
                        double sent = geq(&L, ib, Tx, ux) - k * gee(&L, ib, Tx, ux);
                        double Tw = NAN;
                        if (wall_T && mask[iy] < n_ids) Tw = wall_T[mask[iy]];
                        if (isnan(Tw))
                            gi = sent;
                        else
                            gi = -sent + (2.0 / omega_t - 1.0) * 2.0 * L.w[i] * Tw;
                        gi += k * gee(&L, i, Tx, ux);
                    }
                    sum += gi;
                }
                T_out[ix] = sum;
            }
    return 0;
}

/* Derivatives of g^(e)_i and g^(e,e)_i with respect to T and to u
 * (componentwise), term by term from geq and gee. */
static void dgeq(const lattice_t *L, int i, double T, const double u[3], double *dT,
                 double du[3], double *deT, double deu[3])
{
    double c = vdot(L, i, u);
    *dT = L->w[i] * (1.0 + 3.0 * c);
    *deT = L->w[i];
    for (int k = 0; k < 3; ++k) {
        /* d/du_k of 4.5 c^2 - 1.5 |u|^2 (zero on the linear lattices) */
        double dq = L->lin ? 0.0 : 9.0 * c * L->v[i][k] - 3.0 * u[k];
        du[k] = L->w[i] * (3.0 * T * L->v[i][k] + dq);
        /* gee = (geq(u) + geq(-u)) / 2 keeps the even terms: T and the quadratic */
        deu[k] = L->w[i] * dq;
    }
}

/*
 * Reverse mode of one temperature step (not in the paper: the exact
 * derivative of oracle_thermal_step with respect to its inputs T and u, by
 * the chain rule through the same terms).  lam holds dL/dT(., t+1); the
 * outputs are lamT = dL/dT(., t) and lamU = dL/du(., t) (D fields, SoA)
 * through this step alone.  A solid node's T is copied through, so its
 * lamT is its lam; its u is never read (lamU = 0).
 */
int oracle_thermal_vjp(int q, int nx, int ny, int nz, double omega_t, const uint8_t *mask,
                       const double *wall_T, int n_ids, const double *T_in, const double *u,
                       const double *lam, double *lamT, double *lamU)
{
    lattice_t L;
    if (make_thermal_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1)) return -1;
    if (!(omega_t > 0.0 && omega_t < 2.0)) return -1;
    long n = (long)nx * ny * nz;
    double k = 2.0 * (omega_t - 1.0) / omega_t;
    for (long ix = 0; ix < n; ++ix) lamT[ix] = 0.0;
    for (long j = 0; j < (long)L.d * n; ++j) lamU[j] = 0.0;

    /* Serial scatter: every output T(x, t+1) adds its cotangent times the
     * derivative of each of its link terms to the inputs that term reads. */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                if (mask && mask[ix] != 0) {
                    lamT[ix] += lam[ix];
                    continue;
                }
                double ux[3];
                load_u(&L, n, ix, u, ux);
                double Tx = T_in[ix];
                double lx = lam[ix];
                for (int i = 0; i < L.q; ++i) {
                    long iy = upstream(&L, nx, ny, nz, x, y, z, i);
                    double dT, du[3], deT, deu[3];
                    /* the own even part k g^(e,e)_i(x), in both branches */
                    dgeq(&L, i, Tx, ux, &dT, du, &deT, deu);
                    lamT[ix] += lx * k * deT;
                    for (int c = 0; c < L.d; ++c) lamU[c * n + ix] += lx * k * deu[c];
                    if (!mask || mask[iy] == 0) {
                        /* g^(e)_i(y) - k g^(e,e)_i(y) */
                        double uy[3];
                        load_u(&L, n, iy, u, uy);
                        dgeq(&L, i, T_in[iy], uy, &dT, du, &deT, deu);
                        lamT[iy] += lx * (dT - k * deT);
                        for (int c = 0; c < L.d; ++c) lamU[c * n + iy] += lx * (du[c] - k * deu[c]);
                    } else {
                        /* +- (g^(e)_ib(x) - k g^(e,e)_ib(x)): the term sent into the wall */
                        int ib = L.opp[i];
                        double Tw = NAN;
                        if (wall_T && mask[iy] < n_ids) Tw = wall_T[mask[iy]];
                        double sgn = isnan(Tw) ? 1.0 : -1.0;
                        dgeq(&L, ib, Tx, ux, &dT, du, &deT, deu);
                        lamT[ix] += lx * sgn * (dT - k * deT);
                        for (int c = 0; c < L.d; ++c)
                            lamU[c * n + ix] += lx * sgn * (du[c] - k * deu[c]);
                    }
                }
            }
    return 0;
}

/*
 * Force and torque on the walls with mask id wall_id by momentum exchange
 * (Section "Moving complex boundaries", Eqs. MEA3, MEA4 and MEA5), from the
 * state (rho, u) at time t.  For every link j from a fluid node x to a solid
 * node x + v_j of that id,
 *   p_j = v_j [f*_j(x, t) + f**_BB(j)(x, t+1)],
 * f*_j = f^(e)_j - (2 - 2/omega) f^(e,o)_j at x (the population x sends into
 * the wall) and f**_BB(j) the population the wall returns along BB(j) before
 * post-combining: f*_j itself for the halfway rule, the interpolation of Eq.
 * ACM2.0cc with qd[j * n + x] when qd is given (the same rule as
 * oracle_step_q).  The paper restricts the formula to bodies at rest; the
 * returned population here excludes the wall-motion term.
 * F = sum p_j, T = sum (x - x_c) x p_j, x being the node the link starts from
 * (coordinates are node indices); out = (F_x, F_y, F_z, T_x, T_y, T_z).
 */
int oracle_wall_force(int q, int nx, int ny, int nz, double omega, const uint8_t *mask,
                      const double *qd, const double *rho, const double *u, int wall_id,
                      const double xc[3], double out[6])
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0 || (L.d == 2 && nz != 1) || !mask || wall_id < 1) return -1;
    long n = (long)nx * ny * nz;
    double a = 2.0 * (omega - 1.0) / omega;
    for (int k = 0; k < 6; ++k) out[k] = 0.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long ix = node_index(nx, ny, x, y, z);
                if (mask[ix] != 0) continue;
                double ux[3];
                load_u(&L, n, ix, u, ux);
                double rx = rho[ix];
                for (int j = 0; j < L.q; ++j) {
                    /* x + v_j is x - v_BB(j) */
                    int i = L.opp[j];
                    long iw = upstream(&L, nx, ny, nz, x, y, z, i);
                    if (mask[iw] != wall_id) continue;
                    double fs = feq(&L, j, rx, ux) - a * feo(&L, j, rx, ux);
                    double fb = fs;
                    if (qd) {
                        double qq = qd[(long)j * n + ix];
                        if (qq < 0.5) {
                            long iz = upstream(&L, nx, ny, nz, x, y, z, j); /* x - v_j */
                            if (mask[iz] == 0) {
                                double uz[3];
                                load_u(&L, n, iz, u, uz);
                                double fz = feq(&L, j, rho[iz], uz) - a * feo(&L, j, rho[iz], uz);
                                fb = 2.0 * qq * fs + (1.0 - 2.0 * qq) * fz;
                            }
                        } else {
                            double fi = feq(&L, i, rx, ux) - a * feo(&L, i, rx, ux);
                            fb = fs / (2.0 * qq) + (1.0 - 1.0 / (2.0 * qq)) * fi;
                        }
                    }
                    double p[3];
                    for (int k = 0; k < 3; ++k) p[k] = L.v[j][k] * (fs + fb);
                    double r[3] = {x - xc[0], y - xc[1], z - xc[2]};
                    for (int k = 0; k < 3; ++k) out[k] += p[k];
                    out[3] += r[1] * p[2] - r[2] * p[1];
                    out[4] += r[2] * p[0] - r[0] * p[2];
                    out[5] += r[0] * p[1] - r[1] * p[0];
                }
            }
    return 0;
}
