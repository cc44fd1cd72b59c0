/*
 * scmc_oracle.c -- plain FP64 CPU oracle of the two-component Shan-Chen
 * lattice Boltzmann method of arXiv:2112.02574 (Sec. 2 and Sec. 3).
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this code.  It is written to be read against the
 * paper, not to be fast: every step follows the order in which the paper
 * states it, in double precision, with no fusion or reordering beyond that.
 * OpenMP only splits the site loops among threads.
 *
 * One time step, from the pre-collision state f(x, t):
 *   1. concentrations n_J = sum_i f_i^J                         (Sec. 2)
 *   2. Shan-Chen force F_J from n and psi at the stencil nodes  (eq. sc_force)
 *   3. common velocity n u = sum_J [sum_i f_i^J xi_i + F_J / 2] (Guo velocity)
 *   4. BGK collision with Guo forcing                           (eq. lbm,
 *      eq. sm:omega_i, equilibrium and forcing term of Sec. 2)
 *   5. streaming f_i(x + xi_i, t + 1) = f*_i(x, t), periodic box (eq. lbm)
 */
#include "scmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0) /* c_s^2 of D2Q9 and D3Q19 (Sec. 4) */
#define INV_CS2 3.0      /* 1 / c_s^2 */
#define INV_CS4 9.0      /* 1 / c_s^4 */
#define HALF_INV_CS4 4.5 /* 1 / (2 c_s^4) */
#define MAXQ 19
#define MAXE 64

/* ------------------------------------------------------------------------ */
/* Lattice tables (Sec. 2: D3Q19 with c_s^2 = 1/3; D2Q9 is its 2D analogue) */

static const int D2Q9_XI[9][3] = {
    {0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double D2Q9_W[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,
                                 1.0 / 9,  1.0 / 9,  1.0 / 36,
                                 1.0 / 36, 1.0 / 36, 1.0 / 36};

static const int D3Q19_XI[19][3] = {
    {0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},   {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double D3Q19_W[19] = {
    1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

int orc_lattice(int dim, double *xi, double *w)
{
    int q, i, a;
    if (dim == 2) q = 9;
    else if (dim == 3) q = 19;
    else return -1;
    for (i = 0; i < q; i++) {
        for (a = 0; a < 3; a++)
            xi[3 * i + a] = dim == 2 ? D2Q9_XI[i][a] : D3Q19_XI[i][a];
        w[i] = dim == 2 ? D2Q9_W[i] : D3Q19_W[i];
    }
    return q;
}

/* Force-stencil weight of a vector with squared length s.  The E4 weights
 * are the ones of Sec. 2 (W(1) = 1/6, W(2) = 1/12 in 3D); their 2D analogue
 * and the E6 / E8 sets solve the isotropy conditions with
 * e2 = sum_a W_a (e_a^x)^2 = 1 (the normalisation stated after eq. bulkp). */
static double stencil_weight(int dim, int order, int s)
{
    if (dim == 3 && order == 4) {
        if (s == 1) return 1.0 / 6;
        if (s == 2) return 1.0 / 12;
        return 0.0;
    }
    if (dim == 3 && order == 6) {
        if (s == 1) return 2.0 / 15;
        if (s == 2) return 1.0 / 15;
        if (s == 3) return 1.0 / 60;
        if (s == 4) return 1.0 / 120;
        return 0.0;
    }
    if (dim == 2 && order == 4) {
        if (s == 1) return 1.0 / 3;
        if (s == 2) return 1.0 / 12;
        return 0.0;
    }
    if (dim == 2 && order == 6) {
        if (s == 1) return 4.0 / 15;
        if (s == 2) return 1.0 / 10;
        if (s == 4) return 1.0 / 120;
        return 0.0;
    }
    if (dim == 2 && order == 8) {
        if (s == 1) return 4.0 / 21;
        if (s == 2) return 4.0 / 45;
        if (s == 4) return 1.0 / 60;
        if (s == 5) return 2.0 / 315;
        if (s == 8) return 1.0 / 5040;
        return 0.0;
    }
    return -1.0;
}

int orc_stencil(int dim, int order, int *e, double *W)
{
    int n = 0, x, y, z, zr;
    if (dim != 2 && dim != 3) return -1;
    if (stencil_weight(dim, order, 1) < 0) return -1;
    zr = dim == 3 ? 2 : 0;
    for (z = -zr; z <= zr; z++)
        for (y = -2; y <= 2; y++)
            for (x = -2; x <= 2; x++) {
                int s = x * x + y * y + z * z;
                double wt;
                if (s == 0) continue;
                wt = stencil_weight(dim, order, s);
                if (wt == 0.0) continue;
                e[3 * n] = x;
                e[3 * n + 1] = y;
                e[3 * n + 2] = z;
                W[n] = wt;
                n++;
            }
    return n;
}

int orc_check(const orc_problem *p)
{
    int e[3 * MAXE];
    double W[MAXE];
    if (p->dim != 2 && p->dim != 3) return -1;
    if (p->dim == 2 && p->nz != 1) return -1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    if (orc_stencil(p->dim, p->stencil, e, W) < 0) return -1;
    if (!(p->tau[0] > 0.5) || !(p->tau[1] > 0.5)) return -1;
    if (p->psi_self != 0 && p->psi_self != 1) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Helpers                                                                   */

static int nq(const orc_problem *p) { return p->dim == 2 ? 9 : 19; }
static long nsites(const orc_problem *p)
{
    return (long)p->nx * p->ny * p->nz;
}
static int wrap(int a, int n) { return ((a % n) + n) % n; }
static long site_of(const orc_problem *p, int x, int y, int z)
{
    return ((long)z * p->ny + y) * p->nx + x;
}
static void coords_of(const orc_problem *p, long s, int *x, int *y, int *z)
{
    *x = (int)(s % p->nx);
    *y = (int)((s / p->nx) % p->ny);
    *z = (int)(s / ((long)p->nx * p->ny));
}
static long shifted(const orc_problem *p, long s, int dx, int dy, int dz)
{
    int x, y, z;
    coords_of(p, s, &x, &y, &z);
    return site_of(p, wrap(x + dx, p->nx), wrap(y + dy, p->ny),
                   wrap(z + dz, p->nz));
}
static void set_threads(const orc_problem *p)
{
#ifdef _OPENMP
    if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#else
    (void)p;
#endif
}

/* Tables and periodic-wrap lookups shared by the site loops of one call:
 * wx[(d + 2) * nx + x] = (x + d) mod nx for d = -2..2 (same for y, z). */
typedef struct {
    int q, ne;
    double xi[3 * MAXQ], w[MAXQ];
    int e[3 * MAXE];
    double W[MAXE];
    int *wx, *wy, *wz;
} ctx_t;

static int ctx_init(const orc_problem *p, ctx_t *c)
{
    int d, a;
    c->q = orc_lattice(p->dim, c->xi, c->w);
    c->ne = orc_stencil(p->dim, p->stencil, c->e, c->W);
    c->wx = (int *)malloc(sizeof(int) * 5 * p->nx);
    c->wy = (int *)malloc(sizeof(int) * 5 * p->ny);
    c->wz = (int *)malloc(sizeof(int) * 5 * p->nz);
    if (!c->wx || !c->wy || !c->wz) return -1;
    for (d = -2; d <= 2; d++) {
        for (a = 0; a < p->nx; a++) c->wx[(d + 2) * p->nx + a] = wrap(a + d, p->nx);
        for (a = 0; a < p->ny; a++) c->wy[(d + 2) * p->ny + a] = wrap(a + d, p->ny);
        for (a = 0; a < p->nz; a++) c->wz[(d + 2) * p->nz + a] = wrap(a + d, p->nz);
    }
    return 0;
}

static void ctx_free(ctx_t *c)
{
    free(c->wx);
    free(c->wy);
    free(c->wz);
}

/* site of (x, y, z) + (dx, dy, dz), periodic; |d| <= 2 */
static long nb_site(const orc_problem *p, const ctx_t *c, int x, int y, int z,
                    int dx, int dy, int dz)
{
    return ((long)c->wz[(dz + 2) * p->nz + z] * p->ny +
            c->wy[(dy + 2) * p->ny + y]) * p->nx +
           c->wx[(dx + 2) * p->nx + x];
}

/* psi for the self term (Sec. 2 and Sec. 4): n or exp(-1/n). */
static double psi_self(const orc_problem *p, double n)
{
    return p->psi_self == 1 ? exp(-1.0 / n) : n;
}

/* ------------------------------------------------------------------------ */
/* Local operators                                                           */

/* Second-order equilibrium (Sec. 2):
 * f_i^eq = n w_i [1 + xi.u / cs2 + ((xi.u)^2 - cs2 u.u) / (2 cs2^2)]. */
static void equilibrium_q(int q, const double *xi, const double *w, double n,
                          const double *u, double *feq)
{
    int i;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (i = 0; i < q; i++) {
        double xu = xi[3 * i] * u[0] + xi[3 * i + 1] * u[1] +
                    xi[3 * i + 2] * u[2];
        feq[i] = n * w[i] *
                 (1.0 + xu / CS2 + (xu * xu - CS2 * uu) / (2.0 * CS2 * CS2));
    }
}

/* Guo forcing term (Sec. 2):
 * S_i = w_i [xi^b / cs2 + (xi^a xi^b - cs2 delta^ab) u_a / cs2^2] F^b
 *     = w_i [xi.F / cs2 + ((xi.u)(xi.F) - cs2 u.F) / cs2^2]. */
static void guo_q(int q, const double *xi, const double *w, const double *u,
                  const double *F, double *S)
{
    int i;
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    for (i = 0; i < q; i++) {
        double xu = xi[3 * i] * u[0] + xi[3 * i + 1] * u[1] +
                    xi[3 * i + 2] * u[2];
        double xF = xi[3 * i] * F[0] + xi[3 * i + 1] * F[1] +
                    xi[3 * i + 2] * F[2];
        S[i] = w[i] * (xF / CS2 + (xu * xF - CS2 * uF) / (CS2 * CS2));
    }
}

void orc_equilibrium(int dim, double n, const double *u, double *feq)
{
    double xi[3 * MAXQ], w[MAXQ];
    int q = orc_lattice(dim, xi, w);
    equilibrium_q(q, xi, w, n, u, feq);
}

void orc_guo_source(int dim, const double *u, const double *F, double *S)
{
    double xi[3 * MAXQ], w[MAXQ];
    int q = orc_lattice(dim, xi, w);
    guo_q(q, xi, w, u, F, S);
}

/* ------------------------------------------------------------------------ */
/* Field operators                                                           */

void orc_init_equilibrium(const orc_problem *p, const double *nA,
                          const double *nB, double *f)
{
    double xi[3 * MAXQ], w[MAXQ];
    int q = orc_lattice(p->dim, xi, w), i;
    long N = nsites(p), s;
    for (i = 0; i < q; i++)
        for (s = 0; s < N; s++) {
            f[(0 * q + i) * N + s] = w[i] * nA[s];
            f[(1 * q + i) * N + s] = w[i] * nB[s];
        }
}

void orc_density(const orc_problem *p, const double *f, double *n)
{
    int q = nq(p);
    long N = nsites(p), s;
    set_threads(p);
#pragma omp parallel for schedule(static)
    for (s = 0; s < N; s++) {
        int J, i;
        for (J = 0; J < 2; J++) {
            double acc = 0.0;
            for (i = 0; i < q; i++) acc += f[(J * q + i) * N + s];
            n[J * N + s] = acc;
        }
    }
}

void orc_pseudopotential(const orc_problem *p, const double *n, double *psi)
{
    long N = nsites(p), s;
    for (s = 0; s < 2 * N; s++) psi[s] = psi_self(p, n[s]);
}

/* Shan-Chen force at (x, y, z) (eq. sc_force):
 * F_J = - g_JK n_J(x) sum_a W_a n_K(x + e_a) e_a      (K != J, cross term)
 *       - g_JJ psi_J(x) sum_a W_a psi_J(x + e_a) e_a  (self term).
 * Densities are read from the field n[2*N]. */
static void force_at(const orc_problem *p, const ctx_t *c, const double *n,
                     int x, int y, int z, double *FA, double *FB)
{
    long N = nsites(p), s = site_of(p, x, y, z);
    int a, k, J;
    double sum_cross[2][3] = {{0, 0, 0}, {0, 0, 0}};
    double sum_self[2][3] = {{0, 0, 0}, {0, 0, 0}};
    double nA = n[s], nB = n[N + s];
    for (a = 0; a < c->ne; a++) {
        const int *e = &c->e[3 * a];
        long t = nb_site(p, c, x, y, z, e[0], e[1], e[2]);
        for (J = 0; J < 2; J++) {
            int K = 1 - J;
            double nK = n[K * N + t];
            double psJ = psi_self(p, n[J * N + t]);
            for (k = 0; k < 3; k++) {
                sum_cross[J][k] += c->W[a] * nK * e[k];
                sum_self[J][k] += c->W[a] * psJ * e[k];
            }
        }
    }
    for (k = 0; k < 3; k++) {
        FA[k] = -p->g[0][1] * nA * sum_cross[0][k] -
                p->g[0][0] * psi_self(p, nA) * sum_self[0][k];
        FB[k] = -p->g[1][0] * nB * sum_cross[1][k] -
                p->g[1][1] * psi_self(p, nB) * sum_self[1][k];
    }
}

void orc_force(const orc_problem *p, const double *n, double *F)
{
    ctx_t c;
    long N = nsites(p);
    int z;
    if (ctx_init(p, &c) != 0) return;
    set_threads(p);
#pragma omp parallel for schedule(static)
    for (z = 0; z < p->nz; z++) {
        int y, x, k;
        for (y = 0; y < p->ny; y++)
            for (x = 0; x < p->nx; x++) {
                double FA[3], FB[3];
                long s = site_of(p, x, y, z);
                force_at(p, &c, n, x, y, z, FA, FB);
                for (k = 0; k < 3; k++) {
                    F[(0 * 3 + k) * N + s] = FA[k];
                    F[(1 * 3 + k) * N + s] = FB[k];
                }
            }
    }
    ctx_free(&c);
}

/* Common velocity (Guo velocity of Sec. 2):
 * (n_A + n_B) u = sum_J [sum_i f_i^J xi_i + F_J / 2].
 * With tau_A != tau_B (which the paper does not use) each component is
 * weighted by 1 / tau_J:
 * sum_J n_J / tau_J u = sum_J [sum_i f_i^J xi_i + F_J / 2] / tau_J,
 * the velocity for which the BGK relaxations of the two components change
 * the total momentum by exactly sum_J F_J. */
static void velocity_site(const orc_problem *p, const ctx_t *c,
                          const double *f, const double *n, const double *FA,
                          const double *FB, long s, double *u)
{
    int i, J, k;
    long N = nsites(p);
    double mom[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (J = 0; J < 2; J++)
        for (i = 0; i < c->q; i++)
            for (k = 0; k < 3; k++)
                mom[J][k] += f[(J * c->q + i) * N + s] * c->xi[3 * i + k];
    for (k = 0; k < 3; k++) {
        if (p->tau[0] == p->tau[1]) {
            u[k] = (mom[0][k] + mom[1][k] + 0.5 * FA[k] + 0.5 * FB[k]) /
                   (n[s] + n[N + s]);
        } else {
            double num = (mom[0][k] + 0.5 * FA[k]) / p->tau[0] +
                         (mom[1][k] + 0.5 * FB[k]) / p->tau[1];
            double den = n[s] / p->tau[0] + n[N + s] / p->tau[1];
            u[k] = num / den;
        }
    }
}

void orc_velocity(const orc_problem *p, const double *f, const double *n,
                  const double *F, double *u)
{
    ctx_t c;
    long N = nsites(p), s;
    if (ctx_init(p, &c) != 0) return;
    set_threads(p);
#pragma omp parallel for schedule(static)
    for (s = 0; s < N; s++) {
        double FA[3], FB[3], us[3];
        int k;
        for (k = 0; k < 3; k++) {
            FA[k] = F[(0 * 3 + k) * N + s];
            FB[k] = F[(1 * 3 + k) * N + s];
        }
        velocity_site(p, &c, f, n, FA, FB, s, us);
        for (k = 0; k < 3; k++) u[k * N + s] = us[k];
    }
    ctx_free(&c);
}

/* BGK collision with Guo forcing for both components at one site
 * (eq. lbm with eq. sm:omega_i):
 * f*_i = f_i - (f_i - f_i^eq(n_J, u)) / tau_J + (1 - 1/(2 tau_J)) S_i(u, F_J). */
static void collide_site(const orc_problem *p, const ctx_t *c,
                         const double *f, const double *n, const double *FA,
                         const double *FB, long s, double *out)
{
    int q = c->q, i, J;
    long N = nsites(p);
    double u[3], feq[MAXQ], S[MAXQ];
    velocity_site(p, c, f, n, FA, FB, s, u);
    for (J = 0; J < 2; J++) {
        equilibrium_q(q, c->xi, c->w, n[J * N + s], u, feq);
        guo_q(q, c->xi, c->w, u, J == 0 ? FA : FB, S);
        for (i = 0; i < q; i++) {
            double fi = f[(J * q + i) * N + s];
            out[J * q + i] = fi - (fi - feq[i]) / p->tau[J] +
                             (1.0 - 1.0 / (2.0 * p->tau[J])) * S[i];
        }
    }
}

long orc_work_doubles(const orc_problem *p)
{
    long N = nsites(p);
    return 2L * nq(p) * N + 4L * N;
}

/* dst[(x + ex) mod nx] = row[x] for one lattice row, |ex| <= 1 */
static void store_shifted_row(double *dst, const double *row, int nx, int ex)
{
    int x;
    if (nx <= 1 || ex == 0) {
        for (x = 0; x < nx; x++) dst[wrap(x + ex, nx)] = row[x];
        return;
    }
    if (ex > 0) {
        for (x = 0; x < nx - 1; x++) dst[x + 1] = row[x];
        dst[0] = row[nx - 1];
    } else {
        for (x = 1; x < nx; x++) dst[x - 1] = row[x];
        dst[nx - 1] = row[0];
    }
}

/* One time step over the lattice, row by row (x innermost).  For every site
 * the arithmetic is the one of force_at / velocity_site / collide_site: the
 * stencil sums run over the neighbours in the same order, then the force,
 * the common velocity, the equilibrium, the Guo term and the BGK update. */
static void step_rows(const orc_problem *p, const ctx_t *c, const double *f,
                      const double *n, const double *psi, double *fnew)
{
    long N = nsites(p);
    int nx = p->nx, q = c->q;
    long nrows = (long)p->ny * p->nz;
    double omegas[2] = {1.0 / p->tau[0], 1.0 / p->tau[1]};
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 26 * nx);
        /* buf rows: sums[J][kind][k] (12 rows: kind 0 = cross, 1 = self),
         * F[J][k] (6), u[k] (3), tot (1), out (1), one component's
         * momentum (3, unequal tau only) */
        double *sums = buf, *F = buf + 12 * nx, *u = buf + 18 * nx;
        double *tot = buf + 21 * nx;
        long r;
#pragma omp for schedule(static)
        for (r = 0; r < nrows; r++) {
            int y = (int)(r % p->ny), z = (int)(r / p->ny);
            int x, a, k, J, i;
            long row = r * nx;
            for (x = 0; x < 21 * nx; x++) buf[x] = 0.0;
            /* stencil sums of eq. sc_force: for every neighbour a, in
             * order, sums[J][cross][k] += W_a e_a^k n_K(x + e_a) and
             * sums[J][self][k] += W_a e_a^k psi_J(x + e_a) */
            for (a = 0; a < c->ne; a++) {
                const int *e = &c->e[3 * a];
                long nrow = ((long)c->wz[(e[2] + 2) * p->nz + z] * p->ny +
                             c->wy[(e[1] + 2) * p->ny + y]) * nx;
                const double *nAr = n + nrow, *nBr = n + N + nrow;
                const double *pAr = psi + nrow, *pBr = psi + N + nrow;
                const int *xs = c->wx + (e[0] + 2) * nx;
                for (k = 0; k < 3; k++) {
                    const double cw = c->W[a] * e[k];
                    double *restrict sAc = sums + (0 * 3 + k) * nx;
                    double *restrict sAs = sums + (1 * 3 + k) * nx;
                    double *restrict sBc = sums + (2 * 3 + k) * nx;
                    double *restrict sBs = sums + (3 * 3 + k) * nx;
                    if (e[k] == 0) continue;
                    for (x = 0; x < nx; x++) {
                        int t = xs[x];
                        sAc[x] += cw * nBr[t];
                        sAs[x] += cw * pAr[t];
                        sBc[x] += cw * nAr[t];
                        sBs[x] += cw * pBr[t];
                    }
                }
            }
            /* force F_J = -g_JK n_J S_cross - g_JJ psi_J S_self */
            for (J = 0; J < 2; J++)
                for (k = 0; k < 3; k++)
                    for (x = 0; x < nx; x++)
                        F[(J * 3 + k) * nx + x] =
                            -p->g[J][1 - J] * n[J * N + row + x] *
                                sums[((J * 2 + 0) * 3 + k) * nx + x] -
                            p->g[J][J] * psi[J * N + row + x] *
                                sums[((J * 2 + 1) * 3 + k) * nx + x];
            /* common velocity (velocity_site) */
            if (p->tau[0] == p->tau[1]) {
                for (J = 0; J < 2; J++)
                    for (i = 0; i < q; i++)
                        for (k = 0; k < 3; k++) {
                            double xk = c->xi[3 * i + k];
                            const double *fr = f + (J * q + i) * N + row;
                            if (xk == 0.0) continue;
                            for (x = 0; x < nx; x++) u[k * nx + x] += fr[x] * xk;
                        }
                for (x = 0; x < nx; x++)
                    tot[x] = n[row + x] + n[N + row + x];
                for (k = 0; k < 3; k++)
                    for (x = 0; x < nx; x++)
                        u[k * nx + x] = (u[k * nx + x] + 0.5 * F[k * nx + x] +
                                         0.5 * F[(3 + k) * nx + x]) / tot[x];
            } else {
                /* each component's momentum + F_J / 2 and density over tau_J */
                for (x = 0; x < nx; x++)
                    tot[x] = n[row + x] / p->tau[0] + n[N + row + x] / p->tau[1];
                for (J = 0; J < 2; J++) {
                    double *mJ = buf + 23 * nx; /* 3 rows: 23..25 */
                    for (x = 0; x < 3 * nx; x++) mJ[x] = 0.0;
                    for (i = 0; i < q; i++)
                        for (k = 0; k < 3; k++) {
                            double xk = c->xi[3 * i + k];
                            const double *fr = f + (J * q + i) * N + row;
                            if (xk == 0.0) continue;
                            for (x = 0; x < nx; x++) mJ[k * nx + x] += fr[x] * xk;
                        }
                    for (k = 0; k < 3; k++)
                        for (x = 0; x < nx; x++)
                            u[k * nx + x] += (mJ[k * nx + x] + 0.5 * F[(J * 3 + k) * nx + x]) /
                                             p->tau[J];
                }
                for (k = 0; k < 3; k++)
                    for (x = 0; x < nx; x++) u[k * nx + x] /= tot[x];
            }
            /* collision and streaming */
            for (J = 0; J < 2; J++)
                for (i = 0; i < q; i++) {
                    const double *xi = &c->xi[3 * i];
                    const double *fr = f + (J * q + i) * N + row;
                    const double *nJ = n + J * N + row;
                    const double *FJ = F + J * 3 * nx;
                    const double wi = c->w[i];
                    const double omega = omegas[J];
                    const double x0 = xi[0], x1 = xi[1], x2 = xi[2];
                    long drow =
                        ((long)c->wz[((int)x2 + 2) * p->nz + z] * p->ny +
                         c->wy[((int)x1 + 2) * p->ny + y]) * nx;
                    double *dst = fnew + (J * q + i) * N + drow;
                    double *restrict orow = buf + 22 * nx;
                    for (x = 0; x < nx; x++) {
                        double ux = u[x], uy = u[nx + x], uz = u[2 * nx + x];
                        double Fx = FJ[x], Fy = FJ[nx + x], Fz = FJ[2 * nx + x];
                        double uu = ux * ux + uy * uy + uz * uz;
                        double xu = x0 * ux + x1 * uy + x2 * uz;
                        double xF = x0 * Fx + x1 * Fy + x2 * Fz;
                        double uF = ux * Fx + uy * Fy + uz * Fz;
                        double feq = nJ[x] * wi *
                                     (1.0 + xu * INV_CS2 +
                                      (xu * xu - CS2 * uu) * HALF_INV_CS4);
                        double S = wi * (xF * INV_CS2 +
                                         (xu * xF - CS2 * uF) * INV_CS4);
                        double out = fr[x] - (fr[x] - feq) * omega +
                                     (1.0 - 0.5 * omega) * S;
                        orow[x] = out;
                    }
                    store_shifted_row(dst, orow, nx, (int)xi[0]);
                }
        }
        free(buf);
    }
}

int orc_run(const orc_problem *p, double *f, long nsteps, double *work)
{
    ctx_t c;
    long N = nsites(p), t, s;
    double *fnew = work, *n, *psi;
    if (orc_check(p) != 0) return -1;
    if (ctx_init(p, &c) != 0) return -1;
    n = work + 2L * c.q * N;
    psi = n + 2L * N;
    set_threads(p);
    for (t = 0; t < nsteps; t++) {
        double *cur = (t % 2 == 0) ? f : fnew;         /* ping-pong */
        double *nxt = (t % 2 == 0) ? fnew : f;
        orc_density(p, cur, n);                        /* step 1 */
#pragma omp parallel for schedule(static)
        for (s = 0; s < 2 * N; s++) psi[s] = psi_self(p, n[s]);
        step_rows(p, &c, cur, n, psi, nxt);            /* steps 2-5 */
    }
    if (nsteps % 2 == 1) memcpy(f, fnew, sizeof(double) * 2L * c.q * N);
    ctx_free(&c);
    return 0;
}

/* Concentrations at one site straight from the populations. */
static void density_at(const orc_problem *p, const double *f, long s,
                       double *nA, double *nB)
{
    int q = nq(p), i;
    long N = nsites(p);
    double a = 0.0, b = 0.0;
    for (i = 0; i < q; i++) {
        a += f[(0 * q + i) * N + s];
        b += f[(1 * q + i) * N + s];
    }
    *nA = a;
    *nB = b;
}

void orc_collide_site(const orc_problem *p, const double *f, long s,
                      double *out)
{
    /* Same operators as orc_run, on a density field that holds correct
     * values only at s and at its stencil neighbours. */
    ctx_t c;
    long N = nsites(p);
    int a, x, y, z;
    double *n = (double *)calloc(2 * N, sizeof(double));
    double FA[3], FB[3];
    if (!n || ctx_init(p, &c) != 0) return;
    coords_of(p, s, &x, &y, &z);
    density_at(p, f, s, &n[s], &n[N + s]);
    for (a = 0; a < c.ne; a++) {
        long t = nb_site(p, &c, x, y, z, c.e[3 * a], c.e[3 * a + 1],
                         c.e[3 * a + 2]);
        density_at(p, f, t, &n[t], &n[N + t]);
    }
    force_at(p, &c, n, x, y, z, FA, FB);
    collide_site(p, &c, f, n, FA, FB, s, out);
    ctx_free(&c);
    free(n);
}

/* ------------------------------------------------------------------------ */
/* Pressure tensor and observables                                           */

/* Lattice pressure tensor (eq. sm:pt):
 * P^mn = (n_A + n_B) cs2 delta^mn
 *      + (g_AB / 2) [n_A sum_a W n_B(x+e) e^m e^n + n_B sum_a W n_A(x+e) e^m e^n]
 *      + sum_J (g_JJ / 2) psi_J sum_a W psi_J(x+e) e^m e^n. */
void orc_pressure_tensor_site(const orc_problem *p, const double *n, long s,
                              double *out)
{
    static const int MU[6] = {0, 1, 2, 0, 0, 1};
    static const int NU[6] = {0, 1, 2, 1, 2, 2};
    int e[3 * MAXE];
    double W[MAXE];
    int ne = orc_stencil(p->dim, p->stencil, e, W), a, k;
    long N = nsites(p);
    double nA = n[s], nB = n[N + s];
    double psA = psi_self(p, nA), psB = psi_self(p, nB);
    for (k = 0; k < 6; k++) {
        double cross_AB = 0.0, cross_BA = 0.0, selfA = 0.0, selfB = 0.0;
        for (a = 0; a < ne; a++) {
            long t = shifted(p, s, e[3 * a], e[3 * a + 1], e[3 * a + 2]);
            double ee = (double)e[3 * a + MU[k]] * e[3 * a + NU[k]];
            cross_AB += W[a] * n[N + t] * ee;
            cross_BA += W[a] * n[t] * ee;
            selfA += W[a] * psi_self(p, n[t]) * ee;
            selfB += W[a] * psi_self(p, n[N + t]) * ee;
        }
        out[k] = (MU[k] == NU[k] ? (nA + nB) * CS2 : 0.0) +
                 0.5 * p->g[0][1] * nA * cross_AB +
                 0.5 * p->g[1][0] * nB * cross_BA +
                 0.5 * p->g[0][0] * psA * selfA +
                 0.5 * p->g[1][1] * psB * selfB;
    }
}

/* Bulk pressure (eq. bulkp) with e2 = 1:
 * P = (n_A + n_B) cs2 + g_AB n_A n_B + (g_AA / 2) psi_A^2 + (g_BB / 2) psi_B^2. */
double orc_bulk_pressure(const orc_problem *p, double nA, double nB)
{
    double psA = psi_self(p, nA), psB = psi_self(p, nB);
    return (nA + nB) * CS2 + p->g[0][1] * nA * nB +
           0.5 * p->g[0][0] * psA * psA + 0.5 * p->g[1][1] * psB * psB;
}

/* Droplet analysis (Sec. 3, eq. gen_sigma, and Sec. 4) from a nodal
 * profile PTr[r], r = 0..rmax, of the tangential pressure.
 * With P_J(r;R) = P_in - dP theta(r - R), the Heaviside part of
 * sigma[R] = int_0^inf (r/R)^(d-1) [P_J(r;R) - P_T(r)] dr integrates exactly,
 * leaving sigma[R] = C_d / R^(d-1) + dP R / d with
 * C_d = int_0^inf r^(d-1) (P_out - P_T(r)) dr, where P_T between lattice
 * nodes is the linear interpolant of its nodal values.
 * Its minimum is R_s = (d (d-1) C_d / dP)^(1/d), where the Laplace law
 * dP = (d-1) sigma_s / R_s holds.  The grid scan locates the same minimum
 * numerically as an independent check of that algebra.  obs[0..7] as
 * orc_droplet_observables. */
static void sigma_from_profile(int d, double Pin, double Pout, const double *PTr,
                               int rmax, double R0, double *obs)
{
    double dP = Pin - Pout, Cd = 0.0, Rs, best = 1e300, Rbest;
    int r, k, nR, kbest = -1;
    double *sig;
    /* C_d = int_0^rmax r^(d-1) g(r) dr with g the piecewise-linear
     * interpolant of P_out - P_T between the lattice nodes, integrated
     * exactly on every interval [k, k+1] */
    for (r = 0; r < rmax; r++) {
        double a = r, b = r + 1.0, m = d - 1;
        double g0 = Pout - PTr[r], g1 = Pout - PTr[r + 1];
        double I0 = (pow(b, m + 1) - pow(a, m + 1)) / (m + 1);
        double I1 = (pow(b, m + 2) - pow(a, m + 2)) / (m + 2) - a * I0;
        Cd += g0 * I0 + (g1 - g0) * I1;
    }
    Rs = pow(d * (d - 1) * Cd / dP, 1.0 / d);
    /* grid scan of sigma[R] on [R0/2, 2 R0] in steps of 0.01 */
    nR = (int)floor((2.0 * R0 - 0.5 * R0) / 0.01) + 1;
    sig = (double *)malloc(sizeof(double) * nR);
    for (k = 0; k < nR; k++) {
        double R = 0.5 * R0 + 0.01 * k;
        sig[k] = Cd / pow(R, d - 1) + dP * R / d;
        if (sig[k] < best) {
            best = sig[k];
            kbest = k;
        }
    }
    Rbest = 0.5 * R0 + 0.01 * kbest;
    if (kbest > 0 && kbest < nR - 1) {
        /* vertex of the parabola through the minimum and its neighbours */
        double ym = sig[kbest - 1], y0 = sig[kbest], yp = sig[kbest + 1];
        double den = ym - 2.0 * y0 + yp;
        if (den != 0.0) Rbest += 0.01 * 0.5 * (ym - yp) / den;
    }
    free(sig);
    obs[0] = Pin;
    obs[1] = Pout;
    obs[2] = dP;
    obs[3] = Cd;
    obs[4] = Rs;
    obs[5] = Rbest;
    obs[6] = dP * Rs / (d - 1);
    obs[7] = best;
}

/* The probes of the droplet analysis: bulk pressure (eq. bulkp) at the centre
 * node c = floor(L/2) and at (c + floor(L/2)) mod L. */
static void pressure_probes(const orc_problem *p, const double *n, double *Pin,
                            double *Pout)
{
    long N = nsites(p);
    int d = p->dim, cx = p->nx / 2, cy = p->ny / 2, cz = d == 3 ? p->nz / 2 : 0;
    long sc = site_of(p, cx, cy, cz);
    long so = site_of(p, (cx + p->nx / 2) % p->nx, (cy + p->ny / 2) % p->ny,
                      d == 3 ? (cz + p->nz / 2) % p->nz : 0);
    *Pin = orc_bulk_pressure(p, n[sc], n[N + sc]);
    *Pout = orc_bulk_pressure(p, n[so], n[N + so]);
}

/* The axis line (Sec. 3): P_N = P^xx and P_T = P^yy at the nodes
 * r = 0..nx/2 along +x from the centre node; obs[8] = max |P^yy - P^zz| on
 * the line (3D). */
int orc_droplet_observables(const orc_problem *p, const double *f, double R0,
                            double *obs, double *PN, double *PT)
{
    int d = p->dim, r, rmax;
    long N = nsites(p);
    int cx = p->nx / 2, cy = p->ny / 2, cz = d == 3 ? p->nz / 2 : 0;
    double *n = (double *)malloc(sizeof(double) * 2 * N);
    double Pin, Pout, maxdiff = 0.0, *pt;
    if (!n) return -1;
    orc_density(p, f, n);
    pressure_probes(p, n, &Pin, &Pout);
    rmax = p->nx / 2;
    pt = (double *)malloc(sizeof(double) * (rmax + 1));
    for (r = 0; r <= rmax; r++) {
        double P6[6];
        long s = site_of(p, (cx + r) % p->nx, cy, cz);
        orc_pressure_tensor_site(p, n, s, P6);
        if (PN) PN[r] = P6[0];
        if (PT) PT[r] = P6[1];
        if (d == 3 && fabs(P6[1] - P6[2]) > maxdiff)
            maxdiff = fabs(P6[1] - P6[2]);
        pt[r] = P6[1];
    }
    sigma_from_profile(d, Pin, Pout, pt, rmax, R0, obs);
    obs[8] = maxdiff;
    free(pt);
    free(n);
    return 0;
}

/* Shell-averaged pressure profiles (a variant of the axis line, not the
 * paper's definition).  Every node x at distance r = |x - c| from the centre
 * node c (no periodic image: x - c in [-floor(L/2), L - 1 - floor(L/2)])
 * belongs to shell k = floor(r + 1/2).  There, with the unit vector
 * u = (x - c) / r, the normal and tangential pressures are
 *   P_N = u . P . u,   P_T = (tr P - P_N) / (d - 1),
 * and P_N = P_T = tr P / d at the centre node.  PN[k], PT[k] are their means
 * over shell k for k = 0..rmax, rmax = floor(min extent / 2) (the largest
 * shell that every axis still reaches), and the droplet analysis runs on PT
 * as on the axis line.  obs[8] = the largest standard deviation of P_T within
 * a shell. */
int orc_shell_observables(const orc_problem *p, const double *f, double R0,
                          double *obs, double *PN, double *PT)
{
    int d = p->dim, x, y, z, k, rmax;
    long N = nsites(p);
    int cx = p->nx / 2, cy = p->ny / 2, cz = d == 3 ? p->nz / 2 : 0;
    int nz = d == 3 ? p->nz : 1;
    double *n = (double *)malloc(sizeof(double) * 2 * N);
    double *sn, *st, *cnt, *pt, Pin, Pout;
    if (!n) return -1;
    rmax = p->nx < p->ny ? p->nx : p->ny;
    if (d == 3 && p->nz < rmax) rmax = p->nz;
    rmax /= 2;
    sn = (double *)calloc(rmax + 1, sizeof(double));
    st = (double *)calloc(rmax + 1, sizeof(double));
    cnt = (double *)calloc(rmax + 1, sizeof(double));
    pt = (double *)malloc(sizeof(double) * (rmax + 1));
    orc_density(p, f, n);
    pressure_probes(p, n, &Pin, &Pout);
    for (z = 0; z < nz; z++)
        for (y = 0; y < p->ny; y++)
            for (x = 0; x < p->nx; x++) {
                double P6[6], v[3], r2, r, tr, pn, ptv;
                v[0] = x - cx;
                v[1] = y - cy;
                v[2] = d == 3 ? z - cz : 0.0;
                r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                r = sqrt(r2);
                k = (int)floor(r + 0.5);
                if (k > rmax) continue;
                orc_pressure_tensor_site(p, n, site_of(p, x, y, z), P6);
                tr = P6[0] + P6[1] + (d == 3 ? P6[2] : 0.0);
                if (r2 == 0.0) {
                    pn = tr / d;
                } else {
                    /* u . P . u with P symmetric: P6 = xx, yy, zz, xy, xz, yz */
                    pn = (v[0] * v[0] * P6[0] + v[1] * v[1] * P6[1] +
                          v[2] * v[2] * P6[2] + 2.0 * v[0] * v[1] * P6[3] +
                          2.0 * v[0] * v[2] * P6[4] + 2.0 * v[1] * v[2] * P6[5]) / r2;
                }
                ptv = (tr - pn) / (d - 1);
                sn[k] += pn;
                st[k] += ptv;
                cnt[k] += 1.0;
            }
    for (k = 0; k <= rmax; k++) {
        pt[k] = st[k] / cnt[k];
        if (PN) PN[k] = sn[k] / cnt[k];
        if (PT) PT[k] = pt[k];
    }
    sigma_from_profile(d, Pin, Pout, pt, rmax, R0, obs);
    obs[8] = 0.0;
    free(sn);
    free(st);
    free(cnt);
    free(pt);
    free(n);
    return 0;
}

/* Flat interface (Sec. 4): sigma0 = int_{Lx/2}^{Lx} [P_N(x) - P_T(x)] dx with
 * P_N = P^xx and P_T = P^yy averaged over the transverse directions; the
 * integral is the sum over the nodes x = nx/2 .. nx-1. */
double orc_flat_sigma0(const orc_problem *p, const double *f, double *PN,
                       double *PT)
{
    long N = nsites(p);
    double *n = (double *)malloc(sizeof(double) * 2 * N);
    double sigma0 = 0.0;
    int x, y, z;
    orc_density(p, f, n);
    for (x = 0; x < p->nx; x++) {
        double pn = 0.0, pt = 0.0;
        for (z = 0; z < p->nz; z++)
            for (y = 0; y < p->ny; y++) {
                double P6[6];
                orc_pressure_tensor_site(p, n, site_of(p, x, y, z), P6);
                pn += P6[0];
                pt += P6[1];
            }
        pn /= (double)p->ny * p->nz;
        pt /= (double)p->ny * p->nz;
        if (PN) PN[x] = pn;
        if (PT) PT[x] = pt;
        if (x >= p->nx / 2) sigma0 += pn - pt;
    }
    free(n);
    return sigma0;
}

void orc_stats(const orc_problem *p, const double *f, double *out)
{
    int q = nq(p), c;
    long N = nsites(p), s, bad = 0;
    double *n = (double *)malloc(sizeof(double) * 2 * N);
    double *F = (double *)malloc(sizeof(double) * 6 * N);
    double *u = (double *)malloc(sizeof(double) * 3 * N);
    double mA = 0, mB = 0, mom[3] = {0, 0, 0}, minA = 1e300, minB = 1e300;
    double umax = 0.0;
    orc_density(p, f, n);
    orc_force(p, n, F);
    orc_velocity(p, f, n, F, u);
    for (s = 0; s < 2L * q * N; s++)
        if (!isfinite(f[s])) bad++;
    for (s = 0; s < N; s++) {
        double un = 0.0;
        mA += n[s];
        mB += n[N + s];
        if (n[s] < minA) minA = n[s];
        if (n[N + s] < minB) minB = n[N + s];
        for (c = 0; c < 3; c++) {
            /* sum_J (sum_i f_i^J xi_i + F_J / 2), which the step conserves
             * (with equal tau it is (n_A + n_B) u) */
            double m = 0.5 * (F[c * N + s] + F[(3 + c) * N + s]);
            int J, i;
            for (J = 0; J < 2; J++)
                for (i = 0; i < q; i++)
                    m += f[(J * q + i) * N + s] *
                         (p->dim == 2 ? D2Q9_XI[i][c] : D3Q19_XI[i][c]);
            mom[c] += m;
            un += u[c * N + s] * u[c * N + s];
        }
        if (sqrt(un) > umax) umax = sqrt(un);
    }
    out[0] = mA;
    out[1] = mB;
    out[2] = mom[0];
    out[3] = mom[1];
    out[4] = mom[2];
    out[5] = minA;
    out[6] = minB;
    out[7] = umax;
    out[8] = (double)bad;
    free(n);
    free(F);
    free(u);
}
