/*
 * Drives every entry point of the oracle on small 2D and 3D boxes, for the
 * sanitizer test (tests/test_oracle_sanitizers.py builds it together with
 * oracle/scmc_oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer).
 * Every array is sized exactly as the oracle's header states, so any access
 * outside one, any leak and any undefined operation ends the run with a
 * sanitizer report and a non-zero status.  Prints "ok" on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/scmc_oracle.h"

static double *alloc(long n)
{
    double *a = (double *)calloc((size_t)n, sizeof(double));
    if (!a) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return a;
}

/* a droplet of radius R between two phases, plus a little deterministic
 * texture so that no tensor component vanishes */
static void droplet(const orc_problem *p, double R, double *nA, double *nB)
{
    int x, y, z, nz = p->dim == 3 ? p->nz : 1;
    for (z = 0; z < nz; z++)
        for (y = 0; y < p->ny; y++)
            for (x = 0; x < p->nx; x++) {
                long s = ((long)z * p->ny + y) * p->nx + x;
                double dx = x - p->nx / 2 + 0.3, dy = y - p->ny / 2 - 0.2;
                double dz = p->dim == 3 ? z - nz / 2 + 0.1 : 0.0;
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                double t = tanh(r - R), e = 0.01 * sin(0.7 * s);
                nA[s] = 0.55 - 0.45 * t + e;
                nB[s] = 0.55 + 0.45 * t - e;
            }
}

static int exercise(int dim, int stencil, int psi, int nx, int ny, int nz)
{
    orc_problem p = {0};
    long N, Q, s;
    double *nA, *nB, *f, *work, *n, *psiv, *F, *u, *out, *P6, obs[9], *PN, *PT;
    double xi[57], w[19], feq[19], S[19], uu[3] = {0.01, -0.02, 0.005};
    double FF[3] = {1e-3, 2e-3, -1e-3}, st[9];
    int e[3 * 64], k, rmax, len;
    double W[64];
    p.dim = dim;
    p.stencil = stencil;
    p.nx = nx;
    p.ny = ny;
    p.nz = dim == 3 ? nz : 1;
    p.tau[0] = 1.0;
    p.tau[1] = 0.8;
    p.g[0][0] = psi ? -1.0 : -0.2;
    p.g[0][1] = p.g[1][0] = psi ? 0.5 : 1.8;
    p.g[1][1] = psi ? -0.6 : 0.0;
    p.psi_self = psi;
    p.nthreads = 1;
    if (orc_check(&p) != 0) return 1;
    Q = orc_lattice(dim, xi, w);
    if (Q != (dim == 3 ? 19 : 9)) return 1;
    if (orc_stencil(dim, stencil, e, W) <= 0) return 1;
    orc_equilibrium(dim, 1.0, uu, feq);
    orc_guo_source(dim, uu, FF, S);
    N = (long)p.nx * p.ny * p.nz;
    nA = alloc(N);
    nB = alloc(N);
    f = alloc(2 * Q * N);
    work = alloc(orc_work_doubles(&p));
    n = alloc(2 * N);
    psiv = alloc(2 * N);
    F = alloc(2 * 3 * N);
    u = alloc(3 * N);
    out = alloc(2 * Q);
    P6 = alloc(6);
    droplet(&p, 3.0, nA, nB);
    orc_init_equilibrium(&p, nA, nB, f);
    if (orc_run(&p, f, 5, work) != 0) return 1;
    orc_density(&p, f, n);
    orc_pseudopotential(&p, n, psiv);
    orc_force(&p, n, F);
    orc_velocity(&p, f, n, F, u);
    for (s = 0; s < N; s += N / 7 + 1) {
        orc_collide_site(&p, f, s, out);
        orc_pressure_tensor_site(&p, n, s, P6);
    }
    (void)orc_bulk_pressure(&p, 0.7, 0.3);
    len = p.nx / 2 + 1;
    PN = alloc(len);
    PT = alloc(len);
    if (orc_droplet_observables(&p, f, 3.0, obs, PN, PT) != 0) return 1;
    free(PN);
    free(PT);
    rmax = p.nx < p.ny ? p.nx : p.ny;
    if (dim == 3 && p.nz < rmax) rmax = p.nz;
    len = rmax / 2 + 1;
    PN = alloc(len);
    PT = alloc(len);
    if (orc_shell_observables(&p, f, 3.0, obs, PN, PT) != 0) return 1;
    free(PN);
    free(PT);
    PN = alloc(p.nx);
    PT = alloc(p.nx);
    (void)orc_flat_sigma0(&p, f, PN, PT);
    free(PN);
    free(PT);
    orc_stats(&p, f, st);
    for (k = 0; k < 9; k++)
        if (!(st[k] == st[k])) return 1;
    free(nA);
    free(nB);
    free(f);
    free(work);
    free(n);
    free(psiv);
    free(F);
    free(u);
    free(out);
    free(P6);
    return 0;
}

int main(void)
{
    static const int cases[][6] = {
        /* dim, stencil, psi, nx, ny, nz */
        {2, 4, 0, 13, 11, 1}, {2, 6, 1, 12, 14, 1}, {2, 8, 0, 17, 15, 1},
        {3, 4, 1, 9, 8, 10},  {3, 6, 0, 11, 9, 10},
    };
    unsigned c;
    for (c = 0; c < sizeof cases / sizeof cases[0]; c++)
        if (exercise(cases[c][0], cases[c][1], cases[c][2], cases[c][3], cases[c][4],
                     cases[c][5]) != 0) {
            printf("case %u failed\n", c);
            return 1;
        }
    printf("ok\n");
    return 0;
}
