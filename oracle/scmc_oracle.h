/*
 * scmc_oracle.h -- plain FP64 CPU oracle of the two-component Shan-Chen
 * lattice Boltzmann step and of its pressure-tensor observables
 * (Lulli, Biferale, Falcucci, Sbragaglia, Shan, "Mesoscale Modelling of the
 * Tolman Length in Multi-component Systems", arXiv:2112.02574).
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the HIP library
 * against the paper.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Conventions of this oracle (they are its own; the GPU library documents its
 * own):
 *   - site index s = (z*ny + y)*nx + x, x fastest; nz = 1 in 2D.
 *   - populations f[(J*Q + i)*N + s], J in {0 = A, 1 = B}.
 *   - the state at integer time t is the post-streaming, pre-collision set
 *     f_i^J(x, t) of the lattice transport equation (Sec. 2, eq. lbm).
 *   - couplings g[J][K] are the products G_JK c_s^2 that multiply the
 *     isotropic stencil sums in the force (Sec. 2, eq. sc_force); the
 *     cross coupling is g[0][1] = g[1][0] = G c_s^2.
 *   - every array is caller-owned; nothing is retained between calls.
 */
#ifndef SCMC_ORACLE_H
#define SCMC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int dim;          /* 2 -> D2Q9, 3 -> D3Q19 */
    int stencil;      /* isotropy order of the force stencil: 4, 6 or 8 */
    int nx, ny, nz;   /* periodic box; nz must be 1 when dim == 2 */
    double tau[2];    /* BGK relaxation times tau_A, tau_B */
    double g[2][2];   /* G_JK c_s^2 */
    int psi_self;     /* self-interaction pseudopotential: 0 -> psi = n,
                         1 -> psi = exp(-1/n); the cross term always uses n */
    int nthreads;     /* OpenMP threads, <= 0 -> library default */
} orc_problem;

/* Velocity set of the lattice: fills xi[Q*3] (integer components stored as
 * doubles) and w[Q]; returns Q (9 or 19) or -1 for a bad dim. */
int orc_lattice(int dim, double *xi, double *w);

/* Force stencil of the given isotropy order: fills e[n*3] and W[n];
 * returns the number of neighbours n, or -1 if the pair is unsupported. */
int orc_stencil(int dim, int order, int *e, double *W);

/* 0 if the problem is usable, -1 otherwise. */
int orc_check(const orc_problem *p);

/* Local operators at one node (Sec. 2). */
void orc_equilibrium(int dim, double n, const double *u, double *feq);
void orc_guo_source(int dim, const double *u, const double *F, double *S);

/* Field operators. n[2*N], F[2*3*N] (component, axis, site), u[3*N]. */
void orc_init_equilibrium(const orc_problem *p, const double *nA,
                          const double *nB, double *f);
void orc_density(const orc_problem *p, const double *f, double *n);
void orc_pseudopotential(const orc_problem *p, const double *n, double *psi);
void orc_force(const orc_problem *p, const double *n, double *F);
void orc_velocity(const orc_problem *p, const double *f, const double *n,
                  const double *F, double *u);

/* Advance nsteps.  f[2*Q*N] holds the state and is overwritten; work[2*Q*N +
 * 2*N + 6*N + 3*N] is scratch.  Returns 0. */
int orc_run(const orc_problem *p, double *f, long nsteps, double *work);
long orc_work_doubles(const orc_problem *p);

/* Post-collision populations f*(x) at one site, computed from the full
 * pre-collision state f by reading only the site's neighbourhood.
 * out[2*Q]. */
void orc_collide_site(const orc_problem *p, const double *f, long site,
                      double *out);

/* Lattice pressure tensor (Sec. 2, eq. sm:pt) at one site, from the density
 * field n[2*N]; out[6] = xx, yy, zz, xy, xz, yz. */
void orc_pressure_tensor_site(const orc_problem *p, const double *n, long site,
                              double *out);

/* Bulk pressure (Sec. 2, eq. bulkp) of a uniform state. */
double orc_bulk_pressure(const orc_problem *p, double nA, double nB);

/* Droplet observables at the current state (Sec. 3 and Sec. 4):
 * obs[0] P_in, [1] P_out, [2] dP, [3] C_d, [4] R_s closed form,
 * [5] R_s from the grid minimum of sigma[R], [6] sigma_s = dP R_s / (d-1),
 * [7] sigma[R] at the grid minimum, [8] max |P^yy - P^zz| on the line (3D).
 * PN, PT (nullable) receive P^xx and P^yy at r = 0..L/2 along +x from the
 * centre node.  R0 sets the grid [R0/2, 2 R0] of the sigma[R] scan. */
int orc_droplet_observables(const orc_problem *p, const double *f, double R0,
                            double *obs, double *PN, double *PT);

/* Shell-averaged variant: PN, PT (nullable, floor(min extent / 2) + 1
 * values) are the means of u.P.u and (tr P - u.P.u)/(d-1) over the shells
 * k = floor(|x - c| + 1/2); obs as orc_droplet_observables, obs[8] = 0. */
int orc_shell_observables(const orc_problem *p, const double *f, double R0,
                          double *obs, double *PN, double *PT);

/* Flat-interface profiles: PN[x], PT[x] = P^xx, P^yy averaged over y (and z);
 * returns sigma0 = sum_{x = nx/2}^{nx-1} (PN - PT). */
double orc_flat_sigma0(const orc_problem *p, const double *f, double *PN,
                       double *PT);

/* Global statistics: out[0..1] mass of A, B; [2..4] momentum
 * sum_x sum_J (sum_i f xi + F/2); [5..6] min n_A, n_B; [7] max |u|;
 * [8] number of non-finite populations. */
void orc_stats(const orc_problem *p, const double *f, double *out);

#ifdef __cplusplus
}
#endif
#endif
