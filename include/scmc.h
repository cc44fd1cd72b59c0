/*
 * scmc.h -- C ABI of libscmc: the two-component Shan-Chen lattice Boltzmann
 * time step and its pressure-tensor observables on AMD Instinct MI355X
 * (gfx950), after Lulli, Biferale, Falcucci, Sbragaglia, Shan, "Mesoscale
 * Modelling of the Tolman Length in Multi-component Systems" (arXiv:2112.02574).
 *
 * The method (paper Sec. 2):
 *   f_i^J(x + xi_i, t + 1) = f_i^J - (f_i^J - f_i^eq(n_J, u)) / tau_J
 *                            + (1 - 1/(2 tau_J)) S_i(u, F_J)          (eq. lbm)
 *   n_J = sum_i f_i^J;  (n_A + n_B) u = sum_J [sum_i f_i^J xi_i + F_J / 2]
 *   F_J = -g_JK n_J sum_a W_a n_K(x + e_a) e_a
 *         -g_JJ psi_J sum_a W_a psi_J(x + e_a) e_a                  (eq. sc_force)
 * with a periodic box, D2Q9 or D3Q19 velocities (c_s^2 = 1/3) and force
 * stencils of isotropy order 4 (the paper's W(1) = 1/6, W(2) = 1/12), 6 or 8,
 * all normalised to e2 = sum_a W_a (e_a^x)^2 = 1 (Sec. 2, after eq. bulkp).
 * The observables are the lattice pressure tensor (eq. sm:pt), the bulk
 * pressure (eq. bulkp), the pressure jump dP, the generalised surface tension
 * sigma[R] and the surface-of-tension radius R_s (Sec. 3, eq. gen_sigma), and
 * the flat-interface sigma_0 (Sec. 4).
 *
 * Conventions
 *   - Status: every call returns SCMC_OK (0) or a negative scmc_status.  No
 *     C++ exception crosses this boundary.  scmc_last_error() gives the text
 *     of the last failure on a handle.
 *   - Memory: the library never allocates device memory.  The caller owns the
 *     device workspace (size from scmc_workspace_bytes, any device pointer
 *     with 256-byte alignment) and the HIP stream, both of which must outlive
 *     the handle.  Host arrays passed in are borrowed for the duration of the
 *     call only.  The library never frees caller memory.
 *   - Layout of host fields: FP64, site index s = (z*ny + y)*nx + x (x
 *     fastest), nz = 1 in 2D.  Population arrays are f[(J*Q + i)*N + s] with
 *     J = 0 (A), 1 (B) and the velocity order given by scmc_velocities().
 *   - State: the populations at integer time t are the pre-collision
 *     (post-streaming) f_i^J(x, t) of eq. lbm; every getter and setter uses
 *     that state.
 *   - Streams: launches are asynchronous on the handle's stream; getters,
 *     scmc_stats and scmc_observables synchronise that stream.
 *   - Threads: one handle per host thread at a time; distinct handles are
 *     independent.
 */
#ifndef SCMC_H
#define SCMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCMC_OK = 0,
    SCMC_EINVAL = -1,       /* NULL pointer, bad enum or size, tau <= 1/2,
                               g_AB != g_BA, non-finite input */
    SCMC_EUNSUPPORTED = -2, /* valid but not implemented (E8 in 3D, a tau = 1
                               design with tau != 1, kernel design for this
                               lattice) */
    SCMC_ENOSPACE = -3,     /* workspace smaller than scmc_workspace_bytes */
    SCMC_EDEVICE = -4,      /* HIP runtime error; see scmc_last_error */
    SCMC_ENONFINITE = -5,   /* the state holds NaN or Inf */
    SCMC_ESTATE = -6        /* call out of order (e.g. step before set) */
} scmc_status;

typedef enum { SCMC_D2Q9 = 0, SCMC_D3Q19 = 1 } scmc_lattice;
typedef enum { SCMC_E4 = 4, SCMC_E6 = 6, SCMC_E8 = 8 } scmc_stencil;
typedef enum { SCMC_PSI_N = 0, SCMC_PSI_EXP_NEG_INV = 1 } scmc_psi;
typedef enum {
    SCMC_F64 = 0,     /* populations stored and updated in FP64 */
    SCMC_F32 = 1,     /* stored and updated in FP32 */
    SCMC_F16_OFF = 2, /* stored as FP16 h = f - w_i n0_J (round to nearest
                         even), updated in FP32 */
    SCMC_BF16_OFF = 3, /* same with bfloat16 */
    SCMC_F16_NODE = 4, /* stored as FP16 2^10 h, h = f*_i(x) -
                          w_i n_J(x + xi_i) (round to nearest even; the
                          exact power-of-two scale keeps offsets down to
                          2^-24 out of the FP16 subnormals), the offset from
                          the equilibrium at rest of the node x + xi_i that
                          pulls it: n_J is the density of the step, kept in
                          FP32 beside the populations (the pulling node
                          decodes against its own), so the stored offsets
                          carry only the departure from rest (zero in a bulk
                          at rest) and the minority phase keeps its
                          precision.  The
                          rest populations, which do not stream, are kept
                          in FP32 and close each node's mass balance on the
                          decoded moving ones.  Updated in FP32.  D3Q19, tau =
                          1, the moment two-pass (TWO_PASS_MOM or AUTO),
                          nearest rounding, single lattices only
                          (SCMC_EUNSUPPORTED otherwise); n0 is unused */
    SCMC_BF16_NODE = 5 /* the same with bfloat16 */
} scmc_storage;
typedef enum {
    SCMC_KERNEL_AUTO = 0,        /* tau_A = tau_B = 1: TWO_PASS_MOM; otherwise
                                    FUSED where it exists (D3Q19, E4/E6,
                                    FP32/FP16/BF16), else TWO_PASS;
                                    scmc_autotune may choose another */
    SCMC_KERNEL_TWO_PASS = 1,    /* density pass + stream/force/collide pass */
    SCMC_KERNEL_FUSED = 2,       /* one z-marching kernel per step (D3Q19 with
                                    E4/E6, FP32/FP16/BF16 storage); the pulled
                                    populations wait in registers */
    SCMC_KERNEL_FUSED_REPULL = 3, /* same, but the populations of the
                                     collided plane are pulled again (from
                                     cache) instead of held in registers */
    SCMC_KERNEL_FUSED_PIPE = 4,   /* fused, with the next plane's loads issued
                                     before the current plane's collision */
    SCMC_KERNEL_FUSED_MOM = 5,    /* fused for tau = 1 only: the collision
                                     then depends on the pulled populations
                                     only through n_J and the total momentum,
                                     so five moments per node wait in
                                     registers instead of 2Q populations */
    SCMC_KERNEL_FUSED_MOM_PIPE = 6, /* the same with the next plane's loads
                                       issued early (tau = 1 only) */
    SCMC_KERNEL_TWO_PASS_MOM = 7  /* two passes for tau = 1 only: the first
                                     pulls and stores n_J and the momentum,
                                     the second collides from those moments
                                     without pulling again (every lattice,
                                     stencil and storage; lattices whose
                                     moments (24 B per site) pass 264 MiB
                                     in FP32, 128 MiB in FP16/BF16, run it
                                     in z-slabs); with a nonzero
                                     tile (D3Q19, FP32/FP16/BF16) the second
                                     pass stages the stencil's concentrations
                                     in LDS (64 x 8 columns, z-chunks of 8) */
} scmc_kernel;
typedef enum {
    SCMC_ROUND_NEAREST = 0,   /* FP16 / BF16 offsets rounded to nearest even */
    SCMC_ROUND_STOCHASTIC = 1 /* rounded up with probability equal to the
                                 discarded fraction of an ulp (unbiased);
                                 the random bits come from a counter-based
                                 hash of (seed, step, site, J, i), so runs
                                 are reproducible.  Two-pass designs only. */
} scmc_rounding;
typedef enum { SCMC_OBS_FLAT = 0, SCMC_OBS_DROPLET = 1, SCMC_OBS_SHELL = 2 } scmc_obs_kind;

typedef struct {
    int lattice;      /* scmc_lattice */
    int stencil;      /* scmc_stencil: isotropy order of the force stencil */
    int nx, ny, nz;   /* periodic box; nz = 1 for D2Q9; every extent
                         >= 2 r_F + 1 where r_F = 1 (E4) or 2 (E6, E8) */
    double tau[2];    /* BGK relaxation times tau_A, tau_B (> 1/2).  When
                         they differ, the common velocity weights each
                         component by 1/tau_J, u = sum_J (j_J + F_J/2)/tau_J
                         / sum_J n_J/tau_J, which keeps the collision's total
                         momentum change equal to sum_J F_J and reduces to
                         the form of Sec. 2 for equal times; the designs
                         TWO_PASS, FUSED, FUSED_REPULL and FUSED_PIPE run
                         it */
    double g[2][2];   /* couplings G_JK c_s^2 multiplying the e2 = 1 stencil
                         sums; g[0][1] == g[1][0] is the cross coupling */
    int psi_self;     /* scmc_psi of the self terms; cross terms use n */
    int storage;      /* scmc_storage */
    double n0[2];     /* offset references of the FP16/BF16 storage */
    int kernel;       /* scmc_kernel */
    int tile[3];      /* fused-kernel tile (x, y, z-chunk); 0 = default */
    int rounding;     /* scmc_rounding of FP16 / BF16 offset stores */
    unsigned int seed; /* seed of the stochastic rounding */
} scmc_problem;

typedef struct {
    double mass[2];      /* sum_x n_J */
    double momentum[3];  /* sum_x sum_J (sum_i f_i xi_i + F_J / 2) */
    double min_n[2];     /* min_x n_J */
    double max_u;        /* max_x |u| */
    double n_nonfinite;  /* number of non-finite populations */
    int64_t step;        /* time t of the state */
} scmc_stats;

typedef struct {
    double P_in, P_out;  /* bulk pressure (eq. bulkp) at the centre node
                            floor(L/2) and at (centre + floor(L/2)) mod L */
    double dP;           /* P_in - P_out */
    double C_d;          /* int_0^{L/2} r^(d-1) (P_out - P_T(r)) dr along +x,
                            P_T = P^yy, linear between nodes, exact per cell */
    double R_s;          /* (d (d-1) C_d / dP)^(1/d): minimum of sigma[R] */
    double sigma_s;      /* dP R_s / (d - 1): sigma at the minimum */
    double R_s_grid;     /* parabolic-vertex minimum of sigma[R] on the grid
                            [R0/2, 2 R0], step 0.01 (cross-check) */
    double sigma0;       /* flat: sum_{x = nx/2}^{nx-1} (P^xx - P^yy), both
                            averaged over y, z */
    double max_PyyPzz;   /* max |P^yy - P^zz| on the droplet line (3D);
                            0 for kind SHELL */
    int64_t step;
} scmc_obs;

/* Defaults: D3Q19, E6, 64^3, tau = 1, g_AB = 1.8, psi = n, FP32, auto. */
int scmc_problem_init(scmc_problem *p);

/* Velocity set of a lattice: xi[Q*3] (ints), w[Q]; returns Q or SCMC_EINVAL. */
int scmc_velocities(int lattice, int *xi, double *w);

/* Device workspace needed by a problem, in bytes (*out). */
int scmc_workspace_bytes(const scmc_problem *p, size_t *out);

typedef struct scmc_sim scmc_sim;

/* Validate p and bind the caller's workspace (d_ws, ws_bytes) and HIP stream
 * (a hipStream_t; NULL = the default stream).  Allocates no device memory.
 * On failure *out is NULL. */
int scmc_create(const scmc_problem *p, void *d_ws, size_t ws_bytes,
                void *stream, scmc_sim **out);
/* Waits for the work queued on the handle's stream (so the caller may reuse
 * the workspace as soon as this returns), then frees the handle; SCMC_EDEVICE
 * if that wait reports a HIP error (the handle is freed anyway). */
int scmc_destroy(scmc_sim *s);

/* f_i^J(x, 0) = w_i n_J(x) (zero velocity; the paper does not state the
 * initial populations), t = 0.  nA, nB: N host doubles each.  EINVAL on a
 * non-finite value.
 * Device state: after scmc_set_density or scmc_set_populations, and until the
 * next step, the state is the first 2*Q*N values of the storage type at the
 * start of the workspace, laid out [J][i][z][y][x]; value (J, i, x) is the
 * post-collision f*_i^J(x) that the next step streams to x + xi_i (FP16 /
 * BF16: the offset f* - w_i n0_J; node storage: the offset
 * f*_i(x) - w_i n_J(x + xi_i) for i > 0, with the n_J and the rest
 * populations f*_0 held as FP32 pairs per node in the workspace's moment
 * field).  scmc_step_static reads and writes buffers of
 * this layout (node storage: SCMC_EUNSUPPORTED). */
int scmc_set_density(scmc_sim *s, const double *nA, const double *nB);

/* Advance nsteps >= 0 time steps, asynchronously.  With graph steps k > 0
 * (scmc_set_graph_steps) runs of k steps replay one instantiated hipGraph. */
int scmc_step(scmc_sim *s, int64_t nsteps);
int scmc_set_graph_steps(scmc_sim *s, int k);
int scmc_synchronize(scmc_sim *s);

/* For callers that cannot allocate device memory and hold no workspace (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): one time step of problem p, as scmc_step takes it, from the
 * caller's device populations src to dst (distinct buffers of 2*Q*N values of
 * the storage type, in the device layout described at scmc_set_density), on
 * the current device and the given stream (NULL = default).  The kernel
 * design is chosen as scmc_create does; the density / moment field of the
 * two-pass designs lives in a static device array of the library,
 * SCMC_STATIC_SCRATCH_BYTES on every GPU it runs on, held until the process
 * ends.  Nothing is allocated.  Every call on one GPU shares that array and
 * fully rewrites the part it reads, so calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Returns SCMC_ENOSPACE when the lattice needs more than the array (7 values
 * of the compute precision per site: 2.39M sites FP32/FP16/BF16, 1.19M FP64),
 * SCMC_EUNSUPPORTED for stochastic rounding (its step counter lives in a
 * workspace); the text is in scmc_last_error(NULL) of the calling thread. */
#define SCMC_STATIC_SCRATCH_BYTES (64u << 20)
int scmc_step_static(const scmc_problem *p, const void *src, void *dst, void *stream);

/* n_J(x, t) and, when u is not NULL, the common velocity u[c*N + s]
 * (c = 0..2) of the current state.  Synchronous. */
int scmc_get_fields(scmc_sim *s, double *nA, double *nB, double *u);

/* Checkpoint / resume: f[2*Q*N] pre-collision populations and the step. */
int scmc_get_populations(scmc_sim *s, double *f, int64_t *step);
int scmc_set_populations(scmc_sim *s, const double *f, int64_t step);

/* FP64 global statistics of the current state (Sec. 2 conservation laws). */
int scmc_stats_get(scmc_sim *s, scmc_stats *out);

/* Observables of the current state; PN, PT (nullable) receive P^xx, P^yy on
 * the droplet line r = 0..floor(nx/2) (kind DROPLET, nx/2 + 1 values) or the
 * transverse-averaged profiles (kind FLAT, nx values).  R0 sets the grid of
 * the sigma[R] scan (DROPLET, SHELL).
 * Kind SHELL is a variant of the droplet analysis that is not the paper's
 * definition (Sec. 3 uses the axis line): every node x at distance
 * r = |x - c| from the centre node c = floor(L/2) (no periodic image) belongs
 * to shell k = floor(r + 1/2), k = 0..rmax with rmax = floor(min extent / 2);
 * with u = (x - c) / r it carries P_N = u.P.u and P_T = (tr P - P_N)/(d - 1)
 * of the lattice tensor (eq. sm:pt; tr P / d at the centre).  PN, PT receive
 * the shell means (rmax + 1 values) and P_in, P_out, dP, C_d, R_s, sigma_s,
 * R_s_grid follow from the shell P_T as from the line's; max_PyyPzz = 0.
 * Averaging over whole shells cuts the lattice and rounding noise of R_s.
 * The sums run in a fixed order (bitwise reproducible). */
int scmc_observables(scmc_sim *s, int kind, double R0, scmc_obs *out,
                     double *PN, double *PT);

/* Convergence monitor of a droplet run (Sec. 4), meant to be called every
 * dt steps (the paper: dt = 2^11).  Each call evaluates the droplet
 * observables at R0 (as scmc_observables), the FP64 velocity field and the
 * centre of the rich component's excess concentration, and compares with the
 * previous call on this handle (the previous velocity field is kept in the
 * workspace; setting a new state forgets it):
 *   dP_change = |dP(t) - dP(t_prev)| / |dP(t_prev)|            (criterion i)
 *   du = (1/N) sum_x sum_a |u_a(x, t) - u_a(x, t_prev)|       (criterion ii)
 * converged = dP_change < tol_dP or du < tol_du (the paper: 1e-5, 1e-12); on
 * the first call there is no comparison (NaN, not converged).  The rich
 * component is the one with the larger concentration at the centre node; its
 * excess is n_rich(x) - n_rich at the far node, and com[a] = c_a +
 * sum ex (x_a - c_a) / sum ex with c_a = floor(L_a / 2) (the paper analyses
 * a run only if every |com_a - c_a| < 1e-3). */
typedef struct {
    double dP, dP_change, du;
    double com[3];
    double com_offset;   /* max_a |com_a - c_a| */
    int rich;            /* 0: A-rich droplet, 1: B-rich */
    int converged;
    int64_t step, prev_step;
} scmc_convergence;
int scmc_convergence_check(scmc_sim *s, double R0, double tol_dP, double tol_du,
                           scmc_convergence *out);
/* Steps in chunks of dt with a check after each (and one before the first),
 * until converged or max_steps have run; *out holds the last check. */
int scmc_run_to_convergence(scmc_sim *s, double R0, int64_t dt, int64_t max_steps,
                            double tol_dP, double tol_du, scmc_convergence *out);
/* (Returns SCMC_ENONFINITE as soon as a check finds Delta P not finite.) */

/* Curvature expansion of the surface tension (eq. sigma_c, Sec. 4):
 *   sigma(R_s) = sigma_0 (1 - 2 delta c + (2 kbar + k) c^2),  c = 1 / R_s,
 * with c signed: positive for a droplet of the A-rich phase, negative for a
 * droplet of the B-rich phase (whose A-rich surroundings curve the other
 * way).  Host-only least-squares fit of the quadratic through n >= 3 points
 * (curvature[i], sigma[i]), e.g. sigma[i] = Delta P R_s / 2 of converged
 * droplets of several sizes.  out[3] = {sigma_0, delta (Tolman length),
 * 2 kbar + k (curvature and Gaussian rigidities)}, in lattice units.  SCMC_EINVAL for
 * NULL pointers, n < 3, non-finite input or fewer than three distinct
 * curvatures.  Host arrays are borrowed for the call. */
int scmc_curvature_fit(int n, const double *curvature, const double *sigma, double *out);

/* Flat-interface steady state (Sec. 4: the droplet runs start from the bulk
 * concentrations of a converged flat interface).  Runs the problem's lattice,
 * stencil, couplings, tau, psi and storage on a transverse-thin periodic box
 * of lx x 5 (x 5 in 3D) nodes holding an A-rich strip x in [lx/4, 3 lx/4)
 * with the guessed bulk values guess = {nA_in, nB_in, nA_out, nB_out} (NULL:
 * {1, 0.04, 0.04, 1}), in chunks of 2048 steps until no bulk concentration
 * (strip centre x = lx/2, box edge x = 0) changes by more than tol over a
 * chunk, or max_steps have run.  out[4] = {nA_in, nB_in, nA_out, nB_out};
 * *steps (nullable) = steps run.  The workspace comes from
 * scmc_flat_workspace_bytes; the call synchronises the stream.  Returns
 * SCMC_ENONFINITE if the run diverges. */
int scmc_flat_workspace_bytes(const scmc_problem *p, int lx, size_t *out);
int scmc_flat_equilibrium(const scmc_problem *p, int lx, const double *guess,
                          int64_t max_steps, double tol, void *d_ws,
                          size_t ws_bytes, void *stream, double *out,
                          int64_t *steps);

/* Many independent lattices advanced together over one tile list (the
 * paper's sweep over droplet sizes and couplings, Sec. 4).  The moment
 * two-pass runs the members in chunks of whole members (a member with 48 MB
 * or more of moments alone, the others packed up to 48 MB), pass 1 and then
 * pass 2 of each chunk: a chunk of one member launches as a single lattice
 * does, the others one workgroup per 256-site tile.  The fused designs run
 * one persistent launch per step.  Members may differ in size and
 * couplings; they must share lattice, stencil, tau and storage.  Member calls
 * take the member index i. */
typedef struct scmc_batch scmc_batch;
int scmc_batch_workspace_bytes(const scmc_problem *ps, int count, size_t *out);
int scmc_batch_create(const scmc_problem *ps, int count, void *d_ws,
                      size_t ws_bytes, void *stream, scmc_batch **out);
int scmc_batch_destroy(scmc_batch *b);  /* waits for the stream, as scmc_destroy */
int scmc_batch_set_density(scmc_batch *b, int i, const double *nA,
                           const double *nB);
/* Advances every member nsteps steps.  Members are independent lattices:
 * with the moment two-pass a call runs chunk by chunk, each chunk a block of
 * steps (a graph's length, else up to 64) before the next, so members pass
 * through different steps while the call's work runs on the stream; all
 * are at the batch's step count once it has completed. */
int scmc_batch_step(scmc_batch *b, int64_t nsteps);
int scmc_batch_set_graph_steps(scmc_batch *b, int k);
int scmc_batch_get_fields(scmc_batch *b, int i, double *nA, double *nB,
                          double *u);
/* Member i's pre-collision populations f[2*Q*N_i] (layout as
 * scmc_get_populations) and the batch's step.  Synchronous. */
int scmc_batch_get_populations(scmc_batch *b, int i, double *f, int64_t *step);
int scmc_batch_stats_get(scmc_batch *b, int i, scmc_stats *out);
int scmc_batch_observables(scmc_batch *b, int i, int kind, double R0,
                           scmc_obs *out, double *PN, double *PT);
/* Tile (x, y, z-chunk) and the fused designs' persistent grid (workgroups
 * before the clamp to those the device holds at once). */
int scmc_batch_config(scmc_batch *b, int *tile, int *grid);

/* Autotuner: times each candidate fused-kernel tile on a scratch state in
 * the handle's workspace (it overwrites the state, so call it before
 * scmc_set_density), keeps the fastest, and returns it in tile[3].  When
 * cache_path is not NULL the result is read from / appended to that text
 * file, keyed by lattice, stencil, storage and box. */
int scmc_autotune(scmc_sim *s, const char *cache_path, int *tile);
int scmc_batch_autotune(scmc_batch *b, const char *cache_path, int *tile);

/* Kernel design and tile in use by a handle. */
int scmc_config(scmc_sim *s, int *kernel, int *tile);

/* Measurement aid, not a step of the method: the streaming half of eq. lbm
 * without its arithmetic.  Copies the 2*Q population planes of one of the
 * handle's buffers into the other with the pull shifts, f_i(x) <- f_i(x -
 * xi_i) (periodic), one site per lane and in the step's access pattern,
 * reps >= 1 times (alternating the buffers), timed with events on the
 * handle's stream; *us = mean microseconds per copy.  Every population is
 * read and written once, as in a step, so 4*Q*s*N bytes / *us is the
 * bandwidth ceiling of any step design that moves each population once (s
 * = bytes per stored value).  The buffers then hold shifted copies: the
 * handle's state is unset (SCMC_ESTATE until scmc_set_density or
 * scmc_set_populations).  Synchronous. */
int scmc_pull_copy(scmc_sim *s, int reps, double *us);

/* Text of the last failure on a handle; with NULL, of the calling thread's
 * last scmc_step_static failure (or "NULL handle"). */
const char *scmc_last_error(const scmc_sim *s);
const char *scmc_batch_last_error(const scmc_batch *b);
const char *scmc_status_str(int status);

#ifdef __cplusplus
}
#endif
#endif
