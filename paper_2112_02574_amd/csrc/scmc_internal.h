// scmc_internal.h -- declarations shared by the host library and the kernel
// translation units of libscmc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace scmc {

// One lattice as the kernels see it.  Populations of a member live at
// pop + pop_off (element offset in the storage type) in both population
// buffers, component-major: [J][i][z][y][x]; its density field lives at
// dens + dens_off as [J][z][y][x] (the moment two-pass: (n_A, n_B) pairs
// [z][y][x], then the momentum planes and the remainders of n_J), with room for 7 fields.
struct Member {
    int nx, ny, nz, N;
    long long pop_off;
    long long dens_off;
    double g[2][2];   // G_JK c_s^2
    double omega[2];  // 1 / tau_J
    double n0[2];     // offset references (FP16 / BF16 storage)
    int psi_self;     // 0: psi = n, 1: psi = exp(-1/n)
    int self_on;      // bit J set when g_JJ != 0
    int sr;           // 1: stochastic rounding of FP16 / BF16 stores
    unsigned seed;    // its seed
    unsigned *step_ctr;  // device step counter: advanced by the first pass of
                         // a two-pass step, read by the second (random stream)
    int zoff, znum;      // z-planes [zoff, zoff + znum) of a launch of the
                         // moment two-pass (the whole lattice: 0, nz)
    // FP16 / BF16 node storage: reference densities (n_A, n_B) per site
    // [z][y][x] of the buffer being pulled (nullptr for the other formats),
    // and the slot (in units of N values) of the (n_A, n_B) pairs that the
    // moment two-pass writes in pass 1 and reads in pass 2 (0 otherwise)
    const float2 *ref;
    int pair_slot;
    // node storage: the rest populations (f*_0^A, f*_0^B) per site in FP32
    // (they do not stream: pass 1 reads and pass 2 writes the node's own)
    float2 *rest;
};

// A unit of work of the batched launches: member index and tile origin.
struct Tile {
    int member, x0, y0, z0;
};

enum StorageKind { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

// kernel selector shared by the launchers
struct StepKey {
    int dim;      // 2 or 3
    int order;    // 4, 6, 8
    int storage;  // StorageKind
    int psi;      // 0 / 1
    int repull = 0;  // fused design: 0 = register ring, 1 = re-pull at collide,
                  // 2 = register ring with loads issued one plane ahead,
                  // 3 / 4 = moment ring (tau = 1), plain / loads ahead
    int mom = 0;     // two-pass design: 1 = moment passes (tau = 1), 2 = the
                     // same with the collision pass's pairs staged in LDS
    int big = 0;     // 1 when a component's Q planes exceed 2^31 bytes: no
                     // 32-bit buffer offsets (fused designs unavailable)
    int node = 0;    // FP16 / BF16 offsets from the per-node reference
                     // (moment two-pass, D3Q19 buffer forms only)
    int sr = 0;      // 1 = stochastic rounding of the 16-bit offsets: the
                     // buffer forms' collision passes are compiled with and
                     // without it (its generator costs registers)
};

// ---- step kernels (step_kernels.hip)
// Two-pass design: density pass then stream/force/collide pass.
hipError_t launch_two_pass(const StepKey &k, const Member &m, const void *src,
                           void *dst, void *dens, hipStream_t st);
// Fused z-marching design: one kernel per step.  tile = (tx, ty, zc).
hipError_t launch_fused(const StepKey &k, const Member &m, const void *src,
                        void *dst, const int *tile, hipStream_t st);
bool fused_supported(const StepKey &k, const int *tile);
// Batched persistent launches over a tile list (device arrays).
// Workgroups of kernel f (threads each, shmem bytes of dynamic LDS) that the
// current device holds at once.  The fused batched launches are persistent
// loops over a tile list and use at most that many: surplus workgroups would
// start only after others had run their whole share of the list.  (The
// two-pass batched launches run one workgroup per 256-site tile.)
int resident_blocks(const void *f, int threads, unsigned shmem = 0);
// grid: workgroups; one per tile runs each tile once.  passes: 1 = pass 1
// only, 2 = pass 2 only, 3 = both.  nt_all: pass 1 loads every population
// non-temporally (FP32 moment two-pass; see pass1_nt_all)
hipError_t launch_batch_two_pass(const StepKey &k, const Member *d_members,
                                 const Tile *d_tiles, int ntiles,
                                 const void *src, void *dst, void *dens,
                                 int grid, hipStream_t st, int passes = 3,
                                 bool nt_all = false);
// Whether pass 1 of the moment two-pass over `sites` sites (one unslabbed
// lattice, or one chunk of a batch) loads every population non-temporally.
bool pass1_nt_all(const StepKey &k, long sites);

hipError_t launch_batch_fused(const StepKey &k, const Member *d_members,
                              const Tile *d_tiles, int ntiles, const void *src,
                              void *dst, const int *tile, int grid,
                              hipStream_t st);
// Kernel function and argument packing for explicit hipGraph nodes.
struct NodeLaunch {
    void *func;
    dim3 grid, block;
    unsigned shmem;
};
// The moment two-pass over a lattice whose moment field does not fit the
// caches runs in z-slabs: pass 2 of a slab follows pass 1 of the next one, so
// the moments it gathers are still cached.  Empty: one launch per pass.
struct SlabOp {
    int pass;    // 1 or 2; 3: pass 2 over [z0, z0 + nz) and, in the same
                 // launch (k_slab_pair), pass 1 over [z1, z1 + n1)
    int z0, nz;
    int z1 = 0, n1 = 0;
};
std::vector<SlabOp> slab_schedule(const StepKey &k, const Member &m);
// the kernel of the pass-3 slab launches (grid and block set per launch)
bool node_slab_pair(const StepKey &k, NodeLaunch *node);
// Blocks of blk linearly numbered sites that cover znum planes of m.
int linear_blocks(const Member &m, int znum, int blk);

bool node_two_pass(const StepKey &k, NodeLaunch *dens_node,
                   NodeLaunch *step_node, const Member &m);
bool node_fused(const StepKey &k, const int *tile, NodeLaunch *node,
                const Member &m);
// One pass (1 or 2) of the moment two-pass over the whole of one batch member,
// launched like a single lattice (linear 256-site blocks, the member's
// description a kernel argument instead of a per-block load from the tile
// list).  D3Q19 buffer forms without node storage or stochastic rounding;
// node_member_pass returns false (launch_member_pass hipErrorNotSupported)
// for every other key.  nt_all as in launch_batch_two_pass.
bool node_member_pass(const StepKey &k, const Member &m, int pass, bool nt_all,
                      NodeLaunch *node);
hipError_t launch_member_pass(const StepKey &k, const Member &m, const void *src, void *dst,
                              void *dens, int pass, bool nt_all, hipStream_t st);
// dens_node_nt_all (optional): the pass-1 node of launch_batch_two_pass's
// nt_all form (the same as dens_node where there is none)
bool node_batch_two_pass(const StepKey &k, int grid, NodeLaunch *dens_node,
                         NodeLaunch *step_node, NodeLaunch *dens_node_nt_all = nullptr);
bool node_batch_fused(const StepKey &k, const int *tile, int grid,
                      NodeLaunch *node);

// ---- bandwidth ceiling (ceiling_kernels.hip): the 2Q population planes of
// src copied to dst with the pull shifts, one site per lane; elements of
// `bytes` bytes (8, 4 or 2)
hipError_t launch_pull_copy(int dim, int bytes, const Member &m, const void *src, void *dst,
                            hipStream_t st);

// ---- FP64 observable kernels (obs_kernels.hip)
// dens64[J][s] = sum_i f_i^J of the current state (pulled, decoded, FP64)
hipError_t launch_density64(const StepKey &k, const Member &m, const void *pop,
                            double *dens64, hipStream_t st);
// per-block partials then a final fixed-order reduction into out[16]
hipError_t launch_stats(const StepKey &k, const Member &m, const void *pop,
                        const double *dens64, double *partials, int nblocks_max,
                        double *out, hipStream_t st);
int stats_blocks(const Member &m);
// velocity field u[3][N] (FP64)
hipError_t launch_velocity64(const StepKey &k, const Member &m, const void *pop,
                             const double *dens64, double *u, hipStream_t st);
// droplet line: out[0..3*(rmax+1)) = P^xx, P^yy, P^zz along +x from the
// centre; out[3*(rmax+1)] = P_in, [+1] = P_out, [+2] = C_d
hipError_t launch_line(const StepKey &k, const Member &m, const double *dens64,
                       double *out, hipStream_t st);
// convergence monitor: out[0] = sum |u - u0| (u0 nullable), out[1] = sum of
// the rich component's excess concentration, out[2..4] = its first moments
// about the centre node; partials as for the stats
hipError_t launch_monitor(const Member &m, int dim, const double *dens64, const double *u,
                          const double *u0, int rich, double n_out, double *partials,
                          double *out, hipStream_t st);
// shell-averaged profiles (variant of the droplet line): shells k = 0..rmax,
// rmax = shell_rmax = floor(min extent / 2); out[k], out[nshell + k] = P_N,
// P_T; out[2 nshell ..] = P_in, P_out, C_d.  partials: capacity in doubles
// (3 per shell and block)
int shell_rmax(const Member &m, int dim);
hipError_t launch_shell(const StepKey &k, const Member &m, const double *dens64,
                        double *partials, long partial_capacity, double *out,
                        hipStream_t st);
// flat: out[0..nx) = <P^xx>_yz, out[nx..2nx) = <P^yy>_yz, out[2nx] = sigma0
hipError_t launch_flat(const StepKey &k, const Member &m, const double *dens64,
                       double *out, hipStream_t st);

}  // namespace scmc
