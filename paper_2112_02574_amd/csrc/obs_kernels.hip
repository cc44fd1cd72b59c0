// obs_kernels.hip -- FP64 reductions on the current state: concentrations,
// global statistics (mass, momentum, extrema, non-finite count), the common
// velocity field, the lattice pressure tensor on the droplet axis and the
// transverse-averaged flat profiles (paper Sec. 2 eq. sm:pt and eq. bulkp,
// Sec. 3 eq. gen_sigma, Sec. 4).  Every reduction runs in a fixed order
// (per-thread sequential, then a butterfly across each wavefront's lanes and
// the wavefronts in order, then one final block), so repeated calls on the
// same state give bitwise-identical results.
#include "site_ops.h"

#include <algorithm>

namespace scmc {

// Common velocity in FP64 from the components' momenta jm[J] = sum_i f_i xi_i:
// u = sum_J (jm_J + F_J / 2) / (n_A + n_B) (Sec. 2); with tau_A != tau_B both
// sums are weighted by omega_J = 1 / tau_J, as in the collision.
__device__ __forceinline__ void common_velocity(const Member &m, const double (&jm)[2][3],
                                                double nA, double nB, const double (&FA)[3],
                                                const double (&FB)[3], double (&u)[3]) {
    const double oA = m.omega[0], oB = m.omega[1];
    for (int c = 0; c < 3; ++c)
        u[c] = oA == oB ? (jm[0][c] + jm[1][c] + 0.5 * (FA[c] + FB[c])) / (nA + nB)
                        : (oA * (jm[0][c] + 0.5 * FA[c]) + oB * (jm[1][c] + 0.5 * FB[c])) /
                              (oA * nA + oB * nB);
}

constexpr int OB_BX = 64, OB_BY = 4, OB_THREADS = OB_BX * OB_BY;

// Population value as a double: the stored value plus, for the offset
// formats, the same single-precision reference the step kernels add.
template <class ST> struct Decode;
template <> struct Decode<StoreF64> {
    __device__ static double get(const double *p, long i, double, double) {
        return p[i];
    }
};
template <> struct Decode<StoreF32> {
    __device__ static double get(const float *p, long i, double, double) {
        return (double)p[i];
    }
};
template <> struct Decode<StoreF16> {
    __device__ static double get(const uint16_t *p, long i, double w, double n0) {
        const float ref = (float)w * (float)n0;
        return (double)__half2float(__ushort_as_half(p[i])) + (double)ref;
    }
};
template <> struct Decode<StoreBF16> {
    __device__ static double get(const uint16_t *p, long i, double w, double n0) {
        const float ref = (float)w * (float)n0;
        return (double)bf16_to_f32(p[i]) + (double)ref;
    }
};

template <int D, class ST>
__device__ __forceinline__ void pull64(const Member &m,
                                       const typename ST::T *__restrict__ src,
                                       int x, int y, int z,
                                       double (&f)[2][Lattice<D>::Q]) {
    using L = Lattice<D>;
    const typename ST::T *base = src + m.pop_off;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap1(x - L::CX[i], m.nx);
        const int ys = wrap1(y - L::CY[i], m.ny);
        const int zs = D == 3 ? wrap1(z - L::CZ[i], m.nz) : 0;
        const long s = ((long)zs * m.ny + ys) * m.nx + xs;
        if constexpr (sizeof(typename ST::T) == 2) {
            if (m.ref) {
                // node storage: decoded exactly as the step's pull does it,
                // the rest populations from their FP32 field
                if (i == 0) {
                    const float2 r = m.rest[s];
                    f[0][0] = (double)r.x;
                    f[1][0] = (double)r.y;
                    continue;
                }
                // the offset pulled into (x, y, z) is taken from this node's
                // own reference densities
                const float2 q = m.ref[((long)z * m.ny + y) * m.nx + x];
                const float w = (float)L::W[i];
                f[0][i] = (double)ST::from_node(base[(long)i * m.N + s], node_ref(w, q.x));
                f[1][i] = (double)ST::from_node(base[(long)(L::Q + i) * m.N + s], node_ref(w, q.y));
                continue;
            }
        }
        f[0][i] = Decode<ST>::get(base, (long)i * m.N + s, L::W[i], m.n0[0]);
        f[1][i] = Decode<ST>::get(base, (long)(L::Q + i) * m.N + s, L::W[i],
                                  m.n0[1]);
    }
}

template <int D, class ST>
__global__ void __launch_bounds__(OB_THREADS)
    k_density64(Member m, const typename ST::T *__restrict__ src,
                double *__restrict__ dens) {
    const int x = blockIdx.x * OB_BX + threadIdx.x;
    const int y = blockIdx.y * OB_BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= m.nx || y >= m.ny) return;
    double f[2][Lattice<D>::Q];
    pull64<D, ST>(m, src, x, y, z, f);
    double nA, nB;
    site_density<D, double>(f, nA, nB);
    const long s = ((long)z * m.ny + y) * m.nx + x;
    dens[s] = nA;
    dens[m.N + s] = nB;
}

// stats slots: 0 mass A, 1 mass B, 2-4 momentum, 5 min n_A, 6 min n_B,
// 7 max |u|, 8 non-finite count
constexpr int NSTAT = 9;

__device__ __forceinline__ double combine(int k, double a, double b) {
    if (k == 5 || k == 6) return fmin(a, b);
    if (k == 7) return fmax(a, b);
    return a + b;
}

// Deterministic reduction of NK values per thread over a block of NT
// threads (linear thread index tid): a butterfly of cross-lane exchanges
// inside each 64-wide wavefront (fixed partners, so every lane ends with the
// same value whatever the hardware's scheduling), then thread 0 combines the
// wavefronts' results in order.  The result is valid in thread 0.
template <int NK, int NT, class Op>
__device__ __forceinline__ void block_reduce(double (&v)[NK], double (&red)[NK][NT / 64], int tid,
                                             Op op) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NK; ++k) v[k] = op(k, v[k], __shfl_xor(v[k], off, 64));
    if ((tid & 63) == 0)
        for (int k = 0; k < NK; ++k) red[k][tid >> 6] = v[k];
    __syncthreads();
    if (tid == 0)
        for (int k = 0; k < NK; ++k) {
            double a = red[k][0];
            for (int w = 1; w < NT / 64; ++w) a = op(k, a, red[k][w]);
            v[k] = a;
        }
}
__device__ __forceinline__ double add_op(int, double a, double b) { return a + b; }

template <int D, int ORDER, class ST, int PSI>
__global__ void __launch_bounds__(OB_THREADS)
    k_stats(Member m, const typename ST::T *__restrict__ src,
            const double *__restrict__ dens, double *__restrict__ partials) {
    __shared__ double red[NSTAT][OB_THREADS / 64];
    const int tid = threadIdx.y * OB_BX + threadIdx.x;
    const int x = blockIdx.x * OB_BX + threadIdx.x;
    const int y = blockIdx.y * OB_BY + threadIdx.y;
    const int z = blockIdx.z;
    double v[NSTAT] = {0, 0, 0, 0, 0, 1e300, 1e300, 0, 0};
    if (x < m.nx && y < m.ny) {
        using L = Lattice<D>;
        double f[2][L::Q];
        pull64<D, ST>(m, src, x, y, z, f);
        const long s = ((long)z * m.ny + y) * m.nx + x;
        const double nA = dens[s], nB = dens[m.N + s];
        double FA[3], FB[3];
        site_force<D, ORDER, PSI, double>(m, dens, dens + m.N, x, y, z, nA,
                                          nB, FA, FB);
        double jm[2][3] = {{0, 0, 0}, {0, 0, 0}}, bad = 0;
#pragma unroll
        for (int J = 0; J < 2; ++J)
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                if (!isfinite(f[J][i])) bad += 1;
                jm[J][0] += L::CX[i] * f[J][i];
                jm[J][1] += L::CY[i] * f[J][i];
                jm[J][2] += L::CZ[i] * f[J][i];
            }
        double mom[3], u[3], uu = 0;
        common_velocity(m, jm, nA, nB, FA, FB, u);
        for (int c = 0; c < 3; ++c) {
            mom[c] = jm[0][c] + jm[1][c] + 0.5 * (FA[c] + FB[c]);
            uu += u[c] * u[c];
        }
        v[0] = nA;
        v[1] = nB;
        v[2] = mom[0];
        v[3] = mom[1];
        v[4] = mom[2];
        v[5] = nA;
        v[6] = nB;
        v[7] = sqrt(uu);
        v[8] = bad;
    }
    block_reduce<NSTAT, OB_THREADS>(v, red, tid, combine);
    if (tid == 0) {
        const long b = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x +
                       blockIdx.x;
        for (int k = 0; k < NSTAT; ++k) partials[b * NSTAT + k] = v[k];
    }
}

__global__ void __launch_bounds__(256)
    k_stats_final(const double *__restrict__ partials, int nblocks,
                  double *__restrict__ out) {
    __shared__ double red[NSTAT][256 / 64];
    const int tid = threadIdx.x;
    double v[NSTAT] = {0, 0, 0, 0, 0, 1e300, 1e300, 0, 0};
    for (int b = tid; b < nblocks; b += 256)
        for (int k = 0; k < NSTAT; ++k)
            v[k] = combine(k, v[k], partials[(long)b * NSTAT + k]);
    block_reduce<NSTAT, 256>(v, red, tid, combine);
    if (tid == 0)
        for (int k = 0; k < NSTAT; ++k) out[k] = v[k];
}

template <int D, int ORDER, class ST, int PSI>
__global__ void __launch_bounds__(OB_THREADS)
    k_velocity64(Member m, const typename ST::T *__restrict__ src,
                 const double *__restrict__ dens, double *__restrict__ u) {
    const int x = blockIdx.x * OB_BX + threadIdx.x;
    const int y = blockIdx.y * OB_BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= m.nx || y >= m.ny) return;
    using L = Lattice<D>;
    double f[2][L::Q];
    pull64<D, ST>(m, src, x, y, z, f);
    const long s = ((long)z * m.ny + y) * m.nx + x;
    const double nA = dens[s], nB = dens[m.N + s];
    double FA[3], FB[3];
    site_force<D, ORDER, PSI, double>(m, dens, dens + m.N, x, y, z, nA, nB,
                                      FA, FB);
    double jm[2][3] = {{0, 0, 0}, {0, 0, 0}}, us[3];
#pragma unroll
    for (int J = 0; J < 2; ++J)
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            jm[J][0] += L::CX[i] * f[J][i];
            jm[J][1] += L::CY[i] * f[J][i];
            jm[J][2] += L::CZ[i] * f[J][i];
        }
    common_velocity(m, jm, nA, nB, FA, FB, us);
    for (int c = 0; c < 3; ++c) u[(long)c * m.N + s] = us[c];
}

// Lattice pressure tensor (eq. sm:pt) at one site, FP64:
// P^mn = c_s^2 (n_A + n_B) delta^mn + 1/2 sum_a W_a e^m e^n
//        [g_AB n_A n_B(x+e) + g_BA n_B n_A(x+e) + g_AA psi_A psi_A(x+e)
//         + g_BB psi_B psi_B(x+e)]
// returns xx, yy, zz
template <int D, int ORDER, int PSI>
__device__ void ptensor_diag(const Member &m, const double *__restrict__ dens,
                             int x, int y, int z, double (&P)[3]) {
    using S = Stencil<D, ORDER>;
    const long s = ((long)z * m.ny + y) * m.nx + x;
    const double nA = dens[s], nB = dens[m.N + s];
    const double pA = psi_of<double, PSI>(nA), pB = psi_of<double, PSI>(nB);
    double acc[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < S::NE; ++a) {
        constexpr auto T = S::T;
        const int e3[3] = {T.e[a][0], T.e[a][1], T.e[a][2]};
        const int xs = wrap1(x + e3[0], m.nx);
        const int ys = wrap1(y + e3[1], m.ny);
        const int zs = D == 3 ? wrap1(z + e3[2], m.nz) : 0;
        const long t = ((long)zs * m.ny + ys) * m.nx + xs;
        const double nAt = dens[t], nBt = dens[m.N + t];
        const double inter =
            m.g[0][1] * nA * nBt + m.g[1][0] * nB * nAt +
            m.g[0][0] * pA * psi_of<double, PSI>(nAt) +
            m.g[1][1] * pB * psi_of<double, PSI>(nBt);
        for (int k = 0; k < 3; ++k)
            acc[k] += T.W[a] * (double)(e3[k] * e3[k]) * inter;
    }
    const double ideal = (nA + nB) / 3.0;
    for (int k = 0; k < 3; ++k) P[k] = ideal + 0.5 * acc[k];
}

// The full tensor at one site: xx, yy, zz, xy, xz, yz (the diagonal as
// ptensor_diag).
template <int D, int ORDER, int PSI>
__device__ void ptensor_full(const Member &m, const double *__restrict__ dens,
                             int x, int y, int z, double (&P)[6]) {
    using S = Stencil<D, ORDER>;
    const long s = ((long)z * m.ny + y) * m.nx + x;
    const double nA = dens[s], nB = dens[m.N + s];
    const double pA = psi_of<double, PSI>(nA), pB = psi_of<double, PSI>(nB);
    double acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < S::NE; ++a) {
        constexpr auto T = S::T;
        const int e3[3] = {T.e[a][0], T.e[a][1], T.e[a][2]};
        const int xs = wrap1(x + e3[0], m.nx);
        const int ys = wrap1(y + e3[1], m.ny);
        const int zs = D == 3 ? wrap1(z + e3[2], m.nz) : 0;
        const long t = ((long)zs * m.ny + ys) * m.nx + xs;
        const double nAt = dens[t], nBt = dens[m.N + t];
        const double inter =
            m.g[0][1] * nA * nBt + m.g[1][0] * nB * nAt +
            m.g[0][0] * pA * psi_of<double, PSI>(nAt) +
            m.g[1][1] * pB * psi_of<double, PSI>(nBt);
        constexpr int MU[6] = {0, 1, 2, 0, 0, 1}, NU[6] = {0, 1, 2, 1, 2, 2};
        for (int k = 0; k < 6; ++k)
            acc[k] += T.W[a] * (double)(e3[MU[k]] * e3[NU[k]]) * inter;
    }
    const double ideal = (nA + nB) / 3.0;
    for (int k = 0; k < 6; ++k) P[k] = (k < 3 ? ideal : 0.0) + 0.5 * acc[k];
}

// Bulk pressure (eq. bulkp, e2 = 1) of the concentrations at one site.
template <int PSI>
__device__ double bulk_pressure(const Member &m, double nA, double nB) {
    const double pA = psi_of<double, PSI>(nA), pB = psi_of<double, PSI>(nB);
    return (nA + nB) / 3.0 + m.g[0][1] * nA * nB + 0.5 * m.g[0][0] * pA * pA +
           0.5 * m.g[1][1] * pB * pB;
}

// One block: the axis line r = 0..rmax along +x from the centre node, the
// two pressure probes, and C_d = int r^(d-1) (P_out - P_T) dr with P_T linear
// between nodes (each cell integrated exactly).
constexpr int LINE_THREADS = 256;
template <int D, int ORDER, int PSI>
__global__ void __launch_bounds__(LINE_THREADS)
    k_line(Member m, const double *__restrict__ dens, double *__restrict__ out) {
    __shared__ double red[1][LINE_THREADS / 64];
    const int cx = m.nx / 2, cy = m.ny / 2, cz = D == 3 ? m.nz / 2 : 0;
    const int rmax = m.nx / 2;
    const int tid = threadIdx.x;
    const long sc = ((long)cz * m.ny + cy) * m.nx + cx;
    const int ox = (cx + m.nx / 2) % m.nx, oy = (cy + m.ny / 2) % m.ny;
    const int oz = D == 3 ? (cz + m.nz / 2) % m.nz : 0;
    const long so = ((long)oz * m.ny + oy) * m.nx + ox;
    const double Pout = bulk_pressure<PSI>(m, dens[so], dens[m.N + so]);
    for (int r = tid; r <= rmax; r += LINE_THREADS) {
        double P[3];
        ptensor_diag<D, ORDER, PSI>(m, dens, (cx + r) % m.nx, cy, cz, P);
        out[r] = P[0];
        out[(rmax + 1) + r] = P[1];
        out[2 * (rmax + 1) + r] = P[2];
    }
    __syncthreads();
    // exact integral of r^(d-1) times the linear interpolant on [r, r+1]
    double acc = 0;
    const double mexp = D - 1;
    for (int r = tid; r < rmax; r += LINE_THREADS) {
        const double g0 = Pout - out[(rmax + 1) + r];
        const double g1 = Pout - out[(rmax + 1) + r + 1];
        const double a = r, b = r + 1.0;
        const double I0 = (pow(b, mexp + 1) - pow(a, mexp + 1)) / (mexp + 1);
        const double I1 =
            (pow(b, mexp + 2) - pow(a, mexp + 2)) / (mexp + 2) - a * I0;
        acc += g0 * I0 + (g1 - g0) * I1;
    }
    double v[1] = {acc};
    block_reduce<1, LINE_THREADS>(v, red, tid, add_op);
    if (tid == 0) {
        out[3 * (rmax + 1)] = bulk_pressure<PSI>(m, dens[sc], dens[m.N + sc]);
        out[3 * (rmax + 1) + 1] = Pout;
        out[3 * (rmax + 1) + 2] = v[0];
    }
}

// Shell-averaged profiles (a variant of the axis line): the node x at
// distance r = |x - c| from the centre node c = floor(L/2) (no periodic
// image) is in shell k = floor(r + 1/2); with u = (x - c) / r it carries
// P_N = u.P.u and P_T = (tr P - P_N) / (d - 1) (tr P / d at the centre).
// Block b sums the nodes [b per, (b + 1) per) of shells 0..rmax in a fixed
// order: the block stages 256 nodes in LDS, then the thread that owns shell
// k (k mod 256, up to SH_MAXQ shells each) adds the staged nodes of shell k
// one by one, so every sum has the same order on every run.
constexpr int SH_THREADS = 256, SH_MAXQ = 4;
template <int D, int ORDER, int PSI>
__global__ void __launch_bounds__(SH_THREADS)
    k_shell(Member m, int rmax, long per, const double *__restrict__ dens,
            double *__restrict__ partials) {
    __shared__ int key[SH_THREADS];
    __shared__ double vn[SH_THREADS], vt[SH_THREADS];
    const int tid = threadIdx.x, nshell = rmax + 1;
    const int nxy = m.nx * m.ny;
    const int cx = m.nx / 2, cy = m.ny / 2, cz = D == 3 ? m.nz / 2 : 0;
    double aN[SH_MAXQ], aT[SH_MAXQ], aC[SH_MAXQ];
#pragma unroll
    for (int q = 0; q < SH_MAXQ; ++q) aN[q] = aT[q] = aC[q] = 0;
    const long s0 = (long)blockIdx.x * per, s1 = min((long)m.N, s0 + per);
    for (long base = s0; base < s1; base += SH_THREADS) {
        const long s = base + tid;
        int k = -1;
        double pn = 0, pt = 0;
        if (s < s1) {
            const int z = (int)(s / nxy), rr = (int)(s - (long)z * nxy);
            const int y = rr / m.nx, x = rr - y * m.nx;
            const double v[3] = {(double)(x - cx), (double)(y - cy), (double)(z - cz)};
            const double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            k = (int)floor(sqrt(r2) + 0.5);
            if (k <= rmax) {
                double P[6];
                ptensor_full<D, ORDER, PSI>(m, dens, x, y, z, P);
                const double tr = P[0] + P[1] + (D == 3 ? P[2] : 0.0);
                pn = r2 == 0 ? tr / D
                             : (v[0] * v[0] * P[0] + v[1] * v[1] * P[1] + v[2] * v[2] * P[2] +
                                2.0 * v[0] * v[1] * P[3] + 2.0 * v[0] * v[2] * P[4] +
                                2.0 * v[1] * v[2] * P[5]) / r2;
                pt = (tr - pn) / (D - 1);
            } else {
                k = -1;
            }
        }
        key[tid] = k;
        vn[tid] = pn;
        vt[tid] = pt;
        __syncthreads();
        for (int j = 0; j < SH_THREADS; ++j) {
            const int kj = key[j];
#pragma unroll
            for (int q = 0; q < SH_MAXQ; ++q)
                if (kj == tid + q * SH_THREADS) {
                    aN[q] += vn[j];
                    aT[q] += vt[j];
                    aC[q] += 1.0;
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < SH_MAXQ; ++q) {
        const int k = tid + q * SH_THREADS;
        if (k < nshell) {
            double *o = partials + ((long)blockIdx.x * nshell + k) * 3;
            o[0] = aN[q];
            o[1] = aT[q];
            o[2] = aC[q];
        }
    }
}

// Shell means over the blocks in order, the two pressure probes and
// C_d = int r^(d-1) (P_out - P_T) dr on the shell profile (P_T linear
// between shells, each cell integrated exactly, summed in order of r):
// out[k], out[nshell + k] = P_N, P_T of shell k; out[2 nshell ..] = P_in,
// P_out, C_d.
template <int D, int PSI>
__global__ void __launch_bounds__(SH_THREADS)
    k_shell_final(Member m, int rmax, int nb, const double *__restrict__ dens,
                  const double *__restrict__ partials, double *__restrict__ out) {
    const int tid = threadIdx.x, nshell = rmax + 1;
    for (int k = tid; k < nshell; k += SH_THREADS) {
        double sn = 0, st = 0, sc = 0;
        for (int b = 0; b < nb; ++b) {
            const double *p = partials + ((long)b * nshell + k) * 3;
            sn += p[0];
            st += p[1];
            sc += p[2];
        }
        out[k] = sn / sc;
        out[nshell + k] = st / sc;
    }
    __syncthreads();
    if (tid != 0) return;
    const int cx = m.nx / 2, cy = m.ny / 2, cz = D == 3 ? m.nz / 2 : 0;
    const long sc = ((long)cz * m.ny + cy) * m.nx + cx;
    const int ox = (cx + m.nx / 2) % m.nx, oy = (cy + m.ny / 2) % m.ny;
    const int oz = D == 3 ? (cz + m.nz / 2) % m.nz : 0;
    const long so = ((long)oz * m.ny + oy) * m.nx + ox;
    const double Pout = bulk_pressure<PSI>(m, dens[so], dens[m.N + so]);
    double Cd = 0;
    const double mexp = D - 1;
    for (int r = 0; r < rmax; ++r) {
        const double g0 = Pout - out[nshell + r], g1 = Pout - out[nshell + r + 1];
        const double a = r, b = r + 1.0;
        const double I0 = (pow(b, mexp + 1) - pow(a, mexp + 1)) / (mexp + 1);
        const double I1 = (pow(b, mexp + 2) - pow(a, mexp + 2)) / (mexp + 2) - a * I0;
        Cd += g0 * I0 + (g1 - g0) * I1;
    }
    out[2 * nshell] = bulk_pressure<PSI>(m, dens[sc], dens[m.N + sc]);
    out[2 * nshell + 1] = Pout;
    out[2 * nshell + 2] = Cd;
}

// One block per x: transverse averages of P^xx and P^yy.
constexpr int FLAT_THREADS = 256;
template <int D, int ORDER, int PSI>
__global__ void __launch_bounds__(FLAT_THREADS)
    k_flat(Member m, const double *__restrict__ dens, double *__restrict__ out) {
    __shared__ double red[2][FLAT_THREADS / 64];
    const int x = blockIdx.x, tid = threadIdx.x;
    const int ntr = m.ny * m.nz;
    double pn = 0, pt = 0;
    for (int k = tid; k < ntr; k += FLAT_THREADS) {
        double P[3];
        ptensor_diag<D, ORDER, PSI>(m, dens, x, k % m.ny, k / m.ny, P);
        pn += P[0];
        pt += P[1];
    }
    double v[2] = {pn, pt};
    block_reduce<2, FLAT_THREADS>(v, red, tid, add_op);
    if (tid == 0) {
        out[x] = v[0] / ntr;
        out[m.nx + x] = v[1] / ntr;
    }
}

// sigma0 = sum_{x = nx/2}^{nx-1} (P_N - P_T), sequential (nx <= a few 1000)
__global__ void k_flat_sigma(int nx, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0;
        for (int x = nx / 2; x < nx; ++x) s += out[x] - out[nx + x];
        out[2 * nx] = s;
    }
}

// ---------------------------------------------------------------- dispatch
template <class F> static bool dispatch_all(const StepKey &k, F &&fn) {
    auto with_st = [&](auto stv) {
        auto go = [&](auto Dc, auto Oc) {
            if (k.psi == 0)
                fn(stv, Dc, Oc, std::integral_constant<int, 0>{});
            else
                fn(stv, Dc, Oc, std::integral_constant<int, 1>{});
        };
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        using O4 = std::integral_constant<int, 4>;
        using O6 = std::integral_constant<int, 6>;
        using O8 = std::integral_constant<int, 8>;
        if (k.dim == 2 && k.order == 4) return go(I2{}, O4{}), true;
        if (k.dim == 2 && k.order == 6) return go(I2{}, O6{}), true;
        if (k.dim == 2 && k.order == 8) return go(I2{}, O8{}), true;
        if (k.dim == 3 && k.order == 4) return go(I3{}, O4{}), true;
        if (k.dim == 3 && k.order == 6) return go(I3{}, O6{}), true;
        return false;
    };
    switch (k.storage) {
        case ST_F64: return with_st(StoreF64{});
        case ST_F32: return with_st(StoreF32{});
        case ST_F16: return with_st(StoreF16{});
        case ST_BF16: return with_st(StoreBF16{});
    }
    return false;
}

static dim3 ob_grid(const Member &m) {
    return dim3((m.nx + OB_BX - 1) / OB_BX, (m.ny + OB_BY - 1) / OB_BY, m.nz);
}

// ---- convergence monitor (Sec. 4): delta u between two velocity fields
// and the centre of the rich component's excess concentration.
// slots: 0 sum_x sum_a |u_a - u0_a|, 1 sum_x ex, 2..4 sum_x ex (x_a - c_a),
// with ex = n_rich(x) - n_rich_out and c_a = floor(L_a / 2).
constexpr int NMON = 5;

__global__ void __launch_bounds__(OB_THREADS)
    k_monitor(Member m, int dim, const double *__restrict__ dens,
              const double *__restrict__ u, const double *__restrict__ u0, int rich,
              double n_out, double *__restrict__ partials) {
    __shared__ double red[NMON][OB_THREADS / 64];
    const int tid = threadIdx.y * OB_BX + threadIdx.x;
    const int x = blockIdx.x * OB_BX + threadIdx.x;
    const int y = blockIdx.y * OB_BY + threadIdx.y;
    const int z = blockIdx.z;
    double v[NMON] = {0, 0, 0, 0, 0};
    if (x < m.nx && y < m.ny) {
        const long s = ((long)z * m.ny + y) * m.nx + x;
        if (u0)
            for (int a = 0; a < dim; ++a) v[0] += fabs(u[a * (long)m.N + s] - u0[a * (long)m.N + s]);
        const double ex = dens[rich * (long)m.N + s] - n_out;
        v[1] = ex;
        v[2] = ex * (x - m.nx / 2);
        v[3] = ex * (y - m.ny / 2);
        v[4] = dim == 3 ? ex * (z - m.nz / 2) : 0.0;
    }
    block_reduce<NMON, OB_THREADS>(v, red, tid, add_op);
    if (tid == 0) {
        const long b = ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        for (int k = 0; k < NMON; ++k) partials[b * NMON + k] = v[k];
    }
}

__global__ void __launch_bounds__(256)
    k_monitor_final(const double *__restrict__ partials, int nblocks,
                    double *__restrict__ out) {
    __shared__ double red[NMON][256 / 64];
    const int tid = threadIdx.x;
    double v[NMON] = {0, 0, 0, 0, 0};
    for (int b = tid; b < nblocks; b += 256)
        for (int k = 0; k < NMON; ++k) v[k] += partials[(long)b * NMON + k];
    block_reduce<NMON, 256>(v, red, tid, add_op);
    if (tid == 0)
        for (int k = 0; k < NMON; ++k) out[k] = v[k];
}

hipError_t launch_monitor(const Member &m, int dim, const double *dens64, const double *u,
                          const double *u0, int rich, double n_out, double *partials,
                          double *out, hipStream_t st) {
    const dim3 g((m.nx + OB_BX - 1) / OB_BX, (m.ny + OB_BY - 1) / OB_BY, m.nz);
    hipLaunchKernelGGL(k_monitor, g, dim3(OB_BX, OB_BY), 0, st, m, dim, dens64, u, u0,
                       rich, n_out, partials);
    const int nb = (int)(g.x * g.y * g.z);
    hipLaunchKernelGGL(k_monitor_final, dim3(1), dim3(256), 0, st, partials, nb, out);
    return hipGetLastError();
}

int stats_blocks(const Member &m) {
    const dim3 g = ob_grid(m);
    return (int)(g.x * g.y * g.z);
}

hipError_t launch_density64(const StepKey &k, const Member &m, const void *pop,
                            double *dens64, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    dispatch_all(k, [&](auto stv, auto Dc, auto, auto) {
        using ST = decltype(stv);
        constexpr int D = decltype(Dc)::value;
        hipLaunchKernelGGL((k_density64<D, ST>), ob_grid(m),
                           dim3(OB_BX, OB_BY), 0, st, m,
                           (const typename ST::T *)pop, dens64);
        err = hipGetLastError();
    });
    return err;
}

hipError_t launch_stats(const StepKey &k, const Member &m, const void *pop,
                        const double *dens64, double *partials, int nblocks_max,
                        double *out, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    const int nb = stats_blocks(m);
    if (nb > nblocks_max) return hipErrorInvalidValue;
    dispatch_all(k, [&](auto stv, auto Dc, auto Oc, auto Pc) {
        using ST = decltype(stv);
        constexpr int D = decltype(Dc)::value;
        constexpr int O = decltype(Oc)::value;
        constexpr int P = decltype(Pc)::value;
        hipLaunchKernelGGL((k_stats<D, O, ST, P>), ob_grid(m),
                           dim3(OB_BX, OB_BY), 0, st, m,
                           (const typename ST::T *)pop, dens64, partials);
        hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, st, partials,
                           nb, out);
        err = hipGetLastError();
    });
    return err;
}

hipError_t launch_velocity64(const StepKey &k, const Member &m, const void *pop,
                             const double *dens64, double *u, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    dispatch_all(k, [&](auto stv, auto Dc, auto Oc, auto Pc) {
        using ST = decltype(stv);
        constexpr int D = decltype(Dc)::value;
        constexpr int O = decltype(Oc)::value;
        constexpr int P = decltype(Pc)::value;
        hipLaunchKernelGGL((k_velocity64<D, O, ST, P>), ob_grid(m),
                           dim3(OB_BX, OB_BY), 0, st, m,
                           (const typename ST::T *)pop, dens64, u);
        err = hipGetLastError();
    });
    return err;
}

hipError_t launch_line(const StepKey &k, const Member &m, const double *dens64,
                       double *out, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    dispatch_all(k, [&](auto, auto Dc, auto Oc, auto Pc) {
        constexpr int D = decltype(Dc)::value;
        constexpr int O = decltype(Oc)::value;
        constexpr int P = decltype(Pc)::value;
        hipLaunchKernelGGL((k_line<D, O, P>), dim3(1), dim3(LINE_THREADS), 0,
                           st, m, dens64, out);
        err = hipGetLastError();
    });
    return err;
}

int shell_rmax(const Member &m, int dim) {
    int e = std::min(m.nx, m.ny);
    if (dim == 3) e = std::min(e, m.nz);
    return e / 2;
}

hipError_t launch_shell(const StepKey &k, const Member &m, const double *dens64,
                        double *partials, long partial_capacity, double *out,
                        hipStream_t st) {
    const int rmax = shell_rmax(m, k.dim), nshell = rmax + 1;
    if (nshell > SH_THREADS * SH_MAXQ) return hipErrorInvalidValue;
    // blocks: at most 1024, as many as the partials hold (3 values per shell)
    long nb = std::min(1024L, partial_capacity / (3L * nshell));
    if (nb < 1) return hipErrorInvalidValue;
    const long per = ((m.N + nb - 1) / nb + SH_THREADS - 1) / SH_THREADS * SH_THREADS;
    nb = (m.N + per - 1) / per;
    hipError_t err = hipErrorInvalidValue;
    dispatch_all(k, [&](auto, auto Dc, auto Oc, auto Pc) {
        constexpr int D = decltype(Dc)::value;
        constexpr int O = decltype(Oc)::value;
        constexpr int P = decltype(Pc)::value;
        hipLaunchKernelGGL((k_shell<D, O, P>), dim3((unsigned)nb), dim3(SH_THREADS), 0, st, m,
                           rmax, per, dens64, partials);
        hipLaunchKernelGGL((k_shell_final<D, P>), dim3(1), dim3(SH_THREADS), 0, st, m, rmax,
                           (int)nb, dens64, partials, out);
        err = hipGetLastError();
    });
    return err;
}

hipError_t launch_flat(const StepKey &k, const Member &m, const double *dens64,
                       double *out, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    dispatch_all(k, [&](auto, auto Dc, auto Oc, auto Pc) {
        constexpr int D = decltype(Dc)::value;
        constexpr int O = decltype(Oc)::value;
        constexpr int P = decltype(Pc)::value;
        hipLaunchKernelGGL((k_flat<D, O, P>), dim3(m.nx), dim3(FLAT_THREADS), 0,
                           st, m, dens64, out);
        hipLaunchKernelGGL(k_flat_sigma, dim3(1), dim3(64), 0, st, m.nx, out);
        err = hipGetLastError();
    });
    return err;
}

}  // namespace scmc
