// site_ops.h -- per-site operators of the two-component Shan-Chen step, shared
// by every kernel design (paper Sec. 2):
//   pull:     f_i^J(x, t) = f*_i^J(x - xi_i, t - 1)        (eq. lbm, streaming)
//   density:  n_J = sum_i f_i^J
//   force:    F_J = -g_JK n_J sum_a W_a n_K(x + e_a) e_a
//                   -g_JJ psi_J sum_a W_a psi_J(x + e_a) e_a   (eq. sc_force)
//   velocity: (n_A + n_B) u = sum_J [sum_i f_i^J xi_i + F_J / 2]
//   collide:  f* = f - omega_J (f - f^eq(n_J, u)) + (1 - omega_J/2) S_i(u, F_J)
//             f^eq = n w_i [1 + 3 xi.u + 9/2 (xi.u)^2 - 3/2 u.u]
//             S_i  = w_i [3 xi.F + 9 (xi.u)(xi.F) - 3 u.F]     (c_s^2 = 1/3)
#pragma once

#include "lattice.h"
#include "scmc_internal.h"

namespace scmc {

__device__ __forceinline__ int wrap1(int v, int n) {
    // periodic wrap of v in [-n, 2n)
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// 32-bit integer hash (xor-shift-multiply finaliser, constants from
// C. Wellons' "lowbias32") used to seed the stochastic-rounding stream.
__host__ __device__ __forceinline__ unsigned hash32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Random stream of one site and step: a hashed key, then a linear
// congruential step per stored value (its top 16 bits are used).
struct SiteRng {
    unsigned s;
    __device__ __forceinline__ SiteRng(unsigned seed, unsigned step, unsigned site)
        : s(hash32(seed ^ hash32(step * 0x9E3779B9u ^ hash32(site)))) {}
    __device__ __forceinline__ unsigned next() {
        s = s * 1664525u + 1013904223u;
        return s >> 16;
    }
};

template <class R, int PSI> __device__ __forceinline__ R psi_of(R n) {
    if constexpr (PSI == 0) {
        return n;
    } else {
        return exp(R(-1) / n);
    }
}

// Pull the 2Q populations of site (x, y, z) from the post-collision buffer.
// NT: populations with xi_x = 0 (whole cache lines per wavefront) are loaded
// non-temporally; the shifted ones keep their lines in L2 for the wavefront
// that shares them.
template <int D, class ST, bool NT = false>
__device__ __forceinline__ void pull_site(
    const Member &m, const typename ST::T *__restrict__ src, int x, int y,
    int z, typename ST::R (&f)[2][Lattice<D>::Q]) {
    using L = Lattice<D>;
    using R = typename ST::R;
    const typename ST::T *base = src + m.pop_off;
    const R n0A = (R)m.n0[0], n0B = (R)m.n0[1];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap1(x - L::CX[i], m.nx);
        const int ys = wrap1(y - L::CY[i], m.ny);
        const int zs = D == 3 ? wrap1(z - L::CZ[i], m.nz) : 0;
        const long s = ((long)zs * m.ny + ys) * m.nx + xs;
        const R w = (R)L::W[i];
        if (NT && L::CX[i] == 0) {
            f[0][i] = ST::from_raw(__builtin_nontemporal_load(base + (long)i * m.N + s), w * n0A);
            f[1][i] = ST::from_raw(__builtin_nontemporal_load(base + (long)(L::Q + i) * m.N + s),
                                   w * n0B);
        } else {
            f[0][i] = ST::load(base, (long)i * m.N + s, w * n0A);
            f[1][i] = ST::load(base, (long)(L::Q + i) * m.N + s, w * n0B);
        }
    }
}

// Order-free sums.  Every sum over populations or stencil neighbours is
// accumulated in FP64: a handful of FP32 values, or products of two FP32
// values, add up exactly there, so the result does not depend on the order of
// the terms.  A mirror reflection of the lattice only permutes those terms
// (and flips signs, which round symmetrically), so with FP32 storage the step
// commutes bit for bit with the reflections: a droplet centred on a node
// keeps its centre, which the convergence gate of Sec. 4 checks to 1e-3,
// instead of being pushed by the same rounding bias every step.
template <int D, class R>
__device__ __forceinline__ void site_density(const R (&f)[2][Lattice<D>::Q],
                                             R &nA, R &nB) {
    double a = 0, b = 0;
#pragma unroll
    for (int i = 0; i < Lattice<D>::Q; ++i) {
        a += (double)f[0][i];
        b += (double)f[1][i];
    }
    nA = (R)a;
    nB = (R)b;
}

// Stencil sums of eq. sc_force around site (x, y, z), with the stencil
// concentrations returned by fetch(t, n_A, n_B) (t = linear site index times
// UNIT, e.g. a byte offset into an array of (n_A, n_B) pairs), then the force
// on both components.  The stencil is point-symmetric, so the sum runs over
// pairs (e, -e): W e (Phi(x + e) - Phi(x - e)).  The difference is exactly
// odd under e -> -e and the pair sums are accumulated in FP64 (the order-free
// sums above).
template <int D, int ORDER, int PSI, class R, int UNIT = 1, class Fetch>
__device__ __forceinline__ void site_force_fn(const Member &m, int x, int y, int z,
                                              R nA, R nB, R (&FA)[3], R (&FB)[3],
                                              Fetch &&fetch) {
    using S = Stencil<D, ORDER>;
    static_assert(S::point_symmetric(), "stencil table must list e and -e mirrored");
    double cA[3] = {0, 0, 0}, cB[3] = {0, 0, 0};
    double sA[3] = {0, 0, 0}, sB[3] = {0, 0, 0};
    const bool selfA = m.self_on & 1, selfB = m.self_on & 2;
    // periodic column, row and plane offsets of x + d, y + d, z + d for
    // d = -2..2, formed once: a stencil neighbour is then two additions
    int xo[5], yo[5], zo[5];
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
        xo[d + 2] = wrap1(x + d, m.nx) * UNIT;
        yo[d + 2] = wrap1(y + d, m.ny) * (m.nx * UNIT);
        zo[d + 2] = D == 3 ? wrap1(z + d, m.nz) * (m.nx * m.ny * UNIT) : 0;
    }
#pragma unroll
    for (int a = S::NE / 2; a < S::NE; ++a) {
        constexpr auto T = S::T;
        const int ex = T.e[a][0], ey = T.e[a][1], ez = T.e[a][2];
        const int tp = zo[2 + ez] + yo[2 + ey] + xo[2 + ex];
        const int tm = zo[2 - ez] + yo[2 - ey] + xo[2 - ex];
        R pAt, pBt, mAt, mBt;  // N * UNIT < 2^31 (the callers' forms)
        fetch(tp, pAt, pBt);
        fetch(tm, mAt, mBt);
        const R dA = pAt - mAt, dB = pBt - mBt;
        const R W = (R)T.W[a];
        const int e3[3] = {ex, ey, ez};
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (e3[k] == 0) continue;
            const double We = (double)(W * (R)e3[k]);
            cA[k] += We * (double)dB;
            cB[k] += We * (double)dA;
        }
        // with psi = n the self sums equal the cross sums (sA = cB, sB = cA)
        if (PSI != 0 && (selfA || selfB)) {
            const R qA = psi_of<R, PSI>(pAt) - psi_of<R, PSI>(mAt);
            const R qB = psi_of<R, PSI>(pBt) - psi_of<R, PSI>(mBt);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                if (e3[k] == 0) continue;
                const double We = (double)(W * (R)e3[k]);
                sA[k] += We * (double)qA;
                sB[k] += We * (double)qB;
            }
        }
    }
    const R gAB = (R)m.g[0][1], gBA = (R)m.g[1][0];
    const R gAA = (R)m.g[0][0], gBB = (R)m.g[1][1];
    const R pA = selfA ? psi_of<R, PSI>(nA) : R(0);
    const R pB = selfB ? psi_of<R, PSI>(nB) : R(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R tA = (R)(PSI == 0 ? cB[k] : sA[k]), tB = (R)(PSI == 0 ? cA[k] : sB[k]);
        FA[k] = -gAB * nA * (R)cA[k] - gAA * pA * tA;
        FB[k] = -gBA * nB * (R)cB[k] - gBB * pB * tB;
    }
}

// The same from a density field laid out [J][z][y][x] (dA, dB).
template <int D, int ORDER, int PSI, class R>
__device__ __forceinline__ void site_force(const Member &m,
                                           const R *__restrict__ dA,
                                           const R *__restrict__ dB, int x,
                                           int y, int z, R nA, R nB, R (&FA)[3],
                                           R (&FB)[3]) {
    site_force_fn<D, ORDER, PSI, R>(m, x, y, z, nA, nB, FA, FB,
                                    [&](int t, R &a, R &b) {
                                        a = dA[t];
                                        b = dB[t];
                                    });
}

// Common velocity, BGK collision with Guo forcing; every f*_i^J is handed to
// sink(J, i, value, w_i n0_J) as soon as it is formed.
template <int D, class R, class Sink>
__device__ __forceinline__ void site_collide(const Member &m,
                                             const R (&f)[2][Lattice<D>::Q],
                                             R nA, R nB, const R (&FA)[3],
                                             const R (&FB)[3], Sink &&sink) {
    using L = Lattice<D>;
    double jx[2] = {0, 0}, jy[2] = {0, 0}, jz[2] = {0, 0};  // order-free sums (see site_density)
#pragma unroll
    for (int J = 0; J < 2; ++J)
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (L::CX[i]) jx[J] += (double)L::CX[i] * (double)f[J][i];
            if (L::CY[i]) jy[J] += (double)L::CY[i] * (double)f[J][i];
            if (D == 3 && L::CZ[i]) jz[J] += (double)L::CZ[i] * (double)f[J][i];
        }
    R ux, uy, uz;
    if (m.omega[0] == m.omega[1]) {
        // common velocity of Sec. 2
        const R inv = R(1) / (nA + nB);
        ux = ((R)(jx[0] + jx[1]) + R(0.5) * (FA[0] + FB[0])) * inv;
        uy = ((R)(jy[0] + jy[1]) + R(0.5) * (FA[1] + FB[1])) * inv;
        uz = D == 3 ? ((R)(jz[0] + jz[1]) + R(0.5) * (FA[2] + FB[2])) * inv : R(0);
    } else {
        // tau_A != tau_B: each component's momentum and density weighted by
        // omega_J = 1 / tau_J, the form under which the collisions change the
        // total momentum by exactly sum_J F_J
        const R oA = (R)m.omega[0], oB = (R)m.omega[1];
        const R inv = R(1) / (oA * nA + oB * nB);
        ux = (oA * ((R)jx[0] + R(0.5) * FA[0]) + oB * ((R)jx[1] + R(0.5) * FB[0])) * inv;
        uy = (oA * ((R)jy[0] + R(0.5) * FA[1]) + oB * ((R)jy[1] + R(0.5) * FB[1])) * inv;
        uz = D == 3 ? (oA * ((R)jz[0] + R(0.5) * FA[2]) + oB * ((R)jz[1] + R(0.5) * FB[2])) * inv
                    : R(0);
    }
    const R uu = ux * ux + uy * uy + uz * uz;
    const R n0[2] = {(R)m.n0[0], (R)m.n0[1]};
    constexpr Opposite<D> OP = Opposite<D>::make();
    // Velocities xi and -xi are collided together: with t = omega n_J xi.u,
    //   E = w [a_J + 9/2 (xi.u) (t + 2 c_f xi.F_J)],  O = w [3 t + 3 c_f xi.F_J],
    //   a_J = omega n_J (1 - 3/2 u.u) - 3 c_f u.F_J,  c_f = 1 - omega / 2,
    // f*_xi = (1 - omega) f_xi + (E + O) and f*_-xi = (1 - omega) f_-xi + (E - O)
    // (eq. lbm with the Guo source).  Every velocity pair then runs the same
    // operations on sign-flipped operands, which keeps the step exactly
    // covariant under mirror reflections (see site_density).
#pragma unroll
    for (int J = 0; J < 2; ++J) {
        const R omega = (R)m.omega[J], keep = R(1) - omega, cf = R(1) - R(0.5) * omega;
        const R *F = J == 0 ? FA : FB;
        const R nJ = J == 0 ? nA : nB;
        const R uF = ux * F[0] + uy * F[1] + uz * F[2];
        const R on = omega * nJ;
        const R a = on * (R(1) - R(1.5) * uu) - R(3) * cf * uF;
        double moving = 0, nJx = (double)f[J][0];
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const int ib = OP.opp[i];
            if (ib < i) continue;
            R xu = 0, xF = 0;
            if (L::CX[i]) { xu += (R)L::CX[i] * ux; xF += (R)L::CX[i] * F[0]; }
            if (L::CY[i]) { xu += (R)L::CY[i] * uy; xF += (R)L::CY[i] * F[1]; }
            if (D == 3 && L::CZ[i]) { xu += (R)L::CZ[i] * uz; xF += (R)L::CZ[i] * F[2]; }
            const R w = (R)L::W[i];
            const R t = on * xu, cF = cf * xF;
            const R E = w * (a + R(4.5) * xu * (t + R(2) * cF));
            const R O = w * (R(3) * t + R(3) * cF);
            const R fp = keep * f[J][i] + (E + O);
            const R fm = keep * f[J][ib] + (E - O);
            sink(J, i, fp, w * n0[J]);
            sink(J, ib, fm, w * n0[J]);
            moving += (double)fp + (double)fm;
            nJx += (double)f[J][i] + (double)f[J][ib];
        }
        // rest population from the mass balance sum_i f*_i = sum_i f_i (BGK
        // and the Guo source conserve mass), both sums exact in FP64: rounded
        // weights and re-rounded sums would otherwise bias the mass by the
        // same relative amount every step
        sink(J, 0, (R)(nJx - moving), (R)L::W[0] * n0[J]);
    }
}

// Moments that the collision needs at omega = 1: n_J and the total momentum
// j = sum_J sum_i f_i^J xi_i.  n_J is summed in FP64 (exact for the 2Q
// storage values) and kept as a pair: mom[J] = its nearest compute-precision
// value, mom[5 + J] = the remainder.  The collision's rest population uses
// the exact n_J to close the mass balance, so a steady site conserves mass
// exactly instead of re-rounding the same sum the same way every step.
constexpr int NMOM = 7;  // n_A, n_B, j_x, j_y, j_z, rem(n_A), rem(n_B)

template <int D, class R>
__device__ __forceinline__ void site_moments(const R (&f)[2][Lattice<D>::Q],
                                             R (&mom)[NMOM]) {
    using L = Lattice<D>;
    double nA = 0, nB = 0;
    double jx = 0, jy = 0, jz = 0;  // order-free sums (see site_density)
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        nA += (double)f[0][i];
        nB += (double)f[1][i];
        const double t = (double)f[0][i] + (double)f[1][i];
        if (L::CX[i]) jx += (double)L::CX[i] * t;
        if (L::CY[i]) jy += (double)L::CY[i] * t;
        if (D == 3 && L::CZ[i]) jz += (double)L::CZ[i] * t;
    }
    mom[0] = (R)nA;
    mom[1] = (R)nB;
    mom[2] = (R)jx;
    mom[3] = (R)jy;
    mom[4] = (R)jz;
    mom[5] = (R)(nA - (double)mom[0]);
    mom[6] = (R)(nB - (double)mom[1]);
}

// The collision at omega = 1 (tau = 1), where f* = f^eq(n_J, u) + S_i / 2
// no longer depends on the individual pre-collision populations.  With
// a_J = n_J (1 - 3/2 u.u) - 3/2 u.F_J, a velocity xi and its opposite share
//   E = w [a_J + 9/2 (xi.u) (n_J xi.u + xi.F_J)]
// and differ in the sign of
//   O = w [3 n_J xi.u + 3/2 xi.F_J],   f*_xi = E + O, f*_-xi = E - O.
// Every f*_i^J goes to emit(J, i, value), which stores it and returns the
// value the next step's pull will see (the stored value as decoded).  The
// rest population closes the mass balance sum_i f*_i = n_J against those
// values with the exact n_J: rounded weights (their binary sum is not exactly
// 1) and re-rounded sums would otherwise bias the mass by the same relative
// amount every step.
template <int D, class R, class Emit>
__device__ __forceinline__ void collide_tau1_emit(const R (&mom)[NMOM], const R (&FA)[3],
                                                  const R (&FB)[3], Emit &&emit) {
    using L = Lattice<D>;
    const R nA = mom[0], nB = mom[1];
    const R inv = R(1) / (nA + nB);
    const R ux = (mom[2] + R(0.5) * (FA[0] + FB[0])) * inv;
    const R uy = (mom[3] + R(0.5) * (FA[1] + FB[1])) * inv;
    const R uz = D == 3 ? (mom[4] + R(0.5) * (FA[2] + FB[2])) * inv : R(0);
    const R uu = ux * ux + uy * uy + uz * uz;
    constexpr Opposite<D> OP = Opposite<D>::make();
#pragma unroll
    for (int J = 0; J < 2; ++J) {
        const R *F = J == 0 ? FA : FB;
        const R nJ = J == 0 ? nA : nB;
        const R uF = ux * F[0] + uy * F[1] + uz * F[2];
        const R a = nJ * (R(1) - R(1.5) * uu) - R(1.5) * uF;
        double moving = 0;
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const int ib = OP.opp[i];
            if (ib < i) continue;
            R xu = 0, xF = 0;
            if (L::CX[i]) { xu += (R)L::CX[i] * ux; xF += (R)L::CX[i] * F[0]; }
            if (L::CY[i]) { xu += (R)L::CY[i] * uy; xF += (R)L::CY[i] * F[1]; }
            if (D == 3 && L::CZ[i]) { xu += (R)L::CZ[i] * uz; xF += (R)L::CZ[i] * F[2]; }
            const R w = (R)L::W[i];
            const R t = nJ * xu;
            const R E = w * (a + R(4.5) * xu * (t + xF));
            const R O = w * (R(3) * t + R(1.5) * xF);
            const R fp = emit(J, i, E + O), fm = emit(J, ib, E - O);
            moving += (double)fp + (double)fm;
        }
        const double nJx = (double)nJ + (double)mom[5 + J];
        emit(J, 0, (R)(nJx - moving));
    }
}

// The same with every f*_i^J handed to sink(J, i, value, w_i n0_J), the
// closure taken on the values as formed.
template <int D, class R, class Sink>
__device__ __forceinline__ void collide_tau1(const Member &m, const R (&mom)[NMOM],
                                             const R (&FA)[3], const R (&FB)[3],
                                             Sink &&sink) {
    using L = Lattice<D>;
    const R n0[2] = {(R)m.n0[0], (R)m.n0[1]};
    collide_tau1_emit<D, R>(mom, FA, FB, [&](int J, int i, R v) {
        sink(J, i, v, (R)L::W[i] * n0[J]);
        return v;
    });
}

// ---- per-node-reference offsets (FP16 / BF16 node storage): a population
// collided at node x, which streams to x + e_i, is stored as
// h = f*_i - w_i n_J(x + e_i), with n_J the FP32 densities of the step (the
// moments of its first pass), which a reference field keeps beside the
// buffer.  The node that pulls it decodes it against its own densities, so
// a pull reads one reference pair per node.  The product and the sum are
// rounded on their own (no contraction into a fused multiply-add), so that
// encoding, decoding and the mass closure agree bit for bit wherever they
// are formed.
__device__ __forceinline__ float node_ref(float w, float n) {
#pragma clang fp contract(off)
    return w * n;
}

// The collision of a node-storage site: encodes each moving population
// against the densities nb[i] = (n_A, n_B)(x + e_i) of the node it streams
// to and closes the mass balance on their decoded values, so the rest
// populations, kept in FP32 (restA, restB: they do not stream), absorb the
// rounding of the 2Q - 2 moving offsets and the node's mass is kept as with
// FP32 storage.
template <int D, class ST, class Sink>
__device__ __forceinline__ void collide_tau1_node(const typename ST::R (&mom)[NMOM],
                                                  const typename ST::R (&FA)[3],
                                                  const typename ST::R (&FB)[3],
                                                  const float2 (&nb)[Lattice<D>::Q], Sink &&sink,
                                                  float &restA, float &restB) {
    using L = Lattice<D>;
    using R = typename ST::R;
    collide_tau1_emit<D, R>(mom, FA, FB, [&](int J, int i, R v) {
        if (i == 0) {
            (J == 0 ? restA : restB) = v;
            return v;
        }
        const R ref = node_ref((R)L::W[i], J == 0 ? nb[i].x : nb[i].y);
        const typename ST::T h = ST::to_node(v, ref);
        sink(J, i, h);
        return ST::from_node(h, ref);
    });
}

// Collide and store f* at site s of the member's block of dst.
template <int D, class ST>
__device__ __forceinline__ void site_collide_store(
    const Member &m, const typename ST::R (&f)[2][Lattice<D>::Q],
    typename ST::R nA, typename ST::R nB, const typename ST::R (&FA)[3],
    const typename ST::R (&FB)[3], typename ST::T *__restrict__ dst, long s) {
    using R = typename ST::R;
    typename ST::T *base = dst + m.pop_off;
    if (m.sr) {
        SiteRng rng(m.seed, *m.step_ctr, (unsigned)(m.pop_off + s));
        site_collide<D, R>(m, f, nA, nB, FA, FB, [&](int J, int i, R v, R ref) {
            __builtin_nontemporal_store(ST::to_raw_sr(v, ref, rng.next()),
                                        base + (long)(J * Lattice<D>::Q + i) * m.N + s);
        });
        return;
    }
    site_collide<D, R>(m, f, nA, nB, FA, FB, [&](int J, int i, R v, R ref) {
        ST::store(base, (long)(J * Lattice<D>::Q + i) * m.N + s, v, ref);
    });
}

// The first pass of a two-pass step advances the step counter that seeds the
// second pass's stochastic rounding (one thread of the launch).
__device__ __forceinline__ void advance_step_counter(const Member &m, bool first) {
    if (m.sr && first && threadIdx.x == 0 && threadIdx.y == 0) m.step_ctr[0] += 1u;
}

// ---- raw-buffer access with 32-bit offsets (used by the fused kernels) ----
// One buffer descriptor per component covers its Q planes; lanes pass 32-bit
// byte offsets, the plane offset goes in the scalar offset.  The hardware
// returns 0 for reads and drops writes outside the descriptor's range.
constexpr int BUF_DATA_FORMAT_32 = 0x00020000;
constexpr int BUF_NT = 2;  // cache policy: non-temporal

template <class T> struct RawBuf;
template <> struct RawBuf<float> {
    __device__ __forceinline__ static float load(__amdgpu_buffer_rsrc_t r, int v,
                                                 int s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
    }
    __device__ __forceinline__ static float load_nt(__amdgpu_buffer_rsrc_t r, int v, int s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, BUF_NT));
    }
    __device__ __forceinline__ static void store_nt(float x, __amdgpu_buffer_rsrc_t r,
                                                    int v, int s) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v,
                                              s, BUF_NT);
    }
};
template <> struct RawBuf<uint16_t> {
    __device__ __forceinline__ static uint16_t load(__amdgpu_buffer_rsrc_t r, int v,
                                                    int s) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    }
    __device__ __forceinline__ static uint16_t load_nt(__amdgpu_buffer_rsrc_t r, int v, int s) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, v, s, BUF_NT);
    }
    __device__ __forceinline__ static void store_nt(uint16_t x,
                                                    __amdgpu_buffer_rsrc_t r, int v,
                                                    int s) {
        __builtin_amdgcn_raw_buffer_store_b16(x, r, v, s, BUF_NT);
    }
};

template <class ST> struct PopBuf {
    __amdgpu_buffer_rsrc_t r[2];
    int plane_bytes;  // N * sizeof(T)
};

template <class ST, int Q>
__device__ __forceinline__ PopBuf<ST> make_popbuf(const typename ST::T *pop,
                                                  const Member &m) {
    using T = typename ST::T;
    PopBuf<ST> b;
    const T *base = pop + m.pop_off;
    const unsigned bytes = (unsigned)Q * (unsigned)m.N * (unsigned)sizeof(T);
    b.r[0] = __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes,
                                               BUF_DATA_FORMAT_32);
    b.r[1] = __builtin_amdgcn_make_buffer_rsrc((void *)(base + (long)Q * m.N), (short)0,
                                               (int)bytes, BUF_DATA_FORMAT_32);
    b.plane_bytes = m.N * (int)sizeof(T);
    return b;
}

// Cache policy of a pull through buffer descriptors.  PULL_NT_ALIGNED: the
// populations with xi_x = 0 are loaded non-temporally, as pull_site's NT.
// PULL_NT_ALL: every population is, so that the populations streaming
// through pass 1 of the moment two-pass push less of the moment field it
// writes out of the Infinity Cache before pass 2 reads it (lattices whose
// moment field comes close to that cache's size).
enum PullPolicy : int { PULL_CACHED = 0, PULL_NT_ALIGNED = 1, PULL_NT_ALL = 2 };

// Pull of site (x, y, z) through buffer descriptors (D3Q19); NT is a
// PullPolicy.  NODE: the buffer holds per-node-reference offsets, decoded
// against the reference densities m.ref of the source nodes.
template <class ST, int NT = PULL_CACHED, bool NODE = false>
__device__ __forceinline__ void pull_site_buf(const Member &m, const PopBuf<ST> &b,
                                              int x, int y, int z,
                                              typename ST::R (&f)[2][19]) {
    using L = Lattice<3>;
    using T = typename ST::T;
    using R = typename ST::R;
    const int nxy = m.nx * m.ny;
    int xo[3], yo[3], zo[3];  // index d + 1 holds coordinate + d, wrapped
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        xo[d + 1] = wrap1(x + d, m.nx);
        yo[d + 1] = wrap1(y + d, m.ny) * m.nx;
        zo[d + 1] = wrap1(z + d, m.nz) * nxy;
    }
    const R n0A = (R)m.n0[0], n0B = (R)m.n0[1];
    float2 own = {0.f, 0.f};  // node storage: this node's reference densities
    if constexpr (NODE) own = m.ref[zo[1] + yo[1] + xo[1]];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int s = zo[1 - L::CZ[i]] + yo[1 - L::CY[i]] + xo[1 - L::CX[i]];
        const int voff = s * (int)sizeof(T), soff = i * b.plane_bytes;
        const R w = (R)L::W[i];
        R refA = w * n0A, refB = w * n0B;
        if constexpr (NODE) {
            if (i == 0) {  // the rest populations, FP32 at the node itself
                const float2 r = m.rest[s];
                f[0][0] = r.x;
                f[1][0] = r.y;
                continue;
            }
            refA = node_ref(w, own.x);
            refB = node_ref(w, own.y);
        }
        const bool nt = NT == PULL_NT_ALL || (NT == PULL_NT_ALIGNED && L::CX[i] == 0);
        const T ra = nt ? RawBuf<T>::load_nt(b.r[0], voff, soff)
                        : RawBuf<T>::load(b.r[0], voff, soff);
        const T rb = nt ? RawBuf<T>::load_nt(b.r[1], voff, soff)
                        : RawBuf<T>::load(b.r[1], voff, soff);
        if constexpr (NODE) {
            f[0][i] = ST::from_node(ra, refA);
            f[1][i] = ST::from_node(rb, refB);
        } else {
            f[0][i] = ST::from_raw(ra, refA);
            f[1][i] = ST::from_raw(rb, refB);
        }
    }
}

}  // namespace scmc
