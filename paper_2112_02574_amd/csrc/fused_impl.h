// fused_impl.h -- one kernel per time step: stream + density + Shan-Chen
// force + BGK/Guo collide, z-marching ("2.5D") for D3Q19.
//
// The force at (x, y, z) needs the concentrations of the stencil nodes at the
// same time level (eq. sc_force), which exist only after those nodes have been
// streamed.  A workgroup owns a TX x TY column tile and marches a z-chunk of
// ZC planes.  At every step of the march it
//   1. pulls the lead plane zl (2Q loads per node) over the tile plus a halo
//      of HR nodes in x and y, sums the concentrations and writes them to a
//      ring of planes in LDS; the pulled populations of the tile's own nodes
//      stay in a register ring for ZR more steps;
//   2. after one barrier, collides plane zl - ZR: the stencil concentrations
//      come from the LDS ring (planes zc - ZR .. zc + ZR), the populations
//      from the register ring, and f* is stored with coalesced writes.
// HR = ZR = 1 for E4 (nearest neighbours) and 2 for E6 (the (2, 0, 0) shell).
// The ring holds 2 ZR + 2 planes, so a single barrier per plane suffices: the
// plane written at step k + 1 is never one read at step k.
// HBM traffic per site is the 2Q reads + 2Q writes of the populations; the
// halo and the 2 ZR warm-up planes are extra pulls that mostly hit in L2 / the
// Infinity Cache.  Workgroups are numbered so that the tiles of one z-chunk
// (which share y-halo rows) land on the same XCD.
#pragma once

#include "site_ops.h"

namespace scmc {

constexpr int NXCD = 8;

template <int ORDER> struct FusedGeom {
    static constexpr int HR = ORDER == 4 ? 1 : 2;   // halo in x, y
    static constexpr int ZR = ORDER == 4 ? 1 : 2;   // reach in z
    static constexpr int NSLOT = 2 * ZR + 2;        // LDS plane ring
    static constexpr int NRING = ZR + 1;            // register plane ring
};

// Linear workgroup id -> logical tile id such that consecutive logical tiles
// share an XCD (the hardware deals workgroups round-robin over the XCDs).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    const int per = nb / NXCD, rem = nb % NXCD;
    const int xcd = bid % NXCD, k = bid / NXCD;
    // XCDs 0..rem-1 own per+1 tiles, the others own per
    const int start = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return start + k;
}

// Concentrations of node (tx, ty) of the plane collided at march step k and
// the Shan-Chen forces on both components, from the LDS concentration ring
// (planes k - 2 ZR .. k of the ring hold z - ZR .. z + ZR).
template <int TX, int TY, int ORDER, class R, int PSI>
__device__ __forceinline__ void lds_force(
    const Member &m,
    float2 (*lds)[TY + 2 * FusedGeom<ORDER>::HR][TX + 2 * FusedGeom<ORDER>::HR],
    int k, int tx, int ty, R &nA, R &nB, R (&FA)[3], R (&FB)[3]) {
    using G = FusedGeom<ORDER>;
    using Sten = Stencil<3, ORDER>;
    constexpr int HR = G::HR, ZR = G::ZR;
    const float2 own = lds[(k - ZR) % G::NSLOT][ty + HR][tx + HR];
    nA = own.x;
    nB = own.y;
    // pairs (e, -e) summed in FP64, as in site_force_fn
    static_assert(Sten::point_symmetric(), "stencil table must list e and -e mirrored");
    double cA[3] = {0, 0, 0}, cB[3] = {0, 0, 0}, sA[3] = {0, 0, 0}, sB[3] = {0, 0, 0};
    const bool selfA = m.self_on & 1, selfB = m.self_on & 2;
#pragma unroll
    for (int a = Sten::NE / 2; a < Sten::NE; ++a) {
        constexpr auto T = Sten::T;
        const int ex = T.e[a][0], ey = T.e[a][1], ez = T.e[a][2];
        const float2 p = lds[(k - ZR + ez) % G::NSLOT][ty + HR + ey][tx + HR + ex];
        const float2 q = lds[(k - ZR - ez) % G::NSLOT][ty + HR - ey][tx + HR - ex];
        const R pAt = p.x, pBt = p.y, mAt = q.x, mBt = q.y;
        const R dA = pAt - mAt, dB = pBt - mBt;
        const R W = (R)T.W[a];
        const int e3[3] = {ex, ey, ez};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (e3[c] == 0) continue;
            const double We = (double)(W * (R)e3[c]);
            cA[c] += We * (double)dB;
            cB[c] += We * (double)dA;
        }
        // with psi = n the self sums equal the cross sums (sA = cB, sB = cA)
        if (PSI != 0 && (selfA || selfB)) {
            const R qA = psi_of<R, PSI>(pAt) - psi_of<R, PSI>(mAt);
            const R qB = psi_of<R, PSI>(pBt) - psi_of<R, PSI>(mBt);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (e3[c] == 0) continue;
                const double We = (double)(W * (R)e3[c]);
                sA[c] += We * (double)qA;
                sB[c] += We * (double)qB;
            }
        }
    }
    const R gAB = (R)m.g[0][1], gBA = (R)m.g[1][0];
    const R gAA = (R)m.g[0][0], gBB = (R)m.g[1][1];
    const R pA = selfA ? psi_of<R, PSI>(nA) : R(0);
    const R pB = selfB ? psi_of<R, PSI>(nB) : R(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R tA = (R)(PSI == 0 ? cB[c] : sA[c]), tB = (R)(PSI == 0 ? cA[c] : sB[c]);
        FA[c] = -gAB * nA * (R)cA[c] - gAA * pA * tA;
        FB[c] = -gBA * nB * (R)cB[c] - gBB * pB * tB;
    }
}

// Force, velocity, collision and store of node (tx, ty) of plane zc, collided
// at march step k, from its pulled populations f.
template <int TX, int TY, int ORDER, class ST, int PSI>
__device__ __forceinline__ void fused_collide(
    const Member &m, const PopBuf<ST> &dst,
    float2 (*lds)[TY + 2 * FusedGeom<ORDER>::HR][TX + 2 * FusedGeom<ORDER>::HR],
    const typename ST::R (&f)[2][19], int k, int x0, int y0, int zc, int tx,
    int ty) {
    using R = typename ST::R;
    using T = typename ST::T;
    R nA, nB, FA[3], FB[3];
    lds_force<TX, TY, ORDER, R, PSI>(m, lds, k, tx, ty, nA, nB, FA, FB);
    const int voff = (((zc * m.ny) + (y0 + ty)) * m.nx + (x0 + tx)) * (int)sizeof(T);
    site_collide<3, R>(m, f, nA, nB, FA, FB, [&](int J, int i, R v, R ref) {
        RawBuf<T>::store_nt(ST::to_raw(v, ref), dst.r[J], voff, i * dst.plane_bytes);
    });
}

// The same at omega = 1 from the node's moments (n_A, n_B, j).
template <int TX, int TY, int ORDER, class ST, int PSI>
__device__ __forceinline__ void fused_collide_mom(
    const Member &m, const PopBuf<ST> &dst,
    float2 (*lds)[TY + 2 * FusedGeom<ORDER>::HR][TX + 2 * FusedGeom<ORDER>::HR],
    const typename ST::R (&mom)[NMOM], int k, int x0, int y0, int zc, int tx, int ty) {
    using R = typename ST::R;
    using T = typename ST::T;
    R nA, nB, FA[3], FB[3];
    lds_force<TX, TY, ORDER, R, PSI>(m, lds, k, tx, ty, nA, nB, FA, FB);
    const int voff = (((zc * m.ny) + (y0 + ty)) * m.nx + (x0 + tx)) * (int)sizeof(T);
    collide_tau1<3, R>(m, mom, FA, FB, [&](int J, int i, R v, R ref) {
        RawBuf<T>::store_nt(ST::to_raw(v, ref), dst.r[J], voff, i * dst.plane_bytes);
    });
}

// Local position (lx, ly) of halo node h of a wx x wy tile with halo HR:
// HR full rows above, then HR nodes left and right of every tile row, then
// HR full rows below.
template <int HR>
__device__ __forceinline__ void halo_pos(int h, int wx, int wy, int &lx, int &ly) {
    const int bw = wx + 2 * HR;
    const int ntop = HR * bw, nmid = wy * 2 * HR;
    if (h < ntop) {
        ly = h / bw;
        lx = h - ly * bw;
    } else if (h < ntop + nmid) {
        const int q = h - ntop;
        ly = HR + q / (2 * HR);
        const int c = q - (ly - HR) * 2 * HR;
        lx = c < HR ? c : wx + c;
    } else {
        const int q = h - ntop - nmid;
        const int r = q / bw;
        ly = HR + wy + r;
        lx = q - r * bw;
    }
}

template <int TX, int TY, int ORDER, class ST, int PSI, int REPULL, int S>
__device__ __forceinline__ void fused_plane(
    const Member &m, const PopBuf<ST> &src, const PopBuf<ST> &dst, float2 (*lds)[TY + 2 * FusedGeom<ORDER>::HR]
                                                   [TX + 2 * FusedGeom<ORDER>::HR],
    typename ST::R (&ring)[REPULL ? 1 : FusedGeom<ORDER>::NRING][2][19], int k, int x0,
    int y0, int z0, int wx, int wy, int tx, int ty, bool active) {
    using G = FusedGeom<ORDER>;
    using R = typename ST::R;
    constexpr int HR = G::HR, ZR = G::ZR;
    constexpr int NT = TX * TY;
    const int tid = ty * TX + tx;
    const int zl = wrap1(z0 - ZR + k, m.nz);
    auto &plane = lds[k % G::NSLOT];

    // ---- phase 1: concentrations of the lead plane over tile + halo
    if (active) {
        auto lead = [&](R(&f)[2][19]) {
            pull_site_buf<ST>(m, src, x0 + tx, y0 + ty, zl, f);
            R nA, nB;
            site_density<3, R>(f, nA, nB);
            plane[ty + HR][tx + HR] = make_float2((float)nA, (float)nB);
        };
        if constexpr (REPULL) {
            R fl[2][19];
            lead(fl);
        } else {
            lead(ring[S]);
        }
    }
    {
        const int nhalo = 2 * HR * (wx + 2 * HR) + wy * 2 * HR;
        for (int h = tid; h < nhalo; h += NT) {
            int lx, ly;
            halo_pos<HR>(h, wx, wy, lx, ly);
            const int gx = wrap1(x0 - HR + lx, m.nx);
            const int gy = wrap1(y0 - HR + ly, m.ny);
            R f[2][19];
            pull_site_buf<ST>(m, src, gx, gy, zl, f);
            R nA, nB;
            site_density<3, R>(f, nA, nB);
            plane[ly][lx] = make_float2((float)nA, (float)nB);
        }
    }
    __syncthreads();

    // ---- phase 2: collide plane zc = zl - ZR
    if (k >= 2 * ZR && active) {
        const int zc = wrap1(z0 + k - 2 * ZR, m.nz);
        if constexpr (REPULL) {
            R fl[2][19];
            pull_site_buf<ST>(m, src, x0 + tx, y0 + ty, zc, fl);
            fused_collide<TX, TY, ORDER, ST, PSI>(m, dst, lds, fl, k, x0, y0, zc,
                                                  tx, ty);
        } else {
            fused_collide<TX, TY, ORDER, ST, PSI>(m, dst, lds,
                                                  ring[(S + 1) % G::NRING], k,
                                                  x0, y0, zc, tx, ty);
        }
    }
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}


// Tiles that span the whole x extent (wx == nx, one tile per row) take their
// x halo from their own rows: the periodic images of the first and last HR
// columns are written to LDS beside the row, and only the HR rows above and
// below are pulled (2 HR wx nodes, coalesced, instead of the general halo).
template <int HR>
__device__ __forceinline__ int halo_count(int wx, int wy, bool full_row) {
    return full_row ? 2 * HR * wx : 2 * HR * (wx + 2 * HR) + wy * 2 * HR;
}

template <int HR>
__device__ __forceinline__ void halo_node(int h, int wx, int wy, bool full_row,
                                          int &lx, int &ly) {
    if (full_row) {
        const int r = h / wx;
        lx = HR + (h - r * wx);
        ly = r < HR ? r : wy + r;
    } else {
        halo_pos<HR>(h, wx, wy, lx, ly);
    }
}

// Store a concentration pair at LDS column lx of a row, plus its periodic
// image when the tile spans the row.
template <int HR, int W>
__device__ __forceinline__ void put_lds(float2 (&row)[W], int lx, float2 v, int wx,
                                        bool full_row) {
    row[lx] = v;
    if (full_row) {
        if (lx < 2 * HR) row[lx + wx] = v;
        else if (lx >= wx) row[lx - wx] = v;
    }
}

// Software-pipelined march: the lead plane's loads (tile and halo) are issued
// one plane ahead, right after the barrier and before the collision, and are
// consumed at the top of the next step.  The collision's stores therefore come
// after those loads, so waiting for the loads never waits for the stores, and
// the load latency overlaps the collision arithmetic.  Every thread owns at
// most one halo node (the tile sizes are chosen so), whose populations wait in
// registers like the tile's own.
template <int TX, int TY, int ORDER, class ST, int PSI>
__device__ __forceinline__ void fused_tile_pipe(const Member &m,
                                                const typename ST::T *__restrict__ src,
                                                typename ST::T *__restrict__ dst,
                                                int x0, int y0, int z0, int len) {
    using G = FusedGeom<ORDER>;
    using R = typename ST::R;
    constexpr int HR = G::HR, ZR = G::ZR, NSLOT = G::NSLOT, NR = ZR + 2;
    __shared__ float2 lds[NSLOT][TY + 2 * HR][TX + 2 * HR];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int wx = min(TX, m.nx - x0), wy = min(TY, m.ny - y0);
    const bool active = tx < wx && ty < wy;
    const int nhalo = 2 * HR * (wx + 2 * HR) + wy * 2 * HR;
    const bool has_halo = tid < nhalo;
    int hlx = 0, hly = 0;
    if (has_halo) halo_pos<HR>(tid, wx, wy, hlx, hly);
    const int hgx = wrap1(x0 - HR + hlx, m.nx), hgy = wrap1(y0 - HR + hly, m.ny);
    const PopBuf<ST> sb = make_popbuf<ST, 19>(src, m);
    const PopBuf<ST> db = make_popbuf<ST, 19>(dst, m);
    R ring[NR][2][19];
    R H[2][19];

    auto put = [&](float2(&plane)[TY + 2 * HR][TX + 2 * HR], int ly, int lx,
                   const R(&f)[2][19]) {
        R nA, nB;
        site_density<3, R>(f, nA, nB);
        plane[ly][lx] = make_float2((float)nA, (float)nB);
    };

    // prologue: planes z0 - ZR .. z0 + ZR - 1, pulled and summed in place
    static_for<-ZR, ZR>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const int z = wrap1(z0 + r, m.nz);
        auto &plane = lds[(r + ZR) % NSLOT];
        if (active) {
            if constexpr (r >= 0) {
                pull_site_buf<ST>(m, sb, x0 + tx, y0 + ty, z, ring[r]);
                put(plane, ty + HR, tx + HR, ring[r]);
            } else {
                R f[2][19];
                pull_site_buf<ST>(m, sb, x0 + tx, y0 + ty, z, f);
                put(plane, ty + HR, tx + HR, f);
            }
        }
        if (has_halo) {
            pull_site_buf<ST>(m, sb, hgx, hgy, z, H);
            put(plane, hly, hlx, H);
        }
    });
    {   // first lead plane z0 + ZR
        const int z = wrap1(z0 + ZR, m.nz);
        if (active) pull_site_buf<ST>(m, sb, x0 + tx, y0 + ty, z, ring[ZR]);
        if (has_halo) pull_site_buf<ST>(m, sb, hgx, hgy, z, H);
    }

    for (int j0 = 0; j0 < len; j0 += NR) {
        static_for<0, NR>([&](auto sc) {
            constexpr int S = decltype(sc)::value;
            const int j = j0 + S;
            if (j < len) {
                // consume the lead plane z0 + j + ZR
                auto &plane = lds[(j + 2 * ZR) % NSLOT];
                if (active) put(plane, ty + HR, tx + HR, ring[(S + ZR) % NR]);
                if (has_halo) put(plane, hly, hlx, H);
                __syncthreads();
                // issue the next lead plane
                if (j + 1 < len) {
                    const int z = wrap1(z0 + j + ZR + 1, m.nz);
                    if (active)
                        pull_site_buf<ST>(m, sb, x0 + tx, y0 + ty, z,
                                          ring[(S + ZR + 1) % NR]);
                    if (has_halo) pull_site_buf<ST>(m, sb, hgx, hgy, z, H);
                }
                // collide plane z0 + j
                if (active)
                    fused_collide<TX, TY, ORDER, ST, PSI>(m, db, lds, ring[S],
                                                          j + 2 * ZR, x0, y0,
                                                          z0 + j, tx, ty);
            }
        });
    }
}

// tiles whose halo has at most one node per thread
template <int TX, int TY, int ORDER> constexpr bool pipe_fits() {
    constexpr int HR = FusedGeom<ORDER>::HR;
    return 2 * HR * (TX + 2 * HR) + TY * 2 * HR <= TX * TY;
}

// March the chunk [z0, z0 + zc_len) of the column tile at (x0, y0).
template <int TX, int TY, int ORDER, class ST, int PSI, int REPULL>
__device__ __forceinline__ void fused_tile(const Member &m,
                                           const typename ST::T *__restrict__ src,
                                           typename ST::T *__restrict__ dst,
                                           int x0, int y0, int z0, int zc_len) {
    using G = FusedGeom<ORDER>;
    using R = typename ST::R;
    constexpr int HR = G::HR;
    __shared__ float2 lds[G::NSLOT][TY + 2 * HR][TX + 2 * HR];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int wx = min(TX, m.nx - x0), wy = min(TY, m.ny - y0);
    const bool active = tx < wx && ty < wy;
    const PopBuf<ST> sb = make_popbuf<ST, 19>(src, m);
    const PopBuf<ST> db = make_popbuf<ST, 19>(dst, m);
    R ring[REPULL ? 1 : G::NRING][2][19];
    const int kend = zc_len + 2 * G::ZR;
    for (int k = 0; k < kend; k += G::NRING) {
        fused_plane<TX, TY, ORDER, ST, PSI, REPULL, 0>(
            m, sb, db, lds, ring, k, x0, y0, z0, wx, wy, tx, ty, active);
        if (k + 1 < kend)
            fused_plane<TX, TY, ORDER, ST, PSI, REPULL, 1>(
                m, sb, db, lds, ring, k + 1, x0, y0, z0, wx, wy, tx, ty, active);
        if constexpr (G::NRING == 3) {
            if (k + 2 < kend)
                fused_plane<TX, TY, ORDER, ST, PSI, REPULL, 2>(
                    m, sb, db, lds, ring, k + 2, x0, y0, z0, wx, wy, tx, ty,
                    active);
        }
    }
}

// ---- omega = 1: moment ring
// At tau = 1 the collision forgets the pre-collision populations except for
// n_J and the total momentum j, so the march keeps those moments per node and
// plane (n_J as an exact value-plus-remainder pair, NMOM values) instead of
// the 2Q populations.  The register ring shrinks from (ZR + 1) x 2Q to
// (ZR + 1) x NMOM values, which lets more waves share a SIMD (and larger
// tiles fit), while the HBM traffic stays 2Q reads + 2Q writes.
template <int TX, int TY, int ORDER, class ST, int PSI>
__device__ __forceinline__ void fused_tile_mom(const Member &m,
                                               const typename ST::T *__restrict__ src,
                                               typename ST::T *__restrict__ dst,
                                               int x0, int y0, int z0, int len) {
    using G = FusedGeom<ORDER>;
    using R = typename ST::R;
    constexpr int HR = G::HR, ZR = G::ZR, NSLOT = G::NSLOT, NR = ZR + 1;
    constexpr int NT = TX * TY;
    __shared__ float2 lds[NSLOT][TY + 2 * HR][TX + 2 * HR];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int wx = min(TX, m.nx - x0), wy = min(TY, m.ny - y0);
    const bool active = tx < wx && ty < wy;
    const bool full_row = wx == m.nx;
    const int nhalo = halo_count<HR>(wx, wy, full_row);
    const PopBuf<ST> sb = make_popbuf<ST, 19>(src, m);
    const PopBuf<ST> db = make_popbuf<ST, 19>(dst, m);
    R mom[NR][NMOM];
    const int kend = len + 2 * ZR;
    for (int k0 = 0; k0 < kend; k0 += NR) {
        static_for<0, NR>([&](auto sc) {
            constexpr int S = decltype(sc)::value;
            const int k = k0 + S;
            if (k >= kend) return;
            // lead plane z0 - ZR + k: moments of the tile, concentrations of
            // tile and halo into LDS
            const int zl = wrap1(z0 - ZR + k, m.nz);
            auto &plane = lds[k % NSLOT];
            if (active) {
                R f[2][19];
                pull_site_buf<ST>(m, sb, x0 + tx, y0 + ty, zl, f);
                site_moments<3, R>(f, mom[S]);
                put_lds<HR>(plane[ty + HR], tx + HR,
                            make_float2((float)mom[S][0], (float)mom[S][1]), wx, full_row);
            }
            for (int h = tid; h < nhalo; h += NT) {
                int lx, ly;
                halo_node<HR>(h, wx, wy, full_row, lx, ly);
                R f[2][19], nA, nB;
                pull_site_buf<ST>(m, sb, wrap1(x0 - HR + lx, m.nx),
                                  wrap1(y0 - HR + ly, m.ny), zl, f);
                site_density<3, R>(f, nA, nB);
                put_lds<HR>(plane[ly], lx, make_float2((float)nA, (float)nB), wx, full_row);
            }
            __syncthreads();
            // collide plane z0 + k - 2 ZR, the lead plane of step k - ZR
            if (k >= 2 * ZR && active)
                fused_collide_mom<TX, TY, ORDER, ST, PSI>(
                    m, db, lds, mom[(S + 1) % NR], k, x0, y0,
                    wrap1(z0 + k - 2 * ZR, m.nz), tx, ty);
        });
    }
}

// The moment ring with the next lead plane's loads (tile and halo) issued
// right after the barrier, before the current collision, as in
// fused_tile_pipe; the loaded populations wait in registers (2 x 2Q values)
// until the top of the next step.
template <int TX, int TY, int ORDER, class ST, int PSI>
__device__ __forceinline__ void fused_tile_mom_pipe(const Member &m,
                                                    const typename ST::T *__restrict__ src,
                                                    typename ST::T *__restrict__ dst,
                                                    int x0, int y0, int z0, int len) {
    using G = FusedGeom<ORDER>;
    using R = typename ST::R;
    constexpr int HR = G::HR, ZR = G::ZR, NSLOT = G::NSLOT, NR = ZR + 1;
    __shared__ float2 lds[NSLOT][TY + 2 * HR][TX + 2 * HR];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int wx = min(TX, m.nx - x0), wy = min(TY, m.ny - y0);
    const bool active = tx < wx && ty < wy;
    const bool full_row = wx == m.nx;
    const int nhalo = halo_count<HR>(wx, wy, full_row);
    const bool has_halo = tid < nhalo;
    int hlx = 0, hly = 0;
    if (has_halo) halo_node<HR>(tid, wx, wy, full_row, hlx, hly);
    const int hgx = wrap1(x0 - HR + hlx, m.nx), hgy = wrap1(y0 - HR + hly, m.ny);
    const PopBuf<ST> sb = make_popbuf<ST, 19>(src, m);
    const PopBuf<ST> db = make_popbuf<ST, 19>(dst, m);
    R mom[NR][NMOM];  // plane z0 + p lives in mom[p % NR]
    R fo[2][19], H[2][19];

    auto put_density = [&](float2(&plane)[TY + 2 * HR][TX + 2 * HR], int ly, int lx,
                           const R(&f)[2][19]) {
        R nA, nB;
        site_density<3, R>(f, nA, nB);
        put_lds<HR>(plane[ly], lx, make_float2((float)nA, (float)nB), wx, full_row);
    };

    // prologue: planes z0 - ZR .. z0 + ZR - 1 into LDS slots 0 .. 2 ZR - 1
    static_for<-ZR, ZR>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const int z = wrap1(z0 + r, m.nz);
        auto &plane = lds[(r + ZR) % NSLOT];
        if (active) {
            pull_site_buf<ST>(m, sb, x0 + tx, y0 + ty, z, fo);
            if constexpr (r >= 0) {
                site_moments<3, R>(fo, mom[r % NR]);
                put_lds<HR>(plane[ty + HR], tx + HR,
                            make_float2((float)mom[r % NR][0], (float)mom[r % NR][1]),
                            wx, full_row);
            } else {
                put_density(plane, ty + HR, tx + HR, fo);
            }
        }
        if (has_halo) {
            pull_site_buf<ST>(m, sb, hgx, hgy, z, H);
            put_density(plane, hly, hlx, H);
        }
    });
    {   // first lead plane z0 + ZR
        const int z = wrap1(z0 + ZR, m.nz);
        if (active) pull_site_buf<ST>(m, sb, x0 + tx, y0 + ty, z, fo);
        if (has_halo) pull_site_buf<ST>(m, sb, hgx, hgy, z, H);
    }
    for (int j0 = 0; j0 < len; j0 += NR) {
        static_for<0, NR>([&](auto sc) {
            constexpr int S = decltype(sc)::value;
            const int j = j0 + S;
            if (j >= len) return;
            // consume the lead plane z0 + j + ZR
            auto &plane = lds[(j + 2 * ZR) % NSLOT];
            if (active) {
                site_moments<3, R>(fo, mom[(S + ZR) % NR]);
                put_lds<HR>(plane[ty + HR], tx + HR,
                            make_float2((float)mom[(S + ZR) % NR][0],
                                        (float)mom[(S + ZR) % NR][1]),
                            wx, full_row);
            }
            if (has_halo) put_density(plane, hly, hlx, H);
            __syncthreads();
            // issue the next lead plane
            if (j + 1 < len) {
                const int z = wrap1(z0 + j + ZR + 1, m.nz);
                if (active) pull_site_buf<ST>(m, sb, x0 + tx, y0 + ty, z, fo);
                if (has_halo) pull_site_buf<ST>(m, sb, hgx, hgy, z, H);
            }
            // collide plane z0 + j
            if (active)
                fused_collide_mom<TX, TY, ORDER, ST, PSI>(m, db, lds, mom[S % NR],
                                                          j + 2 * ZR, x0, y0,
                                                          wrap1(z0 + j, m.nz), tx, ty);
        });
    }
}

// March the column tile (x0, y0), z-chunk [z0, z0 + len) with design VAR.
template <int TX, int TY, int ORDER, class ST, int PSI, int VAR>
__device__ __forceinline__ void fused_tile_any(const Member &m,
                                               const typename ST::T *__restrict__ src,
                                               typename ST::T *__restrict__ dst,
                                               int x0, int y0, int z0, int len) {
    if constexpr (VAR == 2)
        fused_tile_pipe<TX, TY, ORDER, ST, PSI>(m, src, dst, x0, y0, z0, len);
    else if constexpr (VAR == 3)
        fused_tile_mom<TX, TY, ORDER, ST, PSI>(m, src, dst, x0, y0, z0, len);
    else if constexpr (VAR == 4)
        fused_tile_mom_pipe<TX, TY, ORDER, ST, PSI>(m, src, dst, x0, y0, z0, len);
    else
        fused_tile<TX, TY, ORDER, ST, PSI, VAR>(m, src, dst, x0, y0, z0, len);
}

// Waves per SIMD the compiler is asked to allow for: the population-ring
// designs need most of the register file, the moment ring fits three waves
// (four for 1024-thread tiles, which the launch bound imposes), its
// pipelined form (two planes of loads in flight) two.
template <int VAR> constexpr int fused_waves() {
    return VAR == 3 ? 3 : VAR == 4 ? 2 : 1;
}

template <int TX, int TY, int ORDER, class ST, int PSI, int VAR>
__global__ void __launch_bounds__(TX *TY)
    __attribute__((amdgpu_waves_per_eu(fused_waves<VAR>())))
    k_fused(Member m, const typename ST::T *__restrict__ src,
            typename ST::T *__restrict__ dst, int zc_len) {
    const int ntx = (m.nx + TX - 1) / TX, nty = (m.ny + TY - 1) / TY;
    const int nb = gridDim.x;
    const int t = xcd_remap(blockIdx.x, nb);
    const int bx = t % ntx, by = (t / ntx) % nty, bz = t / (ntx * nty);
    const int z0 = bz * zc_len;
    const int len = min(zc_len, m.nz - z0);
    fused_tile_any<TX, TY, ORDER, ST, PSI, VAR>(m, src, dst, bx * TX, by * TY, z0, len);
}

template <int TX, int TY, int ORDER, class ST, int PSI, int VAR>
__global__ void __launch_bounds__(TX *TY)
    __attribute__((amdgpu_waves_per_eu(fused_waves<VAR>())))
    kb_fused(const Member *__restrict__ members, const Tile *__restrict__ tiles,
             int ntiles, const typename ST::T *__restrict__ src,
             typename ST::T *__restrict__ dst, int zc_len) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Member m = members[tl.member];
        const int len = min(zc_len, m.nz - tl.z0);
        fused_tile_any<TX, TY, ORDER, ST, PSI, VAR>(m, src, dst, tl.x0, tl.y0, tl.z0,
                                                    len);
        __syncthreads();  // the next tile reuses the LDS ring
    }
}

// ---------------------------------------------------------------- dispatch
// compiled tiles (TX, TY); the z-chunk is a runtime argument
#define SCMC_FUSED_TILES(X) \
    X(64, 4) X(32, 8) X(64, 8) X(32, 16) X(128, 4) X(128, 8) X(64, 16)

// Designs a tile is compiled for: 1024-thread tiles only with the plain
// moment ring (the others do not fit four waves per SIMD); the pipelined
// designs only where every thread owns at most one halo node.
template <int VAR, int TX, int TY, int ORDER> constexpr bool fused_valid() {
    if (TX * TY > 512 && VAR != 3) return false;
    if ((VAR == 2 || VAR == 4) && !pipe_fits<TX, TY, ORDER>()) return false;
    return true;
}

inline int fused_blocks(const Member &m, const int *tile) {
    const int ntx = (m.nx + tile[0] - 1) / tile[0];
    const int nty = (m.ny + tile[1] - 1) / tile[1];
    const int ntz = (m.nz + tile[2] - 1) / tile[2];
    return ntx * nty * ntz;
}

// Launchers of one storage format and stencil order; each (ST, ORDER) pair is
// instantiated in its own translation unit.
template <class ST, int ORDER> struct FusedOps {
    template <class F> static bool dispatch(const StepKey &k, const int *tile, F &&fn) {
        if (tile[2] < 1) return false;
        bool ok = false;
        auto with_p = [&](auto Pc) {
            auto with_r = [&](auto Rc) {
#define SCMC_TRY(TXv, TYv)                                                   \
    if (tile[0] == TXv && tile[1] == TYv) {                                  \
        if constexpr (fused_valid<decltype(Rc)::value, TXv, TYv, ORDER>()) { \
            fn(Pc, Rc, std::integral_constant<int, TXv>{},                   \
               std::integral_constant<int, TYv>{});                          \
            ok = true;                                                       \
        }                                                                    \
        return;                                                              \
    }
                SCMC_FUSED_TILES(SCMC_TRY)
#undef SCMC_TRY
            };
            switch (k.repull) {
                case 1: with_r(std::integral_constant<int, 1>{}); break;
                case 2: with_r(std::integral_constant<int, 2>{}); break;
                case 3: with_r(std::integral_constant<int, 3>{}); break;
                case 4: with_r(std::integral_constant<int, 4>{}); break;
                default: with_r(std::integral_constant<int, 0>{}); break;
            }
        };
        if (k.psi == 0) with_p(std::integral_constant<int, 0>{});
        else with_p(std::integral_constant<int, 1>{});
        return ok;
    }
    static bool supported(const StepKey &k, const int *tile);
    static hipError_t launch(const StepKey &k, const Member &m, const void *src,
                             void *dst, const int *tile, hipStream_t st);
    static bool node(const StepKey &k, const int *tile, NodeLaunch *node,
                     const Member &m);
    static hipError_t launch_batch(const StepKey &k, const Member *d_members,
                                   const Tile *d_tiles, int ntiles,
                                   const void *src, void *dst, const int *tile,
                                   int grid, hipStream_t st);
    static bool node_batch(const StepKey &k, const int *tile, int grid,
                           NodeLaunch *node);
};

#ifdef SCMC_FUSED_DEFINE
template <class ST, int ORDER>
bool FusedOps<ST, ORDER>::supported(const StepKey &k, const int *tile) {
    return dispatch(k, tile, [](auto, auto, auto, auto) {});
}

template <class ST, int ORDER>
hipError_t FusedOps<ST, ORDER>::launch(const StepKey &k, const Member &m,
                                       const void *src, void *dst,
                                       const int *tile, hipStream_t st) {
    using T = typename ST::T;
    hipError_t err = hipErrorInvalidValue;
    dispatch(k, tile, [&](auto Pc, auto Rc, auto TXc, auto TYc) {
        constexpr int P = decltype(Pc)::value, RP = decltype(Rc)::value;
        constexpr int TXv = decltype(TXc)::value, TYv = decltype(TYc)::value;
        hipLaunchKernelGGL((k_fused<TXv, TYv, ORDER, ST, P, RP>),
                           dim3(fused_blocks(m, tile)), dim3(TXv, TYv), 0, st, m,
                           (const T *)src, (T *)dst, tile[2]);
        err = hipGetLastError();
    });
    return err;
}

template <class ST, int ORDER>
bool FusedOps<ST, ORDER>::node(const StepKey &k, const int *tile,
                               NodeLaunch *node, const Member &m) {
    return dispatch(k, tile, [&](auto Pc, auto Rc, auto TXc, auto TYc) {
        constexpr int P = decltype(Pc)::value, RP = decltype(Rc)::value;
        constexpr int TXv = decltype(TXc)::value, TYv = decltype(TYc)::value;
        node->func = (void *)&k_fused<TXv, TYv, ORDER, ST, P, RP>;
        node->grid = dim3(fused_blocks(m, tile));
        node->block = dim3(TXv, TYv);
        node->shmem = 0;
    });
}

template <class ST, int ORDER>
hipError_t FusedOps<ST, ORDER>::launch_batch(const StepKey &k,
                                             const Member *d_members,
                                             const Tile *d_tiles, int ntiles,
                                             const void *src, void *dst,
                                             const int *tile, int grid,
                                             hipStream_t st) {
    using T = typename ST::T;
    hipError_t err = hipErrorInvalidValue;
    dispatch(k, tile, [&](auto Pc, auto Rc, auto TXc, auto TYc) {
        constexpr int P = decltype(Pc)::value, RP = decltype(Rc)::value;
        constexpr int TXv = decltype(TXc)::value, TYv = decltype(TYc)::value;
        const void *f = (const void *)&kb_fused<TXv, TYv, ORDER, ST, P, RP>;
        hipLaunchKernelGGL((kb_fused<TXv, TYv, ORDER, ST, P, RP>),
                           dim3(std::min(grid, resident_blocks(f, TXv * TYv))),
                           dim3(TXv, TYv), 0, st, d_members, d_tiles, ntiles,
                           (const T *)src, (T *)dst, tile[2]);
        err = hipGetLastError();
    });
    return err;
}

template <class ST, int ORDER>
bool FusedOps<ST, ORDER>::node_batch(const StepKey &k, const int *tile,
                                     int grid, NodeLaunch *node) {
    return dispatch(k, tile, [&](auto Pc, auto Rc, auto TXc, auto TYc) {
        constexpr int P = decltype(Pc)::value, RP = decltype(Rc)::value;
        constexpr int TXv = decltype(TXc)::value, TYv = decltype(TYc)::value;
        node->func = (void *)&kb_fused<TXv, TYv, ORDER, ST, P, RP>;
        node->grid = dim3(std::min(grid, resident_blocks(node->func, TXv * TYv)));
        node->block = dim3(TXv, TYv);
        node->shmem = 0;
    });
}
#endif

}  // namespace scmc
