// fused_kernels.hip -- one kernel per time step: stream + density + Shan-Chen
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

template <int TX, int TY, int ORDER, class ST, int PSI, int S>
__device__ __forceinline__ void fused_plane(
    const Member &m, const typename ST::T *__restrict__ src,
    typename ST::T *__restrict__ dst, float2 (*lds)[TY + 2 * FusedGeom<ORDER>::HR]
                                                   [TX + 2 * FusedGeom<ORDER>::HR],
    typename ST::R (&ring)[FusedGeom<ORDER>::NRING][2][19], int k, int x0,
    int y0, int z0, int wx, int wy, int tx, int ty, bool active) {
    using G = FusedGeom<ORDER>;
    using L = Lattice<3>;
    using R = typename ST::R;
    constexpr int HR = G::HR, ZR = G::ZR, BX = TX + 2 * HR;
    constexpr int NT = TX * TY;
    const int tid = ty * TX + tx;
    const int zl = wrap1(z0 - ZR + k, m.nz);
    auto &plane = lds[k % G::NSLOT];

    // ---- phase 1: concentrations of the lead plane over tile + halo
    if (active) {
        R(&f)[2][19] = ring[S];
        pull_site<3, ST>(m, src, x0 + tx, y0 + ty, zl, f);
        R nA, nB;
        site_density<3, R>(f, nA, nB);
        plane[ty + HR][tx + HR] = make_float2((float)nA, (float)nB);
    }
    {
        const int bw = wx + 2 * HR;
        const int ntop = HR * bw, nmid = wy * 2 * HR;
        const int nhalo = 2 * ntop + nmid;
        for (int h = tid; h < nhalo; h += NT) {
            int lx, ly;
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
            const int gx = wrap1(x0 - HR + lx, m.nx);
            const int gy = wrap1(y0 - HR + ly, m.ny);
            R f[2][19];
            pull_site<3, ST>(m, src, gx, gy, zl, f);
            R nA, nB;
            site_density<3, R>(f, nA, nB);
            plane[ly][lx] = make_float2((float)nA, (float)nB);
        }
    }
    __syncthreads();

    // ---- phase 2: collide plane zc = zl - ZR
    if (k >= 2 * ZR && active) {
        using Sten = Stencil<3, ORDER>;
        const int zc = wrap1(z0 + k - 2 * ZR, m.nz);
        R(&f)[2][19] = ring[(S + 1) % G::NRING];
        const float2 own = lds[(k - ZR) % G::NSLOT][ty + HR][tx + HR];
        const R nA = own.x, nB = own.y;
        R cA[3] = {0, 0, 0}, cB[3] = {0, 0, 0}, sA[3] = {0, 0, 0},
          sB[3] = {0, 0, 0};
        const bool selfA = m.self_on & 1, selfB = m.self_on & 2;
#pragma unroll
        for (int a = 0; a < Sten::NE; ++a) {
            constexpr auto T = Sten::T;
            const int ex = T.e[a][0], ey = T.e[a][1], ez = T.e[a][2];
            const float2 d = lds[(k - ZR + ez) % G::NSLOT][ty + HR + ey][tx + HR + ex];
            const R nAt = d.x, nBt = d.y;
            const R W = (R)T.W[a];
            const int e3[3] = {ex, ey, ez};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (e3[c] == 0) continue;
                const R We = W * (R)e3[c];
                cA[c] += We * nBt;
                cB[c] += We * nAt;
            }
            if (selfA || selfB) {
                const R pA = psi_of<R, PSI>(nAt), pB = psi_of<R, PSI>(nBt);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (e3[c] == 0) continue;
                    const R We = W * (R)e3[c];
                    sA[c] += We * pA;
                    sB[c] += We * pB;
                }
            }
        }
        const R gAB = (R)m.g[0][1], gBA = (R)m.g[1][0];
        const R gAA = (R)m.g[0][0], gBB = (R)m.g[1][1];
        const R pA = selfA ? psi_of<R, PSI>(nA) : R(0);
        const R pB = selfB ? psi_of<R, PSI>(nB) : R(0);
        R FA[3], FB[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            FA[c] = -gAB * nA * cA[c] - gAA * pA * sA[c];
            FB[c] = -gBA * nB * cB[c] - gBB * pB * sB[c];
        }
        const long s = ((long)zc * m.ny + (y0 + ty)) * m.nx + (x0 + tx);
        site_collide_store<3, ST>(m, f, nA, nB, FA, FB, dst, s);
    }
}

// March the chunk [z0, z0 + zc_len) of the column tile at (x0, y0).
template <int TX, int TY, int ORDER, class ST, int PSI>
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
    R ring[G::NRING][2][19];
    const int kend = zc_len + 2 * G::ZR;
    for (int k = 0; k < kend; k += G::NRING) {
        fused_plane<TX, TY, ORDER, ST, PSI, 0>(m, src, dst, lds, ring, k, x0, y0,
                                               z0, wx, wy, tx, ty, active);
        if (k + 1 < kend)
            fused_plane<TX, TY, ORDER, ST, PSI, 1>(m, src, dst, lds, ring, k + 1,
                                                   x0, y0, z0, wx, wy, tx, ty,
                                                   active);
        if constexpr (G::NRING == 3) {
            if (k + 2 < kend)
                fused_plane<TX, TY, ORDER, ST, PSI, 2>(m, src, dst, lds, ring,
                                                       k + 2, x0, y0, z0, wx, wy,
                                                       tx, ty, active);
        }
    }
}

template <int TX, int TY, int ORDER, class ST, int PSI>
__global__ void __launch_bounds__(TX *TY)
    k_fused(Member m, const typename ST::T *__restrict__ src,
            typename ST::T *__restrict__ dst, int zc_len) {
    const int ntx = (m.nx + TX - 1) / TX, nty = (m.ny + TY - 1) / TY;
    const int nb = gridDim.x;
    const int t = xcd_remap(blockIdx.x, nb);
    const int bx = t % ntx, by = (t / ntx) % nty, bz = t / (ntx * nty);
    const int z0 = bz * zc_len;
    const int len = min(zc_len, m.nz - z0);
    fused_tile<TX, TY, ORDER, ST, PSI>(m, src, dst, bx * TX, by * TY, z0, len);
}

template <int TX, int TY, int ORDER, class ST, int PSI>
__global__ void __launch_bounds__(TX *TY)
    kb_fused(const Member *__restrict__ members, const Tile *__restrict__ tiles,
             int ntiles, const typename ST::T *__restrict__ src,
             typename ST::T *__restrict__ dst, int zc_len) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Member m = members[tl.member];
        const int len = min(zc_len, m.nz - tl.z0);
        fused_tile<TX, TY, ORDER, ST, PSI>(m, src, dst, tl.x0, tl.y0, tl.z0, len);
        __syncthreads();  // the next tile reuses the LDS ring
    }
}

// ---------------------------------------------------------------- dispatch
// compiled tiles (TX, TY); the z-chunk is a runtime argument
#define SCMC_FUSED_TILES(X) X(64, 4) X(64, 2) X(32, 8) X(32, 4) X(64, 8)

template <class F> static bool fused_dispatch(const StepKey &k, const int *tile, F &&fn) {
    if (k.dim != 3 || (k.order != 4 && k.order != 6) || k.storage == ST_F64)
        return false;
    if (tile[2] < 1) return false;
    bool ok = false;
    auto with_st = [&](auto stv) {
        auto with_o = [&](auto Oc) {
            auto with_p = [&](auto Pc) {
#define SCMC_TRY(TXv, TYv)                                                   \
    if (tile[0] == TXv && tile[1] == TYv) {                                  \
        fn(stv, Oc, Pc, std::integral_constant<int, TXv>{},                  \
           std::integral_constant<int, TYv>{});                              \
        ok = true;                                                           \
        return;                                                              \
    }
                SCMC_FUSED_TILES(SCMC_TRY)
#undef SCMC_TRY
            };
            if (k.psi == 0) with_p(std::integral_constant<int, 0>{});
            else with_p(std::integral_constant<int, 1>{});
        };
        if (k.order == 4) with_o(std::integral_constant<int, 4>{});
        else with_o(std::integral_constant<int, 6>{});
    };
    switch (k.storage) {
        case ST_F32: with_st(StoreF32{}); break;
        case ST_F16: with_st(StoreF16{}); break;
        case ST_BF16: with_st(StoreBF16{}); break;
    }
    return ok;
}

bool fused_supported(const StepKey &k, const int *tile) {
    return fused_dispatch(k, tile, [](auto, auto, auto, auto, auto) {});
}

static int fused_blocks(const Member &m, const int *tile) {
    const int ntx = (m.nx + tile[0] - 1) / tile[0];
    const int nty = (m.ny + tile[1] - 1) / tile[1];
    const int ntz = (m.nz + tile[2] - 1) / tile[2];
    return ntx * nty * ntz;
}

hipError_t launch_fused(const StepKey &k, const Member &m, const void *src,
                        void *dst, const int *tile, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    fused_dispatch(k, tile, [&](auto stv, auto Oc, auto Pc, auto TXc, auto TYc) {
        using ST = decltype(stv);
        using T = typename ST::T;
        constexpr int O = decltype(Oc)::value, P = decltype(Pc)::value;
        constexpr int TXv = decltype(TXc)::value, TYv = decltype(TYc)::value;
        hipLaunchKernelGGL((k_fused<TXv, TYv, O, ST, P>), dim3(fused_blocks(m, tile)),
                           dim3(TXv, TYv), 0, st, m, (const T *)src, (T *)dst,
                           tile[2]);
        err = hipGetLastError();
    });
    return err;
}

bool node_fused(const StepKey &k, const int *tile, NodeLaunch *node,
                const Member &m) {
    return fused_dispatch(k, tile, [&](auto stv, auto Oc, auto Pc, auto TXc, auto TYc) {
        using ST = decltype(stv);
        constexpr int O = decltype(Oc)::value, P = decltype(Pc)::value;
        constexpr int TXv = decltype(TXc)::value, TYv = decltype(TYc)::value;
        node->func = (void *)&k_fused<TXv, TYv, O, ST, P>;
        node->grid = dim3(fused_blocks(m, tile));
        node->block = dim3(TXv, TYv);
        node->shmem = 0;
    });
}

hipError_t launch_batch_fused(const StepKey &k, const Member *d_members,
                              const Tile *d_tiles, int ntiles, const void *src,
                              void *dst, const int *tile, int grid,
                              hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    fused_dispatch(k, tile, [&](auto stv, auto Oc, auto Pc, auto TXc, auto TYc) {
        using ST = decltype(stv);
        using T = typename ST::T;
        constexpr int O = decltype(Oc)::value, P = decltype(Pc)::value;
        constexpr int TXv = decltype(TXc)::value, TYv = decltype(TYc)::value;
        hipLaunchKernelGGL((kb_fused<TXv, TYv, O, ST, P>), dim3(grid),
                           dim3(TXv, TYv), 0, st, d_members, d_tiles, ntiles,
                           (const T *)src, (T *)dst, tile[2]);
        err = hipGetLastError();
    });
    return err;
}

bool node_batch_fused(const StepKey &k, const int *tile, int grid,
                      NodeLaunch *node) {
    return fused_dispatch(k, tile, [&](auto stv, auto Oc, auto Pc, auto TXc, auto TYc) {
        using ST = decltype(stv);
        constexpr int O = decltype(Oc)::value, P = decltype(Pc)::value;
        constexpr int TXv = decltype(TXc)::value, TYv = decltype(TYc)::value;
        node->func = (void *)&kb_fused<TXv, TYv, O, ST, P>;
        node->grid = dim3(grid);
        node->block = dim3(TXv, TYv);
        node->shmem = 0;
    });
}

}  // namespace scmc
