// step_kernels.hip -- the two-pass design of the Shan-Chen time step and its
// batched (persistent, tile-list) form.
//
// Pass 1 (k_density): every site pulls its 2Q populations and stores n_A, n_B
// in a density field [J][z][y][x].  Pass 2 (k_collide): every site pulls again,
// reads the stencil densities of eq. sc_force from the field (they stay in L2
// and the Infinity Cache), forms the force, the common velocity and the BGK +
// Guo update, and stores f* into the other population buffer.  A wave covers
// 64 consecutive x, so every pull of every direction is one coalesced row
// segment.  This design handles every lattice, stencil and storage format and
// is the reference path of the fused kernels.
#include "site_ops.h"

namespace scmc {

constexpr int TP_BX = 64, TP_BY = 4;  // two-pass block: 64 x 4 sites

template <int D, class ST>
__global__ void __launch_bounds__(256)
    k_density(Member m, const typename ST::T *__restrict__ src,
              typename ST::R *__restrict__ dens) {
    using R = typename ST::R;
    const int x = blockIdx.x * TP_BX + threadIdx.x;
    const int y = blockIdx.y * TP_BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= m.nx || y >= m.ny) return;
    R f[2][Lattice<D>::Q];
    pull_site<D, ST>(m, src, x, y, z, f);
    R nA, nB;
    site_density<D, R>(f, nA, nB);
    const long s = ((long)z * m.ny + y) * m.nx + x;
    dens[m.dens_off + s] = nA;
    dens[m.dens_off + m.N + s] = nB;
}

template <int D, int ORDER, class ST, int PSI>
__global__ void __launch_bounds__(256)
    k_collide(Member m, const typename ST::T *__restrict__ src,
              typename ST::T *__restrict__ dst,
              const typename ST::R *__restrict__ dens) {
    using R = typename ST::R;
    const int x = blockIdx.x * TP_BX + threadIdx.x;
    const int y = blockIdx.y * TP_BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= m.nx || y >= m.ny) return;
    R f[2][Lattice<D>::Q];
    pull_site<D, ST>(m, src, x, y, z, f);
    R nA, nB;
    site_density<D, R>(f, nA, nB);
    R FA[3], FB[3];
    const R *dA = dens + m.dens_off;
    site_force<D, ORDER, PSI, R>(m, dA, dA + m.N, x, y, z, nA, nB, FA, FB);
    const long s = ((long)z * m.ny + y) * m.nx + x;
    site_collide_store<D, ST>(m, f, nA, nB, FA, FB, dst, s);
}

// ---- batched forms: a persistent grid walks a tile list; a tile is a
// 64 x 4 x 1 block of sites of one member.
template <int D, class ST>
__global__ void __launch_bounds__(256)
    kb_density(const Member *__restrict__ members,
               const Tile *__restrict__ tiles, int ntiles,
               const typename ST::T *__restrict__ src,
               typename ST::R *__restrict__ dens) {
    using R = typename ST::R;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Member m = members[tl.member];
        const int x = tl.x0 + threadIdx.x, y = tl.y0 + threadIdx.y, z = tl.z0;
        if (x < m.nx && y < m.ny) {
            R f[2][Lattice<D>::Q];
            pull_site<D, ST>(m, src, x, y, z, f);
            R nA, nB;
            site_density<D, R>(f, nA, nB);
            const long s = ((long)z * m.ny + y) * m.nx + x;
            dens[m.dens_off + s] = nA;
            dens[m.dens_off + m.N + s] = nB;
        }
    }
}

template <int D, int ORDER, class ST, int PSI>
__global__ void __launch_bounds__(256)
    kb_collide(const Member *__restrict__ members,
               const Tile *__restrict__ tiles, int ntiles,
               const typename ST::T *__restrict__ src,
               typename ST::T *__restrict__ dst,
               const typename ST::R *__restrict__ dens) {
    using R = typename ST::R;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Member m = members[tl.member];
        const int x = tl.x0 + threadIdx.x, y = tl.y0 + threadIdx.y, z = tl.z0;
        if (x < m.nx && y < m.ny) {
            R f[2][Lattice<D>::Q];
            pull_site<D, ST>(m, src, x, y, z, f);
            R nA, nB;
            site_density<D, R>(f, nA, nB);
            R FA[3], FB[3];
            const R *dA = dens + m.dens_off;
            site_force<D, ORDER, PSI, R>(m, dA, dA + m.N, x, y, z, nA, nB, FA,
                                         FB);
            const long s = ((long)z * m.ny + y) * m.nx + x;
            site_collide_store<D, ST>(m, f, nA, nB, FA, FB, dst, s);
        }
    }
}

// ---------------------------------------------------------------- dispatch
template <class F> static bool dispatch_storage(int storage, F &&fn) {
    switch (storage) {
        case ST_F64: fn(StoreF64{}); return true;
        case ST_F32: fn(StoreF32{}); return true;
        case ST_F16: fn(StoreF16{}); return true;
        case ST_BF16: fn(StoreBF16{}); return true;
    }
    return false;
}

template <class ST, class F>
static bool dispatch_shape(const StepKey &k, F &&fn) {
    // fn(integral_constant D, ORDER, PSI)
    auto go = [&](auto Dc, auto Oc) {
        if (k.psi == 0)
            fn(Dc, Oc, std::integral_constant<int, 0>{});
        else
            fn(Dc, Oc, std::integral_constant<int, 1>{});
    };
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using O4 = std::integral_constant<int, 4>;
    using O6 = std::integral_constant<int, 6>;
    using O8 = std::integral_constant<int, 8>;
    if (k.dim == 2 && k.order == 4) { go(I2{}, O4{}); return true; }
    if (k.dim == 2 && k.order == 6) { go(I2{}, O6{}); return true; }
    if (k.dim == 2 && k.order == 8) { go(I2{}, O8{}); return true; }
    if (k.dim == 3 && k.order == 4) { go(I3{}, O4{}); return true; }
    if (k.dim == 3 && k.order == 6) { go(I3{}, O6{}); return true; }
    return false;
}

static dim3 tp_grid(const Member &m) {
    return dim3((m.nx + TP_BX - 1) / TP_BX, (m.ny + TP_BY - 1) / TP_BY, m.nz);
}

hipError_t launch_two_pass(const StepKey &k, const Member &m, const void *src,
                           void *dst, void *dens, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    dispatch_storage(k.storage, [&](auto stv) {
        using ST = decltype(stv);
        using T = typename ST::T;
        using R = typename ST::R;
        dispatch_shape<ST>(k, [&](auto Dc, auto Oc, auto Pc) {
            constexpr int D = decltype(Dc)::value;
            constexpr int O = decltype(Oc)::value;
            constexpr int P = decltype(Pc)::value;
            const dim3 g = tp_grid(m), b(TP_BX, TP_BY, 1);
            hipLaunchKernelGGL((k_density<D, ST>), g, b, 0, st, m,
                               (const T *)src, (R *)dens);
            hipLaunchKernelGGL((k_collide<D, O, ST, P>), g, b, 0, st, m,
                               (const T *)src, (T *)dst, (const R *)dens);
            err = hipGetLastError();
        });
    });
    return err;
}

bool node_two_pass(const StepKey &k, NodeLaunch *dn, NodeLaunch *sn,
                   const Member &m) {
    bool ok = false;
    dispatch_storage(k.storage, [&](auto stv) {
        using ST = decltype(stv);
        dispatch_shape<ST>(k, [&](auto Dc, auto Oc, auto Pc) {
            constexpr int D = decltype(Dc)::value;
            constexpr int O = decltype(Oc)::value;
            constexpr int P = decltype(Pc)::value;
            dn->func = (void *)&k_density<D, ST>;
            sn->func = (void *)&k_collide<D, O, ST, P>;
            dn->grid = sn->grid = tp_grid(m);
            dn->block = sn->block = dim3(TP_BX, TP_BY, 1);
            dn->shmem = sn->shmem = 0;
            ok = true;
        });
    });
    return ok;
}

hipError_t launch_batch_two_pass(const StepKey &k, const Member *d_members,
                                 const Tile *d_tiles, int ntiles,
                                 const void *src, void *dst, void *dens,
                                 int grid, hipStream_t st) {
    hipError_t err = hipErrorInvalidValue;
    dispatch_storage(k.storage, [&](auto stv) {
        using ST = decltype(stv);
        using T = typename ST::T;
        using R = typename ST::R;
        dispatch_shape<ST>(k, [&](auto Dc, auto Oc, auto Pc) {
            constexpr int D = decltype(Dc)::value;
            constexpr int O = decltype(Oc)::value;
            constexpr int P = decltype(Pc)::value;
            const dim3 b(TP_BX, TP_BY, 1);
            hipLaunchKernelGGL((kb_density<D, ST>), dim3(grid), b, 0, st,
                               d_members, d_tiles, ntiles, (const T *)src,
                               (R *)dens);
            hipLaunchKernelGGL((kb_collide<D, O, ST, P>), dim3(grid), b, 0,
                               st, d_members, d_tiles, ntiles, (const T *)src,
                               (T *)dst, (const R *)dens);
            err = hipGetLastError();
        });
    });
    return err;
}

bool node_batch_two_pass(const StepKey &k, int grid, NodeLaunch *dn,
                         NodeLaunch *sn) {
    bool ok = false;
    dispatch_storage(k.storage, [&](auto stv) {
        using ST = decltype(stv);
        dispatch_shape<ST>(k, [&](auto Dc, auto Oc, auto Pc) {
            constexpr int D = decltype(Dc)::value;
            constexpr int O = decltype(Oc)::value;
            constexpr int P = decltype(Pc)::value;
            dn->func = (void *)&kb_density<D, ST>;
            sn->func = (void *)&kb_collide<D, O, ST, P>;
            dn->grid = sn->grid = dim3(grid);
            dn->block = sn->block = dim3(TP_BX, TP_BY, 1);
            dn->shmem = sn->shmem = 0;
            ok = true;
        });
    });
    return ok;
}

}  // namespace scmc
