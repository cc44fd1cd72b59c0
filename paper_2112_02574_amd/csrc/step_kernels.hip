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
//
// At tau = 1 the second pass need not pull again: the collision then depends
// on the populations only through n_J and the total momentum j.  Pass 1
// (k_moments) stores (n_A, n_B) pairs, the j planes and the packed FP64
// remainders of n_A, n_B; pass 2 (k_collide_mom) reads the node's moments and
// the stencil's concentration pairs and stores f*.  Per site it moves 2Q reads
// + 2Q writes of populations plus 24 B of moments each way (FP32), instead of
// 4Q reads + 2Q writes.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "fused_impl.h"  // FusedGeom, lds_force, halo_pos, xcd_remap
#include "site_ops.h"

namespace scmc {

constexpr int TP_BX = 64, TP_BY = 4;  // two-pass block: 64 x 4 sites

// Batched two-pass tiles are runs of TP_BX * TP_BY consecutive sites of one
// member (x fastest, rows wrap), so lattices whose rows are not a multiple of
// 64 leave no lanes idle.  Site of this thread in tile tl, false past the end.
__device__ __forceinline__ bool tile_site(const Member &m, const Tile &tl, int &x, int &y,
                                          int &z) {
    const int s = tl.x0 + threadIdx.y * TP_BX + threadIdx.x;
    if (s >= m.N) return false;
    const int nxy = m.nx * m.ny;
    z = s / nxy;
    const int r = s - z * nxy;
    y = r / m.nx;
    x = r - y * m.nx;
    return true;
}

// The two-pass designs over one lattice number their sites linearly: block b
// takes the BLK consecutive sites from plane zoff on, so no lane idles
// whatever the row length.  False past plane zoff + znum.  Blocks of 256
// sites suit lattices whose moment field stays cached; the z-slab schedule
// of larger lattices runs blocks of 512 (SLAB_BLOCK).
constexpr int LIN_BLOCK = 256, SLAB_BLOCK = 512;
template <int BLK>
__device__ __forceinline__ bool linear_site_at(const Member &m, int block, int &x, int &y,
                                               int &z) {
    const int nxy = m.nx * m.ny;
    const int s = m.zoff * nxy + block * BLK + threadIdx.x;
    if (s >= (m.zoff + m.znum) * nxy) return false;
    z = s / nxy;
    const int r = s - z * nxy;
    y = r / m.nx;
    x = r - y * m.nx;
    return true;
}
template <int BLK>
__device__ __forceinline__ bool linear_site(const Member &m, int &x, int &y, int &z) {
    return linear_site_at<BLK>(m, blockIdx.x, x, y, z);
}

template <int D, class ST>
__global__ void __launch_bounds__(256)
    k_density(Member m, const typename ST::T *__restrict__ src,
              typename ST::R *__restrict__ dens) {
    using R = typename ST::R;
    advance_step_counter(m, blockIdx.x == 0);
    int x, y, z;
    if (!linear_site<LIN_BLOCK>(m, x, y, z)) return;
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
    int x, y, z;
    if (!linear_site<LIN_BLOCK>(m, x, y, z)) return;
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

// ---- tau = 1: moment two-pass
template <class R> using Pair = typename std::conditional<std::is_same<R, float>::value,
                                                          float2, double2>::type;

// The FP64 remainders of n_A, n_B (at most half an ulp of the stored value)
// travel as two halves of one 32-bit word, in units of that ulp: 11 bits of
// the remainder keep the rest population's mass closure exact to 2^-12 ulp,
// far inside its own rounding.  FP64 compute has no remainder.
template <class R>
__device__ __forceinline__ unsigned pack_rem(const R (&mm)[NMOM]) {
    if constexpr (std::is_same<R, double>::value) {
        return 0u;
    } else {
        unsigned out = 0;
#pragma unroll
        for (int J = 0; J < 2; ++J) {
            int e;
            frexpf(mm[J], &e);
            const float q = ldexpf(mm[5 + J], 24 - e);  // remainder / ulp(n_J)
            out |= (unsigned)__half_as_ushort(__float2half_rn(q)) << (16 * J);
        }
        return out;
    }
}

template <class R>
__device__ __forceinline__ void unpack_rem(unsigned w, R (&mm)[NMOM]) {
    if constexpr (std::is_same<R, double>::value) {
        mm[5] = mm[6] = 0;
    } else {
#pragma unroll
        for (int J = 0; J < 2; ++J) {
            int e;
            frexpf(mm[J], &e);
            const float q = __half2float(__ushort_as_half((unsigned short)(w >> (16 * J))));
            mm[5 + J] = ldexpf(q, e - 24);
        }
    }
}

// moment field of a member: (n_A, n_B) pairs [z][y][x], then the planes j_x,
// j_y (, j_z), then the packed remainders of n_A and n_B (plane 5)
template <int D, class ST>
__device__ __forceinline__ void moments_site(const Member &m,
                                             const typename ST::T *__restrict__ src,
                                             typename ST::R *__restrict__ mom, int x,
                                             int y, int z) {
    using R = typename ST::R;
    R f[2][Lattice<D>::Q], mm[NMOM];
    pull_site<D, ST, true>(m, src, x, y, z, f);
    site_moments<D, R>(f, mm);
    const long s = ((long)z * m.ny + y) * m.nx + x;
    R *base = mom + m.dens_off;
    Pair<R> pr;
    pr.x = mm[0];
    pr.y = mm[1];
    reinterpret_cast<Pair<R> *>(base + (long)m.pair_slot * m.N)[s] = pr;
#pragma unroll
    for (int c = 0; c < D; ++c) base[(2 + c) * (long)m.N + s] = mm[2 + c];
    reinterpret_cast<unsigned *>(base + 5 * (long)m.N)[s] = pack_rem<R>(mm);
}

template <int D, int ORDER, class ST, int PSI>
__device__ __forceinline__ void collide_mom_site(const Member &m,
                                                 typename ST::T *__restrict__ dst,
                                                 const typename ST::R *__restrict__ mom,
                                                 int x, int y, int z) {
    using R = typename ST::R;
    const R *base = mom + m.dens_off;
    const Pair<R> *pairs = reinterpret_cast<const Pair<R> *>(base + (long)m.pair_slot * m.N);
    const long s = ((long)z * m.ny + y) * m.nx + x;
    const Pair<R> own = pairs[s];
    R mm[NMOM] = {own.x, own.y, 0, 0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < D; ++c) mm[2 + c] = base[(2 + c) * (long)m.N + s];
    unpack_rem<R>(reinterpret_cast<const unsigned *>(base + 5 * (long)m.N)[s], mm);
    R FA[3], FB[3];
    site_force_fn<D, ORDER, PSI, R>(m, x, y, z, own.x, own.y, FA, FB,
                                    [&](int t, R &a, R &b) {
                                        const Pair<R> q = pairs[t];
                                        a = q.x;
                                        b = q.y;
                                    });
    typename ST::T *out = dst + m.pop_off;
    if (m.sr) {
        SiteRng rng(m.seed, *m.step_ctr, (unsigned)(m.pop_off + s));
        collide_tau1<D, R>(m, mm, FA, FB, [&](int J, int i, R v, R ref) {
            __builtin_nontemporal_store(ST::to_raw_sr(v, ref, rng.next()),
                                        out + (long)(J * Lattice<D>::Q + i) * m.N + s);
        });
        return;
    }
    collide_tau1<D, R>(m, mm, FA, FB, [&](int J, int i, R v, R ref) {
        ST::store(out, (long)(J * Lattice<D>::Q + i) * m.N + s, v, ref);
    });
}

// D3Q19 forms with 32-bit buffer offsets (each component's Q planes below
// 2 GiB): plane offsets go in the scalar offset, lanes carry 32-bit offsets.
// The (n_A, n_B) pairs sit at slot m.pair_slot of the moment field (0 but
// for node storage, whose pass 1 writes the pairs into the reference field
// of the buffer that pass 2 fills).  NT: the pull's PullPolicy.
template <class ST, bool NODE = false, int NT = PULL_NT_ALIGNED>
__device__ __forceinline__ void moments_site_buf(const Member &m, const PopBuf<ST> &sb,
                                                 typename ST::R *__restrict__ mom, int x,
                                                 int y, int z) {
    using R = typename ST::R;
    R f[2][19], mm[NMOM];
    pull_site_buf<ST, NT, NODE>(m, sb, x, y, z, f);
    site_moments<3, R>(f, mm);
    const int s = (z * m.ny + y) * m.nx + x;
    R *base = mom + m.dens_off;
    reinterpret_cast<Pair<R> *>(base + (long)m.pair_slot * m.N)[s] = Pair<R>{mm[0], mm[1]};
#pragma unroll
    for (int c = 0; c < 3; ++c) base[(2 + c) * (long)m.N + s] = mm[2 + c];
    reinterpret_cast<unsigned *>(base + 5 * (long)m.N)[s] = pack_rem<R>(mm);
}

// SR: stores rounded stochastically (16-bit offsets, every member of the
// launch); without it the generator is compiled out.
template <int ORDER, class ST, int PSI, bool NODE = false, bool SR = false>
__device__ __forceinline__ void collide_mom_site_buf(const Member &m, const PopBuf<ST> &db,
                                                     const typename ST::R *__restrict__ mom,
                                                     int x, int y, int z) {
    using R = typename ST::R;
    using T = typename ST::T;
    const R *base = mom + m.dens_off;
    const Pair<R> *pairs = reinterpret_cast<const Pair<R> *>(base + (long)m.pair_slot * m.N);
    const int s = (z * m.ny + y) * m.nx + x;
    const Pair<R> own = pairs[s];
    R mm[NMOM] = {own.x, own.y, 0, 0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) mm[2 + c] = base[(2 + c) * (long)m.N + s];
    unpack_rem<R>(reinterpret_cast<const unsigned *>(base + 5 * (long)m.N)[s], mm);
    R FA[3], FB[3];
    // stencil pairs through a buffer descriptor with 32-bit byte offsets
    // (8 N < 2^31 in these forms): no 64-bit address arithmetic per neighbour
    static_assert(sizeof(Pair<R>) == 8, "FP32 pairs");
    const __amdgpu_buffer_rsrc_t pr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)pairs, (short)0, m.N * 8, BUF_DATA_FORMAT_32);
    site_force_fn<3, ORDER, PSI, R, 8>(
        m, x, y, z, own.x, own.y, FA, FB, [&](int t, R &a, R &b) {
            const auto q = __builtin_amdgcn_raw_buffer_load_b64(pr, t, 0, 0);
            const unsigned qa = q[0], qb = q[1];  // scalars before the cast
            a = __uint_as_float(qa);
            b = __uint_as_float(qb);
        });
    const int voff = s * (int)sizeof(T);
    if constexpr (NODE) {
        // the densities of the nodes the populations stream to (x + e_i)
        using L = Lattice<3>;
        int xo[3], yo[3], zo[3];
#pragma unroll
        for (int d = -1; d <= 1; ++d) {
            xo[d + 1] = wrap1(x + d, m.nx) * 8;
            yo[d + 1] = wrap1(y + d, m.ny) * (m.nx * 8);
            zo[d + 1] = wrap1(z + d, m.nz) * (m.nx * m.ny * 8);
        }
        float2 nb[L::Q];
        nb[0] = float2{own.x, own.y};
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const auto q = __builtin_amdgcn_raw_buffer_load_b64(
                pr, zo[1 + L::CZ[i]] + yo[1 + L::CY[i]] + xo[1 + L::CX[i]], 0, 0);
            const unsigned qa = q[0], qb = q[1];
            nb[i] = float2{__uint_as_float(qa), __uint_as_float(qb)};
        }
        float2 r;
        collide_tau1_node<3, ST>(
            mm, FA, FB, nb,
            [&](int J, int i, T h) { RawBuf<T>::store_nt(h, db.r[J], voff, i * db.plane_bytes); },
            r.x, r.y);
        m.rest[s] = r;
        return;
    }
    if constexpr (SR) {
        SiteRng rng(m.seed, *m.step_ctr, (unsigned)(m.pop_off + s));
        collide_tau1<3, R>(m, mm, FA, FB, [&](int J, int i, R v, R ref) {
            RawBuf<T>::store_nt(ST::to_raw_sr(v, ref, rng.next()), db.r[J], voff,
                                i * db.plane_bytes);
        });
        return;
    }
    collide_tau1<3, R>(m, mm, FA, FB, [&](int J, int i, R v, R ref) {
        RawBuf<T>::store_nt(ST::to_raw(v, ref), db.r[J], voff, i * db.plane_bytes);
    });
}

// Second pass with the stencil's concentration pairs staged in LDS: a
// workgroup marches a TX x TY column through a z-chunk of ZC planes, keeping
// a ring of 2 ZR + 2 pair planes (tile + halo, 8 B per node, coalesced), so
// every pair is fetched about once per chunk instead of once per stencil
// neighbour; the node's momentum and remainders are read directly.
template <int TX, int TY, int ZC, int ORDER, class ST, int PSI, bool NODE = false,
          bool SR = false>
__global__ void __launch_bounds__(TX *TY)
    k_collide_mom_lds(Member m, const typename ST::T *__restrict__ src,
                      typename ST::T *__restrict__ dst,
                      const typename ST::R *__restrict__ mom) {
    using R = typename ST::R;
    using T = typename ST::T;
    using G = FusedGeom<ORDER>;
    constexpr int HR = G::HR, ZR = G::ZR, NSLOT = G::NSLOT, NT = TX * TY;
    __shared__ float2 lds[NSLOT][TY + 2 * HR][TX + 2 * HR];
    const int ntx = (m.nx + TX - 1) / TX, nty = (m.ny + TY - 1) / TY;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (t % ntx) * TX, y0 = ((t / ntx) % nty) * TY;
    const int z0 = (t / (ntx * nty)) * ZC;
    const int len = min(ZC, m.nz - z0);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int wx = min(TX, m.nx - x0), wy = min(TY, m.ny - y0);
    const bool active = tx < wx && ty < wy;
    const int nhalo = 2 * HR * (wx + 2 * HR) + wy * 2 * HR;
    const R *base = mom + m.dens_off;
    const float2 *pairs = reinterpret_cast<const float2 *>(base + (long)m.pair_slot * m.N);
    const PopBuf<ST> db = make_popbuf<ST, 19>(dst, m);
    const int nxy = m.nx * m.ny;
    for (int k = 0; k < len + 2 * ZR; ++k) {
        const int zl = wrap1(z0 - ZR + k, m.nz);
        auto &plane = lds[k % NSLOT];
        if (active) plane[ty + HR][tx + HR] = pairs[zl * nxy + (y0 + ty) * m.nx + x0 + tx];
        for (int h = tid; h < nhalo; h += NT) {
            int lx, ly;
            halo_pos<HR>(h, wx, wy, lx, ly);
            plane[ly][lx] = pairs[zl * nxy + wrap1(y0 - HR + ly, m.ny) * m.nx +
                                  wrap1(x0 - HR + lx, m.nx)];
        }
        __syncthreads();
        if (k >= 2 * ZR && active) {
            const int zc = wrap1(z0 + k - 2 * ZR, m.nz);
            const int s = zc * nxy + (y0 + ty) * m.nx + x0 + tx;
            R mm[NMOM], FA[3], FB[3];
            lds_force<TX, TY, ORDER, R, PSI>(m, lds, k, tx, ty, mm[0], mm[1], FA, FB);
#pragma unroll
            for (int c = 0; c < 3; ++c) mm[2 + c] = base[(2 + c) * (long)m.N + s];
            unpack_rem<R>(reinterpret_cast<const unsigned *>(base + 5 * (long)m.N)[s], mm);
            const int voff = s * (int)sizeof(T);
            if constexpr (NODE) {
                // the densities of the nodes the populations stream to
                using L = Lattice<3>;
                float2 nb[L::Q];
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    nb[i] = lds[(k - ZR + L::CZ[i]) % NSLOT][ty + HR + L::CY[i]][tx + HR + L::CX[i]];
                float2 r;
                collide_tau1_node<3, ST>(
                    mm, FA, FB, nb,
                    [&](int J, int i, T h) {
                        RawBuf<T>::store_nt(h, db.r[J], voff, i * db.plane_bytes);
                    },
                    r.x, r.y);
                m.rest[s] = r;
            } else if constexpr (SR) {
                SiteRng rng(m.seed, *m.step_ctr, (unsigned)(m.pop_off + s));
                collide_tau1<3, R>(m, mm, FA, FB, [&](int J, int i, R v, R ref) {
                    RawBuf<T>::store_nt(ST::to_raw_sr(v, ref, rng.next()), db.r[J], voff,
                                        i * db.plane_bytes);
                });
            } else {
                collide_tau1<3, R>(m, mm, FA, FB, [&](int J, int i, R v, R ref) {
                    RawBuf<T>::store_nt(ST::to_raw(v, ref), db.r[J], voff, i * db.plane_bytes);
                });
            }
        }
    }
}

template <class ST, int BLK, bool NODE = false, int NT = PULL_NT_ALIGNED>
__global__ void __launch_bounds__(BLK)
    k_moments_buf(Member m, const typename ST::T *__restrict__ src,
                  typename ST::R *__restrict__ mom) {
    advance_step_counter(m, blockIdx.x == 0);
    const PopBuf<ST> sb = make_popbuf<ST, 19>(src, m);
    int x, y, z;
    if (linear_site<BLK>(m, x, y, z)) moments_site_buf<ST, NODE, NT>(m, sb, mom, x, y, z);
}

template <int ORDER, class ST, int PSI, int BLK, bool NODE = false, bool SR = false>
__global__ void __launch_bounds__(BLK)
    k_collide_mom_buf(Member m, const typename ST::T *__restrict__ src,
                      typename ST::T *__restrict__ dst,
                      const typename ST::R *__restrict__ mom) {
    const PopBuf<ST> db = make_popbuf<ST, 19>(dst, m);
    int x, y, z;
    if (linear_site<BLK>(m, x, y, z))
        collide_mom_site_buf<ORDER, ST, PSI, NODE, SR>(m, db, mom, x, y, z);
}

// Block b of a launch that runs n2 blocks of pass 2 and n1 of pass 1: groups
// of 8 consecutive blocks alternate between the passes while
// both last, so both spread over every XCD (workgroups go round-robin over
// the 8 XCDs) and every CU mixes the two; the rest of the longer pass
// follows.  Sets p2 and the unit's index within its pass.
__device__ __forceinline__ void pair_unit(int b, int n2, int n1, bool &p2, int &i) {
    const int m8 = (min(n1, n2) / 8) * 8;
    if (b < 2 * m8) {
        p2 = ((b >> 3) & 1) == 0;
        i = ((b >> 4) << 3) | (b & 7);
    } else {
        b -= 2 * m8;
        p2 = b < n2 - m8;
        i = m8 + (p2 ? b : b - (n2 - m8));
    }
}

// One launch of the slab schedule that runs pass 2 over the planes of m2 and
// pass 1 over those of m1 (a later slab, whose moments pass 2 does not read,
// from the source buffer, which pass 2 does not write): nb2 and nb1 blocks of
// BLK sites.
template <int ORDER, class ST, int PSI, int BLK, bool NODE = false>
__global__ void __launch_bounds__(BLK)
    k_slab_pair(Member m2, Member m1, int nb2, int nb1, const typename ST::T *__restrict__ src,
                typename ST::T *__restrict__ dst, typename ST::R *__restrict__ mom) {
    bool p2;
    int bi;
    pair_unit(blockIdx.x, nb2, nb1, p2, bi);
    int x, y, z;
    if (p2) {
        const PopBuf<ST> db = make_popbuf<ST, 19>(dst, m2);
        if (linear_site_at<BLK>(m2, bi, x, y, z))
            collide_mom_site_buf<ORDER, ST, PSI, NODE>(m2, db, mom, x, y, z);
    } else {
        const PopBuf<ST> sb = make_popbuf<ST, 19>(src, m1);
        if (linear_site_at<BLK>(m1, bi, x, y, z)) moments_site_buf<ST, NODE>(m1, sb, mom, x, y, z);
    }
}

template <class ST, int NT = PULL_NT_ALIGNED>
__global__ void __launch_bounds__(256)
    kb_moments_buf(const Member *__restrict__ members, const Tile *__restrict__ tiles,
                   int ntiles, const typename ST::T *__restrict__ src,
                   typename ST::R *__restrict__ mom) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Member m = members[tl.member];
        advance_step_counter(m, t == 0);
        const PopBuf<ST> sb = make_popbuf<ST, 19>(src, m);
        int x, y, z;
        if (tile_site(m, tl, x, y, z)) moments_site_buf<ST, false, NT>(m, sb, mom, x, y, z);
    }
}

template <int ORDER, class ST, int PSI, bool SR = false>
__global__ void __launch_bounds__(256)
    kb_collide_mom_buf(const Member *__restrict__ members, const Tile *__restrict__ tiles,
                       int ntiles, const typename ST::T *__restrict__ src,
                       typename ST::T *__restrict__ dst,
                       const typename ST::R *__restrict__ mom) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Member m = members[tl.member];
        const PopBuf<ST> db = make_popbuf<ST, 19>(dst, m);
        int x, y, z;
        if (tile_site(m, tl, x, y, z))
            collide_mom_site_buf<ORDER, ST, PSI, false, SR>(m, db, mom, x, y, z);
    }
}

template <int D, class ST>
__global__ void __launch_bounds__(256)
    k_moments(Member m, const typename ST::T *__restrict__ src,
              typename ST::R *__restrict__ mom) {
    advance_step_counter(m, blockIdx.x == 0);
    int x, y, z;
    if (linear_site<LIN_BLOCK>(m, x, y, z)) moments_site<D, ST>(m, src, mom, x, y, z);
}

template <int D, int ORDER, class ST, int PSI>
__global__ void __launch_bounds__(256)
    k_collide_mom(Member m, const typename ST::T *__restrict__ src,
                  typename ST::T *__restrict__ dst,
                  const typename ST::R *__restrict__ mom) {
    int x, y, z;
    if (linear_site<LIN_BLOCK>(m, x, y, z)) collide_mom_site<D, ORDER, ST, PSI>(m, dst, mom, x, y, z);
}

template <int D, class ST>
__global__ void __launch_bounds__(256)
    kb_moments(const Member *__restrict__ members, const Tile *__restrict__ tiles,
               int ntiles, const typename ST::T *__restrict__ src,
               typename ST::R *__restrict__ mom) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Member m = members[tl.member];
        advance_step_counter(m, t == 0);
        int x, y, z;
        if (tile_site(m, tl, x, y, z)) moments_site<D, ST>(m, src, mom, x, y, z);
    }
}

template <int D, int ORDER, class ST, int PSI>
__global__ void __launch_bounds__(256)
    kb_collide_mom(const Member *__restrict__ members, const Tile *__restrict__ tiles,
                   int ntiles, const typename ST::T *__restrict__ src,
                   typename ST::T *__restrict__ dst,
                   const typename ST::R *__restrict__ mom) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const Member m = members[tl.member];
        int x, y, z;
        if (tile_site(m, tl, x, y, z)) collide_mom_site<D, ORDER, ST, PSI>(m, dst, mom, x, y, z);
    }
}

// ---- batched forms: a persistent grid walks a tile list; a tile is a run of
// 256 consecutive sites of one member (tile_site).
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
        advance_step_counter(m, t == 0);
        int x, y, z;
        if (tile_site(m, tl, x, y, z)) {
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
        int x, y, z;
        if (tile_site(m, tl, x, y, z)) {
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

// the 32-bit buffer forms serve D3Q19 with FP32-compute storage that fits
template <int D, class ST> constexpr bool buf_form() {
    return D == 3 && !std::is_same<ST, StoreF64>::value;
}
// node storage: the buffer forms of the 16-bit formats
template <int D, class ST> constexpr bool node_form() {
    return buf_form<D, ST>() && sizeof(typename ST::T) == 2;
}
// stochastic rounding: the 16-bit offset formats
template <class ST> constexpr bool sr_form() { return sizeof(typename ST::T) == 2; }
// pass 1 with every load non-temporal: FP32 populations, global reference
template <class ST, bool NODE> constexpr bool nt_all_form() {
    return !NODE && std::is_same<ST, StoreF32>::value;
}

// Pass 1 of an unslabbed FP32 moment two-pass loads every population
// non-temporally once the moment fields it writes reach kNtAllMomentBytes.
// Below that they stay cached between the passes either way, and the
// shifted populations' lines, which neighbouring wavefronts share, are worth
// keeping in L2 (measured: 4-7 % slower steps at 128^3-144^3 with every load
// non-temporal, 1-11 % faster ones at 152^3-168^3).
static constexpr size_t kNtAllMomentBytes = (size_t)80 << 20;

bool pass1_nt_all(const StepKey &k, long sites) {
    return k.storage == ST_F32 && k.mom && !k.node && !k.big &&
           (size_t)sites * 24 >= kNtAllMomentBytes;
}

// The LDS-staged collision pass (StepKey::mom == 2) marches 64 x 8 columns
// through z-chunks of 8 planes (measured on 128^3).
constexpr int CL_TX = 64, CL_TY = 8, CL_ZC = 8;

int linear_blocks(const Member &m, int znum, int blk) {
    return (int)(((long)znum * m.nx * m.ny + blk - 1) / blk);
}

// Launch shapes of the moment two-pass: 256 linearly numbered sites per block
// (linear_site), or the LDS-staged pass 2.
static void mom_blocks(const Member &m, bool lds, dim3 *gm, dim3 *bm, dim3 *gc,
                       dim3 *bc) {
    *bm = dim3(LIN_BLOCK, 1, 1);
    *gm = dim3(linear_blocks(m, m.znum, LIN_BLOCK));
    if (lds) {
        const int ntx = (m.nx + CL_TX - 1) / CL_TX, nty = (m.ny + CL_TY - 1) / CL_TY;
        *bc = dim3(CL_TX, CL_TY, 1);
        *gc = dim3(ntx * nty * ((m.nz + CL_ZC - 1) / CL_ZC), 1, 1);
    } else {
        *bc = *bm;
        *gc = *gm;
    }
}

// Slabs for lattices with more than kSlabMinMomentBytes of moments (24 B per
// site; kSlabMinMomentBytesF32 for FP32 storage); below that enough of the
// moment field stays in the 256 MiB Infinity Cache between the passes.  FP32
// lattices get up to about that cache's size unslabbed, where their pass 1
// loads every population non-temporally (pass1_nt_all): measured faster than
// the slabs up to 224^3 (270 MB of moments) and slower from 228^3 (284 MB).
// The 16-bit formats, whose pass 1 keeps the shifted populations cached,
// measured faster in slabs from 208^3 on.  A slab has at least the stencil's
// z-radius planes and about kSlabTouchBytes of traffic per pair of passes
// (moments written and read, populations read and written: 352 B per site in
// FP32, 200 B in FP16/BF16), so the slabs of the launches in flight stay
// cached.  Stochastic rounding keeps whole launches (its step counter
// advances at the first block of pass 1).  Pass 2 of slab k needs the
// moments of slabs k-1..k+1, and pass 1 only reads the source buffer, which
// no pass 2 writes.  n slabs run in n + 2 launches:
//   P1(n-1);  P1(0..1);  then for k = 0..n-1 one launch of P2(k) together
//   with P1(k+2) while k+2 <= n-2 (k_slab_pair), P2(k) alone after that.
// Pass 2 of slab k then finds slabs k-1..k+1 done, and the pass 1 beside it
// writes slab k+2, which it does not read.
static constexpr size_t kSlabTouchBytes = (size_t)192 << 20;
static constexpr size_t kSlabMinMomentBytes = (size_t)128 << 20;
static constexpr size_t kSlabMinMomentBytesF32 = (size_t)264 << 20;

std::vector<SlabOp> slab_schedule(const StepKey &k, const Member &m) {
    std::vector<SlabOp> ops;
    if (k.dim != 3 || k.storage == ST_F64 || k.mom != 1 || k.big || m.sr) return ops;
    const size_t sites = (size_t)m.nx * m.ny;
    const size_t min_bytes = k.storage == ST_F32 ? kSlabMinMomentBytesF32 : kSlabMinMomentBytes;
    if (sites * 24 * m.nz <= min_bytes) return ops;
    const size_t pop = k.storage == ST_F32 ? 4 : 2;
    const size_t touch = 2 * 24 + 4 * 19 * pop + (k.node ? 24 : 0);
    const int rz = k.order == 4 ? 1 : 2;
    const int per = std::max(rz, (int)(kSlabTouchBytes / (sites * touch)));
    const int n = (m.nz + per - 1) / per;
    if (n < 3 || m.nz / n < rz) return ops;
    std::vector<int> z0(n + 1, 0);
    for (int i = 0; i < n; ++i) z0[i + 1] = z0[i] + m.nz / n + (i < m.nz % n ? 1 : 0);
    ops.push_back({1, z0[n - 1], z0[n] - z0[n - 1]});
    ops.push_back({1, z0[0], z0[2] - z0[0]});  // n >= 3: slabs 0 and 1
    for (int i = 0; i < n; ++i) {
        if (i + 2 <= n - 2)
            ops.push_back({3, z0[i], z0[i + 1] - z0[i], z0[i + 2], z0[i + 3] - z0[i + 2]});
        else
            ops.push_back({2, z0[i], z0[i + 1] - z0[i]});
    }
    return ops;
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
            const dim3 g(linear_blocks(m, m.znum, LIN_BLOCK)), b(LIN_BLOCK, 1, 1);
            bool done = false;
            if constexpr (buf_form<D, ST>()) {
                auto go = [&](auto Nc, auto Sc) {
                    constexpr bool NODE = decltype(Nc)::value, SR = decltype(Sc)::value;
                    const std::vector<SlabOp> slabs = slab_schedule(k, m);
                    if (!slabs.empty()) {
                        const dim3 b(SLAB_BLOCK, 1, 1);
                        for (const SlabOp &o : slabs) {
                            Member ms = m;
                            ms.zoff = o.z0;
                            ms.znum = o.nz;
                            const dim3 g(linear_blocks(m, o.nz, SLAB_BLOCK));
                            if (o.pass == 3) {
                                Member m1 = m;
                                m1.zoff = o.z1;
                                m1.znum = o.n1;
                                const int nb2 = (int)g.x;
                                const int nb1 = linear_blocks(m, o.n1, SLAB_BLOCK);
                                hipLaunchKernelGGL((k_slab_pair<O, ST, P, SLAB_BLOCK, NODE>),
                                                   dim3(nb2 + nb1), b, 0, st, ms, m1, nb2, nb1,
                                                   (const T *)src, (T *)dst, (R *)dens);
                            } else if (o.pass == 1)
                                hipLaunchKernelGGL((k_moments_buf<ST, SLAB_BLOCK, NODE>), g, b, 0,
                                                   st, ms, (const T *)src, (R *)dens);
                            else
                                hipLaunchKernelGGL((k_collide_mom_buf<O, ST, P, SLAB_BLOCK, NODE>),
                                                   g, b, 0, st, ms, (const T *)src, (T *)dst,
                                                   (const R *)dens);
                        }
                        done = true;
                    } else if (k.mom && !k.big) {
                        dim3 gm, bm, gc, bc;
                        mom_blocks(m, k.mom == 2, &gm, &bm, &gc, &bc);
                        bool nt_all = false;
                        if constexpr (nt_all_form<ST, NODE>()) nt_all = pass1_nt_all(k, m.N);
                        if (nt_all)
                            hipLaunchKernelGGL((k_moments_buf<ST, LIN_BLOCK, false, PULL_NT_ALL>),
                                               gm, bm, 0, st, m, (const T *)src, (R *)dens);
                        else
                            hipLaunchKernelGGL((k_moments_buf<ST, LIN_BLOCK, NODE>), gm, bm, 0, st,
                                               m, (const T *)src, (R *)dens);
                        if (k.mom == 2)
                            hipLaunchKernelGGL(
                                (k_collide_mom_lds<CL_TX, CL_TY, CL_ZC, O, ST, P, NODE, SR>), gc,
                                bc, 0, st, m, (const T *)src, (T *)dst, (const R *)dens);
                        else
                            hipLaunchKernelGGL((k_collide_mom_buf<O, ST, P, LIN_BLOCK, NODE, SR>),
                                               gc, bc, 0, st, m, (const T *)src, (T *)dst,
                                               (const R *)dens);
                        done = true;
                    }
                };
                if (k.node) {
                    if constexpr (node_form<D, ST>()) go(std::true_type{}, std::false_type{});
                } else if (k.sr) {
                    if constexpr (sr_form<ST>()) go(std::false_type{}, std::true_type{});
                } else {
                    go(std::false_type{}, std::false_type{});
                }
            }
            if (done) {
            } else if (k.node) {  // node storage runs in the buffer forms only
                err = hipErrorNotSupported;
                return;
            } else if (k.mom) {
                hipLaunchKernelGGL((k_moments<D, ST>), g, b, 0, st, m,
                                   (const T *)src, (R *)dens);
                hipLaunchKernelGGL((k_collide_mom<D, O, ST, P>), g, b, 0, st, m,
                                   (const T *)src, (T *)dst, (const R *)dens);
            } else {
                hipLaunchKernelGGL((k_density<D, ST>), g, b, 0, st, m,
                                   (const T *)src, (R *)dens);
                hipLaunchKernelGGL((k_collide<D, O, ST, P>), g, b, 0, st, m,
                                   (const T *)src, (T *)dst, (const R *)dens);
            }
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
            dn->func = k.mom ? (void *)&k_moments<D, ST> : (void *)&k_density<D, ST>;
            sn->func = k.mom ? (void *)&k_collide_mom<D, O, ST, P>
                             : (void *)&k_collide<D, O, ST, P>;
            dn->grid = sn->grid = dim3(linear_blocks(m, m.znum, LIN_BLOCK));
            dn->block = sn->block = dim3(LIN_BLOCK, 1, 1);
            dn->shmem = sn->shmem = 0;
            if constexpr (buf_form<D, ST>()) {
                auto set = [&](auto Nc, auto Sc) {
                    constexpr bool NODE = decltype(Nc)::value, SR = decltype(Sc)::value;
                    dn->func = (void *)&k_moments_buf<ST, LIN_BLOCK, NODE>;
                    if constexpr (nt_all_form<ST, NODE>())
                        if (pass1_nt_all(k, m.N))
                            dn->func = (void *)&k_moments_buf<ST, LIN_BLOCK, false, PULL_NT_ALL>;
                    sn->func =
                        k.mom == 2
                            ? (void *)&k_collide_mom_lds<CL_TX, CL_TY, CL_ZC, O, ST, P, NODE, SR>
                            : (void *)&k_collide_mom_buf<O, ST, P, LIN_BLOCK, NODE, SR>;
                    mom_blocks(m, k.mom == 2, &dn->grid, &dn->block, &sn->grid, &sn->block);
                    if (!slab_schedule(k, m).empty()) {  // slab launches: grid set per slab
                        dn->func = (void *)&k_moments_buf<ST, SLAB_BLOCK, NODE>;
                        sn->func = (void *)&k_collide_mom_buf<O, ST, P, SLAB_BLOCK, NODE>;
                        dn->block = sn->block = dim3(SLAB_BLOCK, 1, 1);
                    }
                };
                if (k.mom && !k.big) {
                    if (k.node) {
                        if constexpr (node_form<D, ST>()) set(std::true_type{}, std::false_type{});
                    } else if (k.sr) {
                        if constexpr (sr_form<ST>()) set(std::false_type{}, std::true_type{});
                    } else {
                        set(std::false_type{}, std::false_type{});
                    }
                }
            }
            ok = !k.node || (node_form<D, ST>() && k.mom && !k.big);
        });
    });
    return ok;
}

bool node_slab_pair(const StepKey &k, NodeLaunch *pn) {
    bool ok = false;
    dispatch_storage(k.storage, [&](auto stv) {
        using ST = decltype(stv);
        dispatch_shape<ST>(k, [&](auto Dc, auto Oc, auto Pc) {
            constexpr int D = decltype(Dc)::value;
            constexpr int O = decltype(Oc)::value;
            constexpr int P = decltype(Pc)::value;
            if constexpr (buf_form<D, ST>()) {
                auto set = [&](auto Nc) {
                    constexpr bool NODE = decltype(Nc)::value;
                    pn->func = (void *)&k_slab_pair<O, ST, P, SLAB_BLOCK, NODE>;
                    pn->block = dim3(SLAB_BLOCK, 1, 1);
                    pn->shmem = 0;
                    ok = true;
                };
                if (!k.node) {
                    set(std::false_type{});
                } else if constexpr (node_form<D, ST>()) {
                    set(std::true_type{});
                }
            }
        });
    });
    return ok;
}

int resident_blocks(const void *f, int threads, unsigned shmem) {
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, int, unsigned>, int> cache;
    constexpr int kNoLimit = 1 << 30;  // occupancy unknown: keep the caller's grid
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kNoLimit;
    const auto key = std::make_tuple(f, dev, threads, shmem);
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, threads, shmem) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per < 1 || ncu < 1)
        return kNoLimit;
    return cache[key] = per * ncu;
}

hipError_t launch_batch_two_pass(const StepKey &k, const Member *d_members,
                                 const Tile *d_tiles, int ntiles,
                                 const void *src, void *dst, void *dens,
                                 int grid, hipStream_t st, int passes, bool nt_all) {
    const bool p1 = passes & 1, p2 = passes & 2;
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
            bool done = false;
            if constexpr (buf_form<D, ST>()) {
                if (k.mom && !k.big) {
                    bool all = false;
                    if constexpr (nt_all_form<ST, false>()) all = nt_all;
                    if (p1 && all)
                        hipLaunchKernelGGL((kb_moments_buf<ST, PULL_NT_ALL>), dim3(grid), b, 0, st,
                                           d_members, d_tiles, ntiles, (const T *)src,
                                           (R *)dens);
                    else if (p1)
                        hipLaunchKernelGGL((kb_moments_buf<ST>), dim3(grid), b, 0, st,
                                           d_members, d_tiles, ntiles, (const T *)src,
                                           (R *)dens);
                    if (p2 && k.sr) {
                        if constexpr (!sr_form<ST>()) {
                            err = hipErrorNotSupported;
                            return;
                        } else {
                            hipLaunchKernelGGL((kb_collide_mom_buf<O, ST, P, true>), dim3(grid), b,
                                               0, st, d_members, d_tiles, ntiles, (const T *)src,
                                               (T *)dst, (const R *)dens);
                        }
                    } else if (p2) {
                        hipLaunchKernelGGL((kb_collide_mom_buf<O, ST, P>), dim3(grid), b, 0,
                                           st, d_members, d_tiles, ntiles, (const T *)src,
                                           (T *)dst, (const R *)dens);
                    }
                    done = true;
                }
            }
            if (done) {
            } else if (k.mom) {
                if (p1)
                    hipLaunchKernelGGL((kb_moments<D, ST>), dim3(grid), b, 0, st,
                                       d_members, d_tiles, ntiles, (const T *)src,
                                       (R *)dens);
                if (p2)
                    hipLaunchKernelGGL((kb_collide_mom<D, O, ST, P>), dim3(grid), b, 0,
                                       st, d_members, d_tiles, ntiles, (const T *)src,
                                       (T *)dst, (const R *)dens);
            } else {
                if (p1)
                    hipLaunchKernelGGL((kb_density<D, ST>), dim3(grid), b, 0, st,
                                       d_members, d_tiles, ntiles, (const T *)src,
                                       (R *)dens);
                if (p2)
                    hipLaunchKernelGGL((kb_collide<D, O, ST, P>), dim3(grid), b, 0,
                                       st, d_members, d_tiles, ntiles, (const T *)src,
                                       (T *)dst, (const R *)dens);
            }
            err = hipGetLastError();
        });
    });
    return err;
}

bool node_member_pass(const StepKey &k, const Member &m, int pass, bool nt_all,
                      NodeLaunch *nl) {
    bool ok = false;
    if (k.node || k.sr || !k.mom || k.big) return false;
    dispatch_storage(k.storage, [&](auto stv) {
        using ST = decltype(stv);
        dispatch_shape<ST>(k, [&](auto Dc, auto Oc, auto Pc) {
            constexpr int D = decltype(Dc)::value;
            constexpr int O = decltype(Oc)::value;
            constexpr int P = decltype(Pc)::value;
            if constexpr (buf_form<D, ST>()) {
                nl->grid = dim3(linear_blocks(m, m.znum, LIN_BLOCK));
                nl->block = dim3(LIN_BLOCK, 1, 1);
                nl->shmem = 0;
                if (pass == 1) {
                    nl->func = (void *)&k_moments_buf<ST, LIN_BLOCK>;
                    if constexpr (nt_all_form<ST, false>())
                        if (nt_all)
                            nl->func = (void *)&k_moments_buf<ST, LIN_BLOCK, false, PULL_NT_ALL>;
                } else {
                    nl->func = (void *)&k_collide_mom_buf<O, ST, P, LIN_BLOCK>;
                }
                ok = true;
            }
        });
    });
    return ok;
}

hipError_t launch_member_pass(const StepKey &k, const Member &m, const void *src, void *dst,
                              void *dens, int pass, bool nt_all, hipStream_t st) {
    NodeLaunch nl{};
    if (!node_member_pass(k, m, pass, nt_all, &nl)) return hipErrorNotSupported;
    Member mv = m;
    const void *srcv = src;
    void *dstv = dst, *densv = dens;
    void *a1[] = {(void *)&mv, (void *)&srcv, (void *)&densv};
    void *a2[] = {(void *)&mv, (void *)&srcv, (void *)&dstv, (void *)&densv};
    return hipLaunchKernel(nl.func, nl.grid, nl.block, pass == 1 ? a1 : a2, 0, st);
}

bool node_batch_two_pass(const StepKey &k, int grid, NodeLaunch *dn,
                         NodeLaunch *sn, NodeLaunch *dn_all) {
    bool ok = false;
    dispatch_storage(k.storage, [&](auto stv) {
        using ST = decltype(stv);
        dispatch_shape<ST>(k, [&](auto Dc, auto Oc, auto Pc) {
            constexpr int D = decltype(Dc)::value;
            constexpr int O = decltype(Oc)::value;
            constexpr int P = decltype(Pc)::value;
            dn->func = k.mom ? (void *)&kb_moments<D, ST> : (void *)&kb_density<D, ST>;
            sn->func = k.mom ? (void *)&kb_collide_mom<D, O, ST, P>
                             : (void *)&kb_collide<D, O, ST, P>;
            if constexpr (buf_form<D, ST>()) {
                if (k.mom && !k.big) {
                    dn->func = (void *)&kb_moments_buf<ST>;
                    sn->func = (void *)&kb_collide_mom_buf<O, ST, P>;
                    if constexpr (sr_form<ST>())
                        if (k.sr) sn->func = (void *)&kb_collide_mom_buf<O, ST, P, true>;
                }
            }
            dn->grid = sn->grid = dim3(grid);
            dn->block = sn->block = dim3(TP_BX, TP_BY, 1);
            dn->shmem = sn->shmem = 0;
            if (dn_all) {
                *dn_all = *dn;
                if constexpr (buf_form<D, ST>() && nt_all_form<ST, false>())
                    if (k.mom && !k.big) dn_all->func = (void *)&kb_moments_buf<ST, PULL_NT_ALL>;
            }
            ok = true;
        });
    });
    return ok;
}

}  // namespace scmc
