// ceiling_kernels.hip -- the streaming half of the step without its
// arithmetic: every population of one buffer copied to the other with the
// pull shifts of eq. lbm, f_i(x) <- f_i(x - xi_i), periodic.  It reads and
// writes every population once in the step's access pattern (one site per
// lane, x-aligned loads non-temporal, non-temporal stores), so its bandwidth
// is the practical ceiling of any step design that moves each population
// once; the benchmark states the step's bandwidth against it.
#include "site_ops.h"

namespace scmc {

template <int D, class T>
__global__ void __launch_bounds__(256)
    k_pull_copy(Member m, const T *__restrict__ src, T *__restrict__ dst) {
    using L = Lattice<D>;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= m.N) return;
    const int nxy = m.nx * m.ny;
    const int z = s / nxy, r = s - z * nxy, y = r / m.nx, x = r - y * m.nx;
    T v[2 * L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int zs = D == 3 ? wrap1(z - L::CZ[i], m.nz) : 0;
        const int t = (zs * m.ny + wrap1(y - L::CY[i], m.ny)) * m.nx + wrap1(x - L::CX[i], m.nx);
        const T *a = src + (long)i * m.N + t, *b = src + (long)(L::Q + i) * m.N + t;
        if (L::CX[i] == 0) {
            v[i] = __builtin_nontemporal_load(a);
            v[L::Q + i] = __builtin_nontemporal_load(b);
        } else {
            v[i] = *a;
            v[L::Q + i] = *b;
        }
    }
#pragma unroll
    for (int k = 0; k < 2 * L::Q; ++k) __builtin_nontemporal_store(v[k], dst + (long)k * m.N + s);
}

hipError_t launch_pull_copy(int dim, int bytes, const Member &m, const void *src, void *dst,
                            hipStream_t st) {
    const dim3 g((m.N + 255) / 256), b(256);
    auto go = [&](auto Dc, auto tv) {
        constexpr int D = decltype(Dc)::value;
        using T = decltype(tv);
        hipLaunchKernelGGL((k_pull_copy<D, T>), g, b, 0, st, m, (const T *)src, (T *)dst);
    };
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    if (dim == 2 && bytes == 8) go(I2{}, double{});
    else if (dim == 2 && bytes == 4) go(I2{}, float{});
    else if (dim == 2 && bytes == 2) go(I2{}, uint16_t{});
    else if (dim == 3 && bytes == 8) go(I3{}, double{});
    else if (dim == 3 && bytes == 4) go(I3{}, float{});
    else if (dim == 3 && bytes == 2) go(I3{}, uint16_t{});
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace scmc
