// lattice.h -- compile-time tables of the GPU library: velocity sets, lattice
// weights and force stencils, plus the population storage formats.
//
// Velocity sets (paper Sec. 2): D3Q19 with c_s^2 = 1/3, and its 2D analogue
// D2Q9.  Force stencils (eq. sc_force): vectors e_a with squared length s and
// weight W(s), normalised so that e2 = sum_a W_a (e_a^x)^2 = 1 (Sec. 2, after
// eq. bulkp).  Order 4 in 3D is the paper's W(1) = 1/6, W(2) = 1/12; the other
// sets solve the isotropy conditions of the corresponding order:
//   2D E4: W(1) = 1/3, W(2) = 1/12
//   2D E6: W(1) = 4/15, W(2) = 1/10, W(4) = 1/120
//   2D E8: W(1) = 4/21, W(2) = 4/45, W(4) = 1/60, W(5) = 2/315, W(8) = 1/5040
//   3D E6: W(1) = 2/15, W(2) = 1/15, W(3) = 1/60, W(4) = 1/120
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace scmc {

// ---------------------------------------------------------------- velocities
template <int D> struct Lattice;

template <> struct Lattice<2> {
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int CZ[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double W[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,
                                    1.0 / 9,  1.0 / 9,  1.0 / 36,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36};
};

template <> struct Lattice<3> {
    static constexpr int D = 3;
    static constexpr int Q = 19;
    static constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1,
                                   -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1,
                                   1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0,
                                   0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr double W[19] = {
        1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

// opp[i] = index of the velocity opposite to xi_i
template <int D> struct Opposite {
    int opp[Lattice<D>::Q];
    static constexpr Opposite make() {
        using L = Lattice<D>;
        Opposite o{};
        for (int i = 0; i < L::Q; ++i)
            for (int j = 0; j < L::Q; ++j)
                if (L::CX[j] == -L::CX[i] && L::CY[j] == -L::CY[i] &&
                    L::CZ[j] == -L::CZ[i])
                    o.opp[i] = j;
        return o;
    }
};

// ------------------------------------------------------------ force stencils
constexpr double stencil_weight(int D, int order, int s) {
    if (D == 2 && order == 4) return s == 1 ? 1.0 / 3 : s == 2 ? 1.0 / 12 : 0.0;
    if (D == 2 && order == 6)
        return s == 1 ? 4.0 / 15 : s == 2 ? 1.0 / 10 : s == 4 ? 1.0 / 120 : 0.0;
    if (D == 2 && order == 8)
        return s == 1   ? 4.0 / 21
               : s == 2 ? 4.0 / 45
               : s == 4 ? 1.0 / 60
               : s == 5 ? 2.0 / 315
               : s == 8 ? 1.0 / 5040
                        : 0.0;
    if (D == 3 && order == 4) return s == 1 ? 1.0 / 6 : s == 2 ? 1.0 / 12 : 0.0;
    if (D == 3 && order == 6)
        return s == 1   ? 2.0 / 15
               : s == 2 ? 1.0 / 15
               : s == 3 ? 1.0 / 60
               : s == 4 ? 1.0 / 120
                        : 0.0;
    return 0.0;
}

constexpr int stencil_count(int D, int order) {
    int n = 0;
    for (int z = (D == 3 ? -2 : 0); z <= (D == 3 ? 2 : 0); ++z)
        for (int y = -2; y <= 2; ++y)
            for (int x = -2; x <= 2; ++x) {
                int s = x * x + y * y + z * z;
                if (s > 0 && stencil_weight(D, order, s) != 0.0) ++n;
            }
    return n;
}

template <int D, int ORDER> struct Stencil {
    static constexpr int NE = stencil_count(D, ORDER);
    static constexpr int R = ORDER == 4 ? 1 : 2;  // radius (max |e^k|)
    struct Table {
        int e[NE][3];
        double W[NE];
    };
    static constexpr Table make() {
        Table t{};
        int n = 0;
        for (int z = (D == 3 ? -2 : 0); z <= (D == 3 ? 2 : 0); ++z)
            for (int y = -2; y <= 2; ++y)
                for (int x = -2; x <= 2; ++x) {
                    int s = x * x + y * y + z * z;
                    double w = s > 0 ? stencil_weight(D, ORDER, s) : 0.0;
                    if (w != 0.0) {
                        t.e[n][0] = x;
                        t.e[n][1] = y;
                        t.e[n][2] = z;
                        t.W[n] = w;
                        ++n;
                    }
                }
        return t;
    }
    static constexpr Table T = make();
    // the table runs lexicographically over (z, y, x), so entry NE - 1 - a is
    // the opposite of entry a with the same weight
    static constexpr bool point_symmetric() {
        for (int a = 0; a < NE; ++a)
            for (int k = 0; k < 3; ++k)
                if (T.e[NE - 1 - a][k] != -T.e[a][k] || T.W[NE - 1 - a] != T.W[a]) return false;
        return NE % 2 == 0;
    }
};

// ----------------------------------------------------------- storage formats
// load(p, i, ref) returns the population in compute precision; ref = w_i n0_J
// is the offset reference (used by the FP16 / BF16 offset formats only).
// Stores are non-temporal: every population is written once per step and
// only read again by the next step, after the whole buffer has streamed.
struct StoreF64 {
    using T = double;
    using R = double;
    static constexpr int BYTES = 8;
    __device__ __forceinline__ static R from_raw(T v, R) { return v; }
    __device__ __forceinline__ static T to_raw(R v, R) { return v; }
    __device__ __forceinline__ static R load(const T *p, long i, R) { return p[i]; }
    __device__ __forceinline__ static void store(T *p, long i, R v, R) {
        __builtin_nontemporal_store(v, p + i);
    }
    __device__ __forceinline__ static T to_raw_sr(R v, R, unsigned) { return v; }
};

struct StoreF32 {
    using T = float;
    using R = float;
    static constexpr int BYTES = 4;
    __device__ __forceinline__ static R from_raw(T v, R) { return v; }
    __device__ __forceinline__ static T to_raw(R v, R) { return v; }
    __device__ __forceinline__ static R load(const T *p, long i, R) { return p[i]; }
    __device__ __forceinline__ static void store(T *p, long i, R v, R) {
        __builtin_nontemporal_store(v, p + i);
    }
    __device__ __forceinline__ static T to_raw_sr(R v, R, unsigned) { return v; }
};

struct StoreF16 {
    using T = uint16_t;
    using R = float;
    static constexpr int BYTES = 2;
    __device__ __forceinline__ static R from_raw(T v, R ref) {
        return __half2float(__ushort_as_half(v)) + ref;
    }
    __device__ __forceinline__ static T to_raw(R v, R ref) {
        return __half_as_ushort(__float2half_rn(v - ref));
    }
    __device__ __forceinline__ static R load(const T *p, long i, R ref) {
        return __half2float(__ushort_as_half(p[i])) + ref;
    }
    __device__ __forceinline__ static void store(T *p, long i, R v, R ref) {
        const T h = __half_as_ushort(__float2half_rn(v - ref));
        __builtin_nontemporal_store(h, p + i);
    }
    // Node storage (offsets from the node's own rest equilibrium, which are
    // small where the flow is slow): the offset is scaled by 2^10 before it
    // is rounded, so offsets down to 2^-24 stay normal numbers with 11
    // significant bits (and up to 64 in size) instead of falling into the
    // half subnormals; the power-of-two scale itself is exact.
    static constexpr float NODE_SCALE = 1024.0f, NODE_UNSCALE = 1.0f / 1024.0f;
    __device__ __forceinline__ static T to_node(R v, R ref) {
        return __half_as_ushort(__float2half_rn((v - ref) * NODE_SCALE));
    }
    __device__ __forceinline__ static R from_node(T v, R ref) {
        return __half2float(__ushort_as_half(v)) * NODE_UNSCALE + ref;
    }
    // Stochastic rounding: 13 random bits added below the half's last
    // mantissa bit, then truncation.  Half subnormals (|h| < 2^-14) are
    // rounded to nearest, their absolute error being below 2^-25.
    __device__ __forceinline__ static T to_raw_sr(R v, R ref, unsigned r) {
        const float x = v - ref;
        if (!(fabsf(x) >= 6.103515625e-05f) || fabsf(x) > 6.5e4f) return to_raw(v, ref);
        const unsigned u = __float_as_uint(x) + (r & 0x1FFFu);
        return __half_as_ushort(__float2half_rz(__uint_as_float(u)));
    }
};

// bfloat16 = the top 16 bits of an IEEE binary32; rounding to nearest even
__host__ __device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float v;
    __builtin_memcpy(&v, &u, 4);
    return v;
}

// The same rounding in one instruction: gfx950 converts binary32 to bfloat16
// in hardware, to nearest even in the default rounding mode, keeping
// subnormals (the FP32 denormal mode of HIP code) and quieting NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_dev(float v) {
    return __builtin_bit_cast(uint16_t, (__bf16)v);
}

struct StoreBF16 {
    using T = uint16_t;
    using R = float;
    static constexpr int BYTES = 2;
    __device__ __forceinline__ static R from_raw(T v, R ref) {
        return bf16_to_f32(v) + ref;
    }
    __device__ __forceinline__ static T to_raw(R v, R ref) {
        return f32_to_bf16_dev(v - ref);
    }
    __device__ __forceinline__ static R load(const T *p, long i, R ref) {
        return bf16_to_f32(p[i]) + ref;
    }
    __device__ __forceinline__ static void store(T *p, long i, R v, R ref) {
        const T h = f32_to_bf16_dev(v - ref);
        __builtin_nontemporal_store(h, p + i);
    }
    // node storage: bfloat16 has the binary32 exponent range, no scale
    __device__ __forceinline__ static T to_node(R v, R ref) { return to_raw(v, ref); }
    __device__ __forceinline__ static R from_node(T v, R ref) { return from_raw(v, ref); }
    // Stochastic rounding: 16 random bits added below the kept half of the
    // binary32 pattern, then truncation (sign-magnitude: unbiased for both
    // signs); infinities and NaN go the nearest-even way.
    __device__ __forceinline__ static T to_raw_sr(R v, R ref, unsigned r) {
        const float x = v - ref;
        const uint32_t u = __float_as_uint(x);
        if ((u & 0x7f800000u) == 0x7f800000u) return f32_to_bf16_dev(x);
        return (uint16_t)((u + (r & 0xFFFFu)) >> 16);
    }
};

}  // namespace scmc
