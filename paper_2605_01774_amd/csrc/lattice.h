// D3Q19 velocity set and the storage forms of the populations (device side).
//
// Velocity order: 0 rest; 1..6 axis (+x, -x, +y, -y, +z, -z); 7..18 edges in opposite
// pairs. Every odd index i >= 1 has its opposite at i + 1. Weights 1/3, 1/18, 1/36;
// cs^2 = 1/3, so the flux lift P_i(a) = (W_i / cs^2) c_i . a = 3 W_i c_i . a (Sec. 2.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace elbm {

constexpr int Q = 19;

__host__ __device__ constexpr int cx(int i) {
    constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double weight(int i) {
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ------------------------------------------------------------------------------------------
// Storage forms. `Real` is the arithmetic type; values are deviations d_i = g_i - W_i phi_ref
// (scaled for 16-bit forms).
// ------------------------------------------------------------------------------------------
struct bf16s {
    uint16_t bits;
};

template <class S>
struct Store;

template <>
struct Store<double> {
    using Real = double;
    __device__ static inline double load(const double* p, double) { return *p; }
    __device__ static inline void put(double* p, double v, double) { *p = v; }
};

template <>
struct Store<float> {
    using Real = float;
    __device__ static inline float load(const float* p, float) { return *p; }
    __device__ static inline void put(float* p, float v, float) { *p = v; }
};

// BF16 keeps the FP32 exponent range, so it is stored unscaled; conversion is the hardware
// round-to-nearest-even (v_cvt_pk_bf16_f32 on gfx950).
template <>
struct Store<bf16s> {
    using Real = float;
    __device__ static inline float load(const bf16s* p, float) {
        return __uint_as_float(uint32_t(p->bits) << 16);
    }
    __device__ static inline void put(bf16s* p, float v, float) {
        p->bits = __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
    }
};

template <>
struct Store<_Float16> {
    using Real = float;
    __device__ static inline float load(const _Float16* p, float scale) { return float(*p) * scale; }
    __device__ static inline void put(_Float16* p, float v, float inv_scale) {
        *p = _Float16(v * inv_scale);
    }
};

}  // namespace elbm
