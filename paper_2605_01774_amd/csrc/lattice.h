// Velocity set (D3Q19, or D3Q27 when built with ELBM_Q=27) and the storage forms of the
// populations (device side).
//
// Velocity order: 0 rest; 1..6 axis (+x, -x, +y, -y, +z, -z); 7..18 the 12 edge
// directions; D3Q27 adds 19..26, the 8 corner directions. Opposite directions are
// adjacent: every odd index i >= 1 has its opposite at i + 1. Weights by the number m of
// nonzero components: D3Q19 1/3, 1/18, 1/36; D3Q27 the tensor-product rule of Sec. 2.1,
// (2/3)^(3-m) (1/6)^m = 8/27, 2/27, 1/54, 1/216. cs^2 = 1/3 for both, so the flux lift is
// P_i(a) = (W_i / cs^2) c_i . a = 3 W_i c_i . a (Sec. 2.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#ifndef ELBM_Q
#define ELBM_Q 19
#endif
#if ELBM_Q != 19 && ELBM_Q != 27
#error "ELBM_Q must be 19 or 27"
#endif

namespace elbm {

constexpr int Q = ELBM_Q;

__host__ __device__ constexpr int cx(int i) {
    constexpr int v[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                           1, -1, 1, -1, 1, -1, -1, 1};
    return v[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int v[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                           1, -1, 1, -1, -1, 1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int v[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                           1, -1, -1, 1, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// number of nonzero velocity components (0 rest, 1 axis, 2 edge, 3 corner)
__host__ __device__ constexpr int vclass(int i) {
    return (cx(i) != 0) + (cy(i) != 0) + (cz(i) != 0);
}
__host__ __device__ constexpr double class_weight(int m) {
    return Q == 19 ? (m == 0 ? 1.0 / 3.0 : (m == 1 ? 1.0 / 18.0 : 1.0 / 36.0))
                   : (m == 0 ? 8.0 / 27.0 : (m == 1 ? 2.0 / 27.0 : (m == 2 ? 1.0 / 54.0 : 1.0 / 216.0)));
}
__host__ __device__ constexpr double weight(int i) { return class_weight(vclass(i)); }
constexpr int NCLASS = Q == 19 ? 3 : 4;

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

// Step counters (fallback, exact root, non-finite, guard), each spread over kCntSlots
// copies 128 bytes apart that blocks pick by their index: the counted events can occur at
// most nodes of a step (fallback and guard on a zero background), and one address taking
// every atomic serialises them. The readout sums the slots.
constexpr int kNumCounters = 4;
constexpr int kCntSlots = 256;
constexpr int kCntStride = 16;  // 64-bit words: 128 bytes
__host__ __device__ inline size_t cnt_index(int counter, unsigned slot) {
    return (size_t(counter) * kCntSlots + (slot & (kCntSlots - 1))) * kCntStride;
}
constexpr size_t kCntWords = size_t(kNumCounters) * kCntSlots * kCntStride;

// ------------------------------------------------------------------------------------------
// Population buffers are row chunks: the Q populations of x-row r = z ny + y are Q
// consecutive runs of nx values ([z][y][i][x]), so the whole state of a row is one
// contiguous block of memory. In the rest-in-FP32 layout of the 16-bit forms, run 0 holds the
// row's nx FP32 rest values (the space of two runs of the 16-bit type) and run i >= 1
// starts at (i + 1) nx.
// ------------------------------------------------------------------------------------------
static_assert((Q + 1) % 2 == 0, "a row's FP32 rest run must fill whole 16-bit runs");

__host__ __device__ inline size_t row_elems(int nx, int rest32) {
    return size_t(Q + (rest32 ? 1 : 0)) * size_t(nx);
}
// element offset of run i (population i) within a row
__host__ __device__ inline size_t run_offset(int i, int nx, int rest32) {
    return size_t((rest32 && i) ? i + 1 : i) * size_t(nx);
}
// element offset of population i of the node at column x of row r
__host__ __device__ inline size_t pop_offset(int i, long long r, int x, int nx, int rest32) {
    return size_t(r) * row_elems(nx, rest32) + run_offset(i, nx, rest32) + size_t(x);
}
// FP32 index of the rest value of the node at column x of row r (rest-in-FP32 layout)
__host__ __device__ inline size_t rest_offset(long long r, int x, int nx) {
    return size_t(r) * (row_elems(nx, 1) / 2) + size_t(x);
}

template <class ST>
__device__ inline typename Store<ST>::Real pop_load(const ST* buf, int i, long long r, int x, int nx,
                                                    int rest32, typename Store<ST>::Real scale) {
    if constexpr (sizeof(ST) == 2) {
        if (rest32 && i == 0) return reinterpret_cast<const float*>(buf)[rest_offset(r, x, nx)];
    }
    return Store<ST>::load(buf + pop_offset(i, r, x, nx, rest32), scale);
}

template <class ST>
__device__ inline void pop_put(ST* buf, int i, long long r, int x, int nx, typename Store<ST>::Real v,
                               int rest32, typename Store<ST>::Real inv_scale) {
    if constexpr (sizeof(ST) == 2) {
        if (rest32 && i == 0) {
            reinterpret_cast<float*>(buf)[rest_offset(r, x, nx)] = v;
            return;
        }
    }
    Store<ST>::put(buf + pop_offset(i, r, x, nx, rest32), v, inv_scale);
}

// ------------------------------------------------------------------------------------------
// Storage rounding of the 16-bit forms.
// ------------------------------------------------------------------------------------------
// 32 random bits from a 32-bit counter: the PCG output permutation used as a hash
// (Jarzynski and Olano, "Hash Functions for GPU Rendering", JCGT 9(3), 2020).
__host__ __device__ inline uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

// The FP32 value a 16-bit store of v holds: round to nearest even, or (sround) stochastic
// rounding with the 32 random bits r by the gfx950 conversions v_cvt_sr_bf16_f32 /
// v_cvt_sr_f16_f32 (FP16 of v / scale). The result converts to the storage type exactly.
// RAW: the result in storage units (FP16: the stored value itself, not times scale).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <class ST, bool RAW = false>
__device__ inline float quantize16(float v, uint32_t r, bool sround, float scale, float inv_scale) {
    if constexpr (std::is_same<ST, bf16s>::value) {
        if (sround) return float(__builtin_amdgcn_cvt_sr_bf16_f32(bf16x2{}, v, r, false)[0]);
        return float(static_cast<__bf16>(v));
    } else {
        const float y = v * inv_scale;
        const float h = sround ? float(__builtin_amdgcn_cvt_sr_f16_f32(f16x2{}, y, r, false)[0]) : float(_Float16(y));
        return RAW ? h : h * scale;
    }
}

// Stochastic rounding of the two members of an opposite pair into the two halves of one
// register: v0 with the random word w, v1 with w rotated by 16 bits (the conversions use the
// word's top bits, so the two draw on disjoint bits). q0 and q1 are the FP32 values the two
// 16-bit stores hold, bitwise the same as quantize16's (RAW: in storage units). Each
// conversion writes one half of the register, so the register needs no clearing first.
template <class ST, bool RAW = false>
__device__ inline void quantize16_sr_pair(float v0, float v1, uint32_t w, float scale, float inv_scale,
                                          float& q0, float& q1) {
    const uint32_t w1 = (w << 16) | (w >> 16);
    if constexpr (std::is_same<ST, bf16s>::value) {
        bf16x2 pk = __builtin_bit_cast(bf16x2, w);
        pk = __builtin_amdgcn_cvt_sr_bf16_f32(pk, v0, w, false);
        pk = __builtin_amdgcn_cvt_sr_bf16_f32(pk, v1, w1, true);
        const uint32_t b = __builtin_bit_cast(uint32_t, pk);
        q0 = __uint_as_float(b << 16);
        q1 = __uint_as_float(b & 0xFFFF0000u);
    } else {
        f16x2 pk = __builtin_bit_cast(f16x2, w);
        pk = __builtin_amdgcn_cvt_sr_f16_f32(pk, v0 * inv_scale, w, false);
        pk = __builtin_amdgcn_cvt_sr_f16_f32(pk, v1 * inv_scale, w1, true);
        q0 = RAW ? float(pk[0]) : float(pk[0]) * scale;
        q1 = RAW ? float(pk[1]) : float(pk[1]) * scale;
    }
}

// Random words for the stochastic rounding of one node: a PCG-hashed seed per node, then a
// Weyl sequence (increments of 2^32 / golden ratio, odd, so also a full-period sequence in
// the low 16 bits). Each word, and each of its two 16-bit halves, is uniform because the
// hashed seed is; the words of one node differ by fixed offsets, which spreads their
// rounding thresholds evenly rather than independently. One add per word, where a
// generator step would need a quarter-rate integer multiply.
struct RoundingBits {
    uint32_t s;
    __device__ explicit RoundingBits(uint32_t seed) : s(pcg_hash(seed)) {}
    __device__ uint32_t next() {
        s += 0x9E3779B9u;
        return s;
    }
};

}  // namespace elbm
