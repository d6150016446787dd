// Reciprocal and ln(1 + x) in the arithmetic type, for the per-node equilibrium factors of a
// velocity field.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace elbm {

// Reciprocal in the arithmetic type, for positive normal arguments near 1 (products of
// equilibrium factors E_i, and 2 + x in log1p_e). FP32: the hardware reciprocal (1 ulp). FP64: the
// hardware estimate refined by two Newton steps r <- r + r (1 - x r), each of which
// doubles the number of correct bits, to about 1 ulp; a third of the instructions of an
// IEEE division, which matters where a velocity field needs 28 of them per node.
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// libm log1p, kept out of line: it is taken only for |u| beyond about 0.1, and inlined
// at each of the Q call sites it would double the kernel's code size.
static __device__ __attribute__((noinline)) double log1p_libm(double x) { return log1p(x); }

// ln E_i = ln(1 + x) from the excess x = E_i - 1 (E_i a positive normal number).
// FP64: for |x| <= 0.4 (every E_i of |u| up to about 0.1) the series
// ln(1 + x) = 2 atanh(t) = 2 (t + t^3/3 + ... + t^25/25), t = x / (2 + x), -1/4 <= t <= 1/6,
// whose first omitted term is below 1e-17 of the result; libm log1p otherwise.
// FP32: the hardware log2 (1 ulp) of u = fl(1 + x), times ln 2, plus the rounding of 1 + x:
// with d = u - 1 (exact) and e = x - d, ln(1 + x) = ln u + ln(1 + e / u) = ln u + e + O(e d),
// and |e| is at most half an ulp of 1, so the O(e d) term stays below an ulp of the result
// (1.6e-7 relative at most over |x| <= 0.4) and small excesses keep their relative
// precision without a division.
__device__ __forceinline__ double log1p_e(double x) {
    if (!(fabs(x) <= 0.4)) return log1p_libm(x);
    const double t = x * recip(2.0 + x);
    const double t2 = t * t;
    double p = 1.0 / 25.0;
    p = fma(p, t2, 1.0 / 23.0);
    p = fma(p, t2, 1.0 / 21.0);
    p = fma(p, t2, 1.0 / 19.0);
    p = fma(p, t2, 1.0 / 17.0);
    p = fma(p, t2, 1.0 / 15.0);
    p = fma(p, t2, 1.0 / 13.0);
    p = fma(p, t2, 1.0 / 11.0);
    p = fma(p, t2, 1.0 / 9.0);
    p = fma(p, t2, 1.0 / 7.0);
    p = fma(p, t2, 1.0 / 5.0);
    p = fma(p, t2, 1.0 / 3.0);
    p = fma(p, t2, 1.0);
    return 2.0 * t * p;
}
__device__ __forceinline__ float log1p_e(float x) {
    const float u = 1.0f + x;
    const float d = u - 1.0f;
    const float l = __builtin_amdgcn_logf(u) * 0.693147180559945309f;
    return l + (x - d);
}

// Sum of h_i ln(1 + x_i) over the terms added. FP64: log1p_e per term. FP32: the terms'
// log2 u_i and rounding corrections x_i - (u_i - 1) are accumulated apart and ln 2 is applied
// once (the same expansion as log1p_e, one multiply less per term). CORR = false (FP32) drops
// the corrections, three instructions per term: each ln(1 + x_i) is then that of fl(1 + x_i),
// off by at most 2^-24 / (1 + x_i) absolute.
template <class Real, bool CORR = true>
struct Log1pSum;
template <bool CORR>
struct Log1pSum<double, CORR> {
    double s = 0.0;
    __device__ __forceinline__ void add(double h, double x) { s += h * log1p_e(x); }
    __device__ __forceinline__ double value() const { return s; }
};
template <>
struct Log1pSum<float, true> {
    float l2 = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float h, float x) {
        const float u = 1.0f + x;
        const float d = u - 1.0f;
        l2 += h * __builtin_amdgcn_logf(u);
        c += h * (x - d);
    }
    __device__ __forceinline__ float value() const { return l2 * 0.693147180559945309f + c; }
};
template <>
struct Log1pSum<float, false> {
    float l2 = 0.0f;
    __device__ __forceinline__ void add(float h, float x) { l2 += h * __builtin_amdgcn_logf(1.0f + x); }
    __device__ __forceinline__ float value() const { return l2 * 0.693147180559945309f; }
};

}  // namespace elbm
