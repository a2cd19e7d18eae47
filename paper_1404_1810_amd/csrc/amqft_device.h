// Device-side building blocks of the AM-QFT kernels for gfx950.
//
// Complex values are held as (re, im) pairs of the arithmetic type R (float
// or double); the recursion of the paper has only real coefficients, so the
// real and imaginary parts of a complex signal run through it in lockstep:
// the same additions and multiplications per point as the paper's two real
// passes (Sec. 3.1, decomposition D_c).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace amqft {

// ---------------------------------------------------------------------------
// 32-bit fixed point (Sec. 7.2: the halvings are binary translations; Sec.
// 7.4: fixed-point implementations).  A value is an int32 in units of the
// input's last bit; a constant f (|f| < 4) is round(f 2^29), ties away from
// zero (Q2.29: the 2cos / 2sin families, cos(pi/4), the +-1 weights and the
// halving 1/2).  Sums wrap modulo 2^32 and are exact otherwise; a product
// a * k is round(a k / 2^29) to nearest, ties away from zero (the binary
// translation of the 64-bit product's magnitude, sign restored), so that
// a * (1/2) is the rounded halving and rounding commutes with negation: the
// kernels may carry a value negated or multiplied by -i (the transposed
// combine does) without changing any rounding.  Every product of the
// transform has a constant as one factor, so the operator needs no notion of
// which operand is data.  With exact sums the result depends only on which
// values are rounded, not on the order in which the sums are formed.
// ---------------------------------------------------------------------------
struct fx32 {
    int v;
    fx32() = default;
    __host__ __device__ constexpr explicit fx32(double f)
        : v((int)(f * 536870912.0 + (f < 0 ? -0.5 : 0.5))) {}
    static __host__ __device__ constexpr fx32 raw(int x) {
        fx32 r(0.0);
        r.v = x;
        return r;
    }
};
__device__ __forceinline__ fx32 operator+(fx32 a, fx32 b) { return fx32::raw((int)((unsigned)a.v + (unsigned)b.v)); }
__device__ __forceinline__ fx32 operator-(fx32 a, fx32 b) { return fx32::raw((int)((unsigned)a.v - (unsigned)b.v)); }
__device__ __forceinline__ fx32 operator-(fx32 a) { return fx32::raw((int)(0u - (unsigned)a.v)); }
// round(a k / 2^29) with ties away from zero = floor((a k + 2^28 - [a k < 0]) / 2^29):
// one 64-bit multiply-add and a funnel shift
__device__ __forceinline__ fx32 operator*(fx32 a, fx32 k) {
    const long long bias = (1ll << 28) + ((a.v ^ k.v) >> 31);
    return fx32::raw((int)(unsigned)(((long long)a.v * k.v + bias) >> 29));
}

// aligned to its full size, so that LDS and global accesses of one complex
// value are single 64-bit (FP32) or 128-bit (FP64) transactions
template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};

// whole-value loads and stores of a complex number (one 64-bit / 128-bit
// access; keeps the compiler from splitting it into two scalar accesses)
template <typename R> struct vec2;
template <> struct vec2<float> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct vec2<double> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct vec2<fx32> { typedef int T __attribute__((ext_vector_type(2))); };
template <typename R>
__device__ __forceinline__ cx<R> ldc(const cx<R>* p) {
    const typename vec2<R>::T v = *reinterpret_cast<const typename vec2<R>::T*>(p);
    return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void stc(cx<R>* p, cx<R> a) {
    typename vec2<R>::T v;
    v.x = a.re;
    v.y = a.im;
    *reinterpret_cast<typename vec2<R>::T*>(p) = v;
}

__device__ __forceinline__ cx<fx32> ldc(const cx<fx32>* p) {
    const vec2<fx32>::T v = *reinterpret_cast<const vec2<fx32>::T*>(p);
    return {fx32::raw(v.x), fx32::raw(v.y)};
}
__device__ __forceinline__ void stc(cx<fx32>* p, cx<fx32> a) {
    vec2<fx32>::T v;
    v.x = a.re.v;
    v.y = a.im.v;
    *reinterpret_cast<vec2<fx32>::T*>(p) = v;
}

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, R k) { return {a.re * k, a.im * k}; }
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) { return {a.re, -a.im}; }

// cos(pi/4) = sin(pi/4): the single constant of the L = 8 base cases of
// dct_oo / dst_oo (Sec. 7.1).
// Accesses of the in-place large-N path to the signal buffer, which it
// rewrites in the positions it read (the CPU emulation of the kernels checks
// that no workgroup touches a position that another workgroup of the same
// launch writes).
template <typename R>
__device__ __forceinline__ cx<R> xld(const cx<R>* p) {
    const cx<R> v = *p;  // in-place signal read
    return v;
}
template <typename R>
__device__ __forceinline__ void xst(cx<R>* p, cx<R> v) {
    *p = v;  // in-place signal write
}

template <typename R> __device__ __forceinline__ R cos_pi_4();
template <> __device__ __forceinline__ float cos_pi_4<float>() { return 0.70710678118654752440f; }
template <> __device__ __forceinline__ double cos_pi_4<double>() { return 0.70710678118654752440; }
template <> __device__ __forceinline__ fx32 cos_pi_4<fx32>() { return fx32::raw(379625062); }  // round(2^29 / sqrt 2)

// ---------------------------------------------------------------------------
// storage types: interleaved (re, im) pairs
// ---------------------------------------------------------------------------
struct bf16x2 {
    uint16_t re, im;
};

template <typename S> struct storage;

template <> struct storage<double2> {
    using R = double;
    static __device__ __forceinline__ cx<double> ld(const double2* p) { double2 v = *p; return {v.x, v.y}; }
    static __device__ __forceinline__ void st(double2* p, cx<double> v) { *p = make_double2(v.re, v.im); }
};
template <> struct storage<float2> {
    using R = float;
    static __device__ __forceinline__ cx<float> ld(const float2* p) { float2 v = *p; return {v.x, v.y}; }
    static __device__ __forceinline__ void st(float2* p, cx<float> v) { *p = make_float2(v.re, v.im); }
};
template <> struct storage<__half2> {
    using R = float;
    static __device__ __forceinline__ cx<float> ld(const __half2* p) {
        float2 v = __half22float2(*p);
        return {v.x, v.y};
    }
    static __device__ __forceinline__ void st(__half2* p, cx<float> v) {
        *p = __float22half2_rn(make_float2(v.re, v.im));
    }
};
// bfloat16 = the upper 16 bits of an IEEE binary32; stores round to nearest,
// ties to even; NaN stays NaN.
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
template <> struct storage<bf16x2> {
    using R = float;
    static __device__ __forceinline__ cx<float> ld(const bf16x2* p) {
        bf16x2 v = *p;
        return {bf16_to_f32(v.re), bf16_to_f32(v.im)};
    }
    static __device__ __forceinline__ void st(bf16x2* p, cx<float> v) {
        bf16x2 o;
        o.re = f32_to_bf16(v.re);
        o.im = f32_to_bf16(v.im);
        *p = o;
    }
};

// complex 32-bit fixed point: (re, im) int32 pairs
template <> struct storage<int2> {
    using R = fx32;
    static __device__ __forceinline__ cx<fx32> ld(const int2* p) { int2 v = *p; return {fx32::raw(v.x), fx32::raw(v.y)}; }
    static __device__ __forceinline__ void st(int2* p, cx<fx32> v) { *p = make_int2(v.re.v, v.im.v); }
};

// ---------------------------------------------------------------------------
// variant traits (Sec. 6 and the general notes at its end)
// ---------------------------------------------------------------------------
template <int V>
struct variant_traits {
    // skeleton A (time indices split first: dct_ot/dst_ot) or B (harmonics
    // first: dct_to/dst_to)
    static constexpr bool skel_a = (V == 1 || V == 4 || V == 5 || V == 8);
    // M5..M8 turn a DCT mother into a DST child and vice versa
    static constexpr bool switches = V >= 5;
    // M1, M3, M5, M7 contain a sequential recurrence (with one halving)
    static constexpr bool recurrence = (V == 1 || V == 3 || V == 5 || V == 7);
    // coefficient of the previous term in that recurrence
    static constexpr int sign = (V == 1 || V == 3) ? -1 : 1;
};

// Constant-table family per variant (Sec. 7.1): 0 = 2cos, 1 = 1/(2cos),
// 2 = 2sin, 3 = 1/(2sin).
__host__ __device__ constexpr int const_family(int v) {
    return (v == 1 || v == 3) ? 0 : (v == 2 || v == 4) ? 1 : (v == 5 || v == 7) ? 2 : 3;
}

}  // namespace amqft
