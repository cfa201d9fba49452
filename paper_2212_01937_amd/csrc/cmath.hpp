// cmath.hpp -- precision traits and a minimal complex type for the gfx950 kernels.
//
// The FP32 path uses the hardware transcendental instructions (v_sqrt_f32,
// v_rcp_f32, v_rsq_f32: about 1 ulp) instead of the correctly rounded sequences;
// the FP64 path uses correctly rounded sqrt and Newton-refined reciprocals.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cosmo {

// A coefficient of the lane loops' polynomials.  FP32: the literal itself (an inline
// operand).  FP64: a 64-bit literal is never an inline operand, so the compiler would
// keep every coefficient of a loop body in a pair of vector registers across the loop
// (some seventy of them in the adjoint); the empty asm statement makes the value opaque
// at its use, so it is materialised there into scalar registers (two scalar moves), the
// operand kind an FP64 vector instruction takes directly.
#ifndef COSMO_KC_OPAQUE // (the host build of the tests defines it away)
#define COSMO_KC_OPAQUE(c) asm volatile("" : "+s"(c))
#endif
template <typename T> __device__ __forceinline__ T kc(double v) {
    if constexpr (sizeof(T) == 8) {
        double c = v;
        COSMO_KC_OPAQUE(c);
        return c;
    } else {
        return T(v);
    }
}

template <typename T> struct Fp;

template <> struct Fp<float> {
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float abs(float x) { return __builtin_fabsf(x); }
    static __device__ __forceinline__ float exp(float x) { return expf(x); }
    static __device__ __forceinline__ float log(float x) { return logf(x); }
    static __device__ __forceinline__ float log1p(float x) { return log1pf(x); }
    static __device__ __forceinline__ float log10(float x) { return log10f(x); }
    // log10 through the hardware base-2 logarithm (v_log_f32, about 1 ulp on normal inputs)
    static __device__ __forceinline__ float log10_fast(float x) {
        return __builtin_amdgcn_logf(x) * 0.30102999566398120f;
    }
    // exp through the hardware base-2 exponential (v_exp_f32, about 1 ulp) after the
    // scaling by log2(e), whose rounding adds a relative error of about eps |x|
    static __device__ __forceinline__ float exp_fast(float x) {
        return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
    }
    static __device__ __forceinline__ float atan(float x) { return atanf(x); }
    static __device__ __forceinline__ float nan() { return __builtin_nanf(""); }
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float rint(float x) { return __builtin_rintf(x); }
    // pi/2 in three parts (P1 + P2 + P3 = pi/2 to about 1e-23) and 2/pi, for sincos
    static constexpr float hp1 = 1.5707963705062866f, hp2 = -4.371138828673793e-08f, hp3 = -1.7151245100058819e-15f;
    static constexpr float two_over_pi = 0.6366197723675814f;
    static constexpr int sin_terms = 4, cos_terms = 5; // sin to r^9, cos to r^10
    static __device__ __forceinline__ float inf() { return __builtin_inff(); }
    // Duplication stopping thresholds: iterate while max|A0 - x_i| 4^-m > tau |A_m|.
    // 7th-order tails (R_F, R_C): remainder ~ tau^8 / 4; 5th-order (R_D, R_J): ~ tau^6.
    static constexpr float tau7 = 0.136f;
    static constexpr float tau5 = 0.070f;
    static constexpr float taujx = 0.018f;  // dR_J/dx (rfjx_s): one duplication beyond tau5
    static constexpr float rc_series_max = 0.02f; // |e| below which R_C(1, 1+e) uses its series
    static constexpr int rc_series_terms = 5;
};

template <> struct Fp<double> {
    static __device__ __forceinline__ double sqrt(double x) { return __builtin_sqrt(x); }
    // Reciprocal and reciprocal square root: hardware estimate refined by two Newton
    // steps (error within 2 ulp for the positive normal arguments used here).
    static __device__ __forceinline__ double rcp(double x) {
        double y = __builtin_amdgcn_rcp(x);
        y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
        return __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
    }
    static __device__ __forceinline__ double rsqrt(double x) {
        double y = __builtin_amdgcn_rsq(x);
        double h = 0.5 * x;
        y = y * __builtin_fma(-h * y, y, 1.5);
        return y * __builtin_fma(-h * y, y, 1.5);
    }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double abs(double x) { return __builtin_fabs(x); }
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double log1p(double x) { return ::log1p(x); }
    static __device__ __forceinline__ double log10(double x) { return ::log10(x); }
    // log10 and exp of the lane loops (mu; the closed forms of the curvature transform)
    // with their coefficients through kc (see there): log x = e ln 2 + log m for
    // x = m 2^e, m in [sqrt(1/2), sqrt(2)), with log m = 2 atanh(s), s = (m - 1)/(m + 1),
    // |s| <= 0.172, by its series to s^21 (first omitted term below 1e-18 relative);
    // exp x = 2^k e^r with r = x - k ln 2 (ln 2 in two parts), |r| <= 0.347, by the
    // Taylor series to r^13 (first omitted term below 5e-18).  x = 0 gives -inf, x < 0
    // NaN, as the library functions.
    static __device__ __forceinline__ double log10_fast(double x) {
        double m = __builtin_amdgcn_frexp_mant(x);
        int e = __builtin_amdgcn_frexp_exp(x);
        if (m < 0.70710678118654752) {
            m *= 2.0;
            e -= 1;
        }
        const double s = (m - 1.0) * rcp(m + 1.0), s2 = s * s;
        double p = kc<double>(1.0 / 21.0);
#pragma unroll
        for (int n = 9; n >= 1; --n) p = p * s2 + kc<double>(1.0 / (2 * n + 1));
        const double lm = 2.0 * s * (p * s2 + 1.0);
        const double ln = __builtin_fma((double)e, kc<double>(0.69314718055994529), __builtin_fma((double)e, kc<double>(2.3190468138462996e-17), lm));
        double r = ln * kc<double>(0.43429448190325182);
        if (!(x > 0.0)) r = x == 0.0 ? -__builtin_inf() : __builtin_nan("");
        if (x == __builtin_inf()) r = x;
        return r;
    }
    static __device__ __forceinline__ double exp_fast(double x) {
        const double k = __builtin_rint(x * kc<double>(1.4426950408889634));
        const double r = __builtin_fma(-k, kc<double>(2.3190468138462996e-17), __builtin_fma(-k, kc<double>(0.69314718055994529), x));
        double c[14];
        c[0] = 1.0;
#pragma unroll
        for (int n = 1; n <= 13; ++n) c[n] = c[n - 1] / n;
        double p = kc<double>(c[13]);
#pragma unroll
        for (int n = 12; n >= 2; --n) p = p * r + kc<double>(c[n]);
        p = p * r + 1.0;
        p = p * r + 1.0;
        return __builtin_amdgcn_ldexp(p, (int)k);
    }
    static __device__ __forceinline__ double atan(double x) { return ::atan(x); }
    static __device__ __forceinline__ double nan() { return __builtin_nan(""); }
    static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double rint(double x) { return __builtin_rint(x); }
    static constexpr double hp1 = 1.5707963267948966, hp2 = 6.123233995736766e-17, hp3 = -1.4973849048591698e-33;
    static constexpr double two_over_pi = 0.6366197723675814;
    static constexpr int sin_terms = 8, cos_terms = 8; // sin to r^17, cos to r^16
    static __device__ __forceinline__ double inf() { return __builtin_inf(); }
    static constexpr double tau7 = 0.0121;
    static constexpr double tau5 = 0.0028;
    static constexpr double taujx = 0.0007;
    static constexpr double rc_series_max = 0.01;
    static constexpr int rc_series_terms = 9;
};

// sin x and cos x together, for |x| < 2^16 (NaN beyond; the curvature transform's
// arguments sqrt|Ok| chi stay within a few pi).  Cody-Waite reduction: k = rint(2x/pi),
// r = x - k pi/2 with pi/2 in three parts (each step one FMA), so |r| <= pi/4 up to the
// rounding of k; then the Taylor polynomials of sin r and cos r, truncated where the
// first omitted term at |r| = pi/4 is below the type's rounding (FP32: 2e-9 for sin to
// r^9, 1e-10 for cos to r^10; FP64: 1e-19, 2e-18), and the quadrant k mod 4.  No
// large-argument reduction (its tables would sit in registers across the lane loops).
template <typename T> __device__ __forceinline__ void sincos_red(T x, T &s, T &c) {
    const T k = Fp<T>::rint(x * Fp<T>::two_over_pi);
    T r = Fp<T>::fma(-k, Fp<T>::hp1, x);
    r = Fp<T>::fma(-k, Fp<T>::hp2, r);
    r = Fp<T>::fma(-k, Fp<T>::hp3, r);
    const T r2 = r * r;
    // Horner from the top: sin r = r (1 - r^2/3! + r^4/5! - ...), cos r = 1 - r^2/2! + ...
    double fs[Fp<T>::sin_terms + 1], fc[Fp<T>::cos_terms + 1];
    fs[0] = 1.0; fc[0] = 1.0;
#pragma unroll
    for (int n = 1; n <= Fp<T>::sin_terms; ++n) fs[n] = -fs[n - 1] / double((2 * n) * (2 * n + 1));
#pragma unroll
    for (int n = 1; n <= Fp<T>::cos_terms; ++n) fc[n] = -fc[n - 1] / double((2 * n - 1) * (2 * n));
    T ps = kc<T>(fs[Fp<T>::sin_terms]), pc = kc<T>(fc[Fp<T>::cos_terms]);
#pragma unroll
    for (int n = Fp<T>::sin_terms - 1; n >= 0; --n) ps = ps * r2 + (n == 0 ? T(1) : kc<T>(fs[n]));
#pragma unroll
    for (int n = Fp<T>::cos_terms - 1; n >= 0; --n) pc = pc * r2 + (n == 0 ? T(1) : kc<T>(fc[n]));
    const T sr = r * ps, cr = pc;
    const int q = (int)k & 3;
    const T sa = (q & 1) ? cr : sr, ca = (q & 1) ? sr : cr;
    s = (q & 2) ? -sa : sa;
    c = ((q + 1) & 2) ? -ca : ca;
    if (!(Fp<T>::abs(x) < T(65536))) s = c = Fp<T>::nan();
}

template <typename T> struct cx {
    T re, im;
};

template <typename T> __device__ __forceinline__ cx<T> mkc(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {s * a.re, s * a.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, T s) { return {a.re + s, a.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, T s) { return {a.re - s, a.im}; }
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T> __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __device__ __forceinline__ T cabs(cx<T> a) { return Fp<T>::sqrt(norm2(a)); }
template <typename T> __device__ __forceinline__ cx<T> crcp(cx<T> a) {
    T s = Fp<T>::rcp(norm2(a));
    return {a.re * s, -a.im * s};
}
template <typename T> __device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) { return a * crcp(b); }

// Principal square root; also returns |w| (= |sqrt(w)|^2), which callers reuse.
// With t = (|w| + |Re w|)/2 and q = 1/sqrt(t), the larger component of sqrt(w)
// is t q and the smaller |Im w| q / 2 (no cancellation on either half-plane).
template <typename T> __device__ __forceinline__ cx<T> csqrt(cx<T> w, T &absw) {
    T r = cabs(w);
    absw = r;
    bool pos = w.re >= T(0);
    T t = T(0.5) * (r + Fp<T>::abs(w.re));
    T q = (t > T(0)) ? Fp<T>::rsqrt(t) : T(0);
    T big = t * q, small = T(0.5) * Fp<T>::abs(w.im) * q;
    cx<T> res;
    res.re = pos ? big : small;
    res.im = pos ? (w.im >= T(0) ? small : -small) : (w.im >= T(0) ? big : -big);
    return res;
}
// As csqrt, with |w| and 1/|w| from one reciprocal square root of |w|^2.
template <typename T> __device__ __forceinline__ cx<T> csqrt_inv(cx<T> w, T &absw, T &iabsw) {
    const T n = norm2(w);
    const T ir = Fp<T>::rsqrt(n);
    const T r = n * ir;
    absw = r;
    iabsw = ir;
    bool pos = w.re >= T(0);
    T t = T(0.5) * (r + Fp<T>::abs(w.re));
    T q = (t > T(0)) ? Fp<T>::rsqrt(t) : T(0);
    T big = t * q, small = T(0.5) * Fp<T>::abs(w.im) * q;
    cx<T> res;
    res.re = pos ? big : small;
    res.im = pos ? (w.im >= T(0) ? small : -small) : (w.im >= T(0) ? big : -big);
    return res;
}
// As csqrt_inv for w = wre + i wim with a non-zero imaginary part that is the same
// on every lane: wim^2, |wim|/2 and sign(wim) come precomputed.  With wim != 0,
// |w| > |wre| and the half-sum t below is positive.
template <typename T>
__device__ __forceinline__ cx<T> csqrt_uim_inv(T wre, T wim2, T hwim, T swim, T &absw, T &iabsw) {
    const T n = wre * wre + wim2;
    const T ir = Fp<T>::rsqrt(n);
    const T r = n * ir;
    absw = r;
    iabsw = ir;
    const T t = T(0.5) * (r + Fp<T>::abs(wre));
    const T q = Fp<T>::rsqrt(t);
    const T big = t * q, small = hwim * q;
    const bool pos = wre >= T(0);
    return mkc(pos ? big : small, swim * (pos ? small : big));
}
template <typename T> __device__ __forceinline__ cx<T> csqrt(cx<T> w) {
    T r;
    return csqrt(w, r);
}

// Real part of the principal square root and |w| only (one sqrt, one rsqrt).
template <typename T> __device__ __forceinline__ T csqrt_re(T wre, T wim, T &absw) {
    T r = Fp<T>::sqrt(wre * wre + wim * wim);
    absw = r;
    T t = T(0.5) * (r + Fp<T>::abs(wre));
    T q = (t > T(0)) ? Fp<T>::rsqrt(t) : T(0);
    return (wre >= T(0) ? t : T(0.5) * Fp<T>::abs(wim)) * q;
}

template <typename T> __device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }

} // namespace cosmo
