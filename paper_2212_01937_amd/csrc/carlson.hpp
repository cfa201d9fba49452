// carlson.hpp -- Carlson symmetric elliptic integrals R_F, R_D, R_J, R_C
// (definitions: sec. 2.2, eqs. 2.6-2.9) by the duplication method the paper
// relies on ([10] in sec. 2.2): repeated application of the duplication
// theorem x -> (x + lambda)/4, lambda = sqrt(x)sqrt(y) + sqrt(x)sqrt(z) +
// sqrt(y)sqrt(z), until every argument is within a relative distance tau of
// the mean A_m, then a Taylor expansion about A_m in the symmetric functions of
// the normalised deviations X_i = (A_0 - x_i) 4^-m / A_m (taken from the
// initial arguments, which avoids the rounding of the iterated ones).  The
// expansions used are the seventh-order one for R_F and R_C and the
// fifth-order one for R_D and R_J (DLMF 19.36.1-2); where a structured routine
// needs R_D next to R_F from one sequence, the R_D tails are the derivatives of
// the R_F expansion (rfd_tails).
//
// Two families:
//  * general complex (rf_c, rd_c, rj_c, rc_c) -- the C-ABI carlson_* entry points;
//  * "structured" real-result versions for the distance kernels, whose argument
//    triples are always (real, real, real) or (real, w, conj(w)).  A triple is
//    passed as (x, a, b): x real; PAIR -> y = a + i b, z = a - i b; otherwise
//    y = a, z = b.  Duplication maps each structure onto itself (lambda is real),
//    so every iterate stays real or a conjugate pair.
#pragma once

#include "cmath.hpp"

namespace cosmo {

// ---------------------------------------------------------------- tails
template <typename T> __device__ __forceinline__ T rf_tail(T E2, T E3) {
    // 1 - E2/10 + E3/14 + E2^2/24 - 3E2E3/44 - 5E2^3/208 + 3E3^2/104 + E2^2E3/16
    return T(1) + E2 * (kc<T>(-0.1) + E2 * (kc<T>(1.0 / 24.0) - kc<T>(5.0 / 208.0) * E2)) +
           E3 * (kc<T>(1.0 / 14.0) + kc<T>(3.0 / 104.0) * E3 - kc<T>(3.0 / 44.0) * E2 + kc<T>(1.0 / 16.0) * E2 * E2);
}
template <typename T> __device__ __forceinline__ cx<T> rf_tail(cx<T> E2, cx<T> E3) {
    cx<T> a = (E2 * T(-5.0 / 208.0)) + T(1.0 / 24.0);
    cx<T> b = (E2 * a) + T(-0.1);
    cx<T> c = (E3 * T(3.0 / 104.0)) - (E2 * T(3.0 / 44.0)) + (E2 * E2 * T(1.0 / 16.0)) + T(1.0 / 14.0);
    return (E2 * b) + (E3 * c) + T(1);
}
// Partial derivatives of rf_tail in E2 and E3.
template <typename T> __device__ __forceinline__ void rf_tail_grad(T E2, T E3, T &t2, T &t3) {
    t2 = kc<T>(-0.1) + E2 * (kc<T>(1.0 / 12.0) - kc<T>(15.0 / 208.0) * E2) + E3 * (kc<T>(-3.0 / 44.0) + kc<T>(0.125) * E2);
    t3 = kc<T>(1.0 / 14.0) + kc<T>(3.0 / 52.0) * E3 + E2 * (kc<T>(-3.0 / 44.0) + kc<T>(1.0 / 16.0) * E2);
}
// 1 - 3E2/14 + E3/6 + 9E2^2/88 - 3E4/22 - 9E2E3/52 + 3E5/26
template <typename T> __device__ __forceinline__ T rj_tail(T E2, T E3, T E4, T E5) {
    return T(1) + E2 * (T(-3.0 / 14.0) + T(9.0 / 88.0) * E2 - T(9.0 / 52.0) * E3) + T(1.0 / 6.0) * E3 -
           T(3.0 / 22.0) * E4 + T(3.0 / 26.0) * E5;
}
template <typename T> __device__ __forceinline__ cx<T> rj_tail(cx<T> E2, cx<T> E3, cx<T> E4, cx<T> E5) {
    cx<T> a = (E2 * T(9.0 / 88.0)) - (E3 * T(9.0 / 52.0)) + T(-3.0 / 14.0);
    return (E2 * a) + (E3 * T(1.0 / 6.0)) - (E4 * T(3.0 / 22.0)) + (E5 * T(3.0 / 26.0)) + T(1);
}
// 1 + 3s^2/10 + s^3/7 + 3s^4/8 + 9s^5/22 + 159s^6/208 + 9s^7/8
template <typename T> __device__ __forceinline__ T rc_tail(T s) {
    return T(1) + s * s * (T(0.3) + s * (T(1.0 / 7.0) + s * (T(0.375) + s * (T(9.0 / 22.0) +
                          s * (T(159.0 / 208.0) + s * T(1.125))))));
}
// d rc_tail / ds
template <typename T> __device__ __forceinline__ T rc_tail_d(T s) {
    return s * (T(0.6) + s * (T(3.0 / 7.0) + s * (T(1.5) + s * (T(45.0 / 22.0) +
                s * (T(954.0 / 208.0) + s * T(63.0 / 8.0))))));
}
template <typename T> __device__ __forceinline__ cx<T> rc_tail(cx<T> s) {
    cx<T> p = (s * T(1.125)) + T(159.0 / 208.0);
    p = (s * p) + T(9.0 / 22.0);
    p = (s * p) + T(0.375);
    p = (s * p) + T(1.0 / 7.0);
    p = (s * p) + T(0.3);
    return (s * s * p) + T(1);
}

constexpr int kMaxDup = 64; // iteration cap: guarantees termination on NaN/degenerate input

// ---------------------------------------------------------------- general complex
template <typename T> __device__ cx<T> rf_c(cx<T> x, cx<T> y, cx<T> z) {
    const T third = T(1.0 / 3.0);
    cx<T> A0 = (x + y + z) * third;
    cx<T> dx = A0 - x, dy = A0 - y;
    T Q = tmax(tmax(cabs(dx), cabs(dy)), cabs(A0 - z));
    cx<T> A = A0;
    T f = T(1);
    for (int m = 0; m < kMaxDup && Q * f > Fp<T>::tau7 * cabs(A); ++m) {
        cx<T> sx = csqrt(x), sy = csqrt(y), sz = csqrt(z);
        cx<T> lam = sx * sy + sx * sz + sy * sz;
        x = (x + lam) * T(0.25);
        y = (y + lam) * T(0.25);
        z = (z + lam) * T(0.25);
        A = (A + lam) * T(0.25);
        f *= T(0.25);
    }
    cx<T> g = crcp(A) * f;
    cx<T> X = dx * g, Y = dy * g;
    cx<T> Z = -(X + Y);
    cx<T> E2 = X * Y - Z * Z, E3 = X * Y * Z;
    return rf_tail(E2, E3) * crcp(csqrt(A));
}

template <typename T> __device__ cx<T> rd_c(cx<T> x, cx<T> y, cx<T> z) {
    cx<T> A0 = (x + y + z * T(3)) * T(0.2);
    cx<T> dx = A0 - x, dy = A0 - y;
    T Q = tmax(tmax(cabs(dx), cabs(dy)), cabs(A0 - z));
    cx<T> A = A0, acc = mkc(T(0), T(0));
    T f = T(1);
    for (int m = 0; m < kMaxDup && Q * f > Fp<T>::tau5 * cabs(A); ++m) {
        cx<T> sx = csqrt(x), sy = csqrt(y), sz = csqrt(z);
        cx<T> lam = sx * sy + sx * sz + sy * sz;
        acc = acc + crcp(sz * (z + lam)) * f;
        x = (x + lam) * T(0.25);
        y = (y + lam) * T(0.25);
        z = (z + lam) * T(0.25);
        A = (A + lam) * T(0.25);
        f *= T(0.25);
    }
    cx<T> g = crcp(A) * f;
    cx<T> X = dx * g, Y = dy * g;
    cx<T> Z = (X + Y) * T(-1.0 / 3.0);
    cx<T> XY = X * Y, Z2 = Z * Z;
    cx<T> E2 = XY - Z2 * T(6), E3 = (XY * T(3) - Z2 * T(8)) * Z;
    cx<T> E4 = (XY - Z2) * Z2 * T(3), E5 = XY * Z2 * Z;
    return rj_tail(E2, E3, E4, E5) * crcp(A * csqrt(A)) * f + acc * T(3);
}

template <typename T> __device__ cx<T> rc_c(cx<T> x, cx<T> y) {
    T scale = T(1);
    if (y.im == T(0) && y.re < T(0) && x.im == T(0) && x.re >= T(0)) {
        // Cauchy principal value: R_C(x, y) = sqrt(x/(x-y)) R_C(x - y, -y)  (DLMF 19.2.20)
        scale = Fp<T>::sqrt(Fp<T>::div(x.re, x.re - y.re));
        x = x - y;
        y = -y;
    }
    cx<T> A0 = (x + y * T(2)) * T(1.0 / 3.0);
    cx<T> dy = y - A0;
    T Q = cabs(A0 - x);
    cx<T> A = A0;
    T f = T(1);
    for (int m = 0; m < kMaxDup && Q * f > Fp<T>::tau7 * cabs(A); ++m) {
        cx<T> lam = csqrt(x) * csqrt(y) * T(2) + y;
        x = (x + lam) * T(0.25);
        y = (y + lam) * T(0.25);
        A = (A + lam) * T(0.25);
        f *= T(0.25);
    }
    cx<T> s = dy * crcp(A) * f;
    return rc_tail(s) * crcp(csqrt(A)) * scale;
}

// R_C(1, 1 + e): series sum_n (-e)^n / (2n+1) for small |e|, else by duplication.
template <typename T> __device__ __forceinline__ cx<T> rc1_c(cx<T> e) {
    if (cabs(e) < Fp<T>::rc_series_max) {
        cx<T> s = mkc(T(0), T(0)), t = mkc(T(1), T(0));
        for (int n = 0; n < Fp<T>::rc_series_terms; ++n) {
            s = s + t * T(1.0 / (2 * n + 1));
            t = t * (-e);
        }
        return s;
    }
    return rc_c(mkc(T(1), T(0)), e + T(1));
}

template <typename T> __device__ cx<T> rj_c(cx<T> x, cx<T> y, cx<T> z, cx<T> p) {
    cx<T> A0 = (x + y + z + p * T(2)) * T(0.2);
    cx<T> dx = A0 - x, dy = A0 - y, dz = A0 - z, dp = A0 - p;
    T Q = tmax(tmax(cabs(dx), cabs(dy)), tmax(cabs(dz), cabs(dp)));
    cx<T> delta = (p - x) * (p - y) * (p - z);
    cx<T> A = A0, acc = mkc(T(0), T(0));
    T f = T(1);
    for (int m = 0; m < kMaxDup && Q * f > Fp<T>::tau5 * cabs(A); ++m) {
        cx<T> sx = csqrt(x), sy = csqrt(y), sz = csqrt(z), sp = csqrt(p);
        cx<T> lam = sx * sy + sx * sz + sy * sz;
        cx<T> d = (sp + sx) * (sp + sy) * (sp + sz);
        cx<T> e = delta * crcp(d * d) * (f * f * f);
        acc = acc + rc1_c(e) * crcp(d) * f;
        x = (x + lam) * T(0.25);
        y = (y + lam) * T(0.25);
        z = (z + lam) * T(0.25);
        p = (p + lam) * T(0.25);
        A = (A + lam) * T(0.25);
        f *= T(0.25);
    }
    cx<T> g = crcp(A) * f;
    cx<T> X = dx * g, Y = dy * g, Z = dz * g, P = dp * g;
    cx<T> xyz = X * Y * Z, P2 = P * P;
    cx<T> E2 = X * Y + X * Z + Y * Z - P2 * T(3);
    cx<T> E3 = xyz + E2 * P * T(2) + P2 * P * T(4);
    cx<T> E4 = (xyz * T(2) + E2 * P + P2 * P * T(3)) * P;
    cx<T> E5 = xyz * P2;
    return rj_tail(E2, E3, E4, E5) * crcp(A * csqrt(A)) * f + acc * T(6);
}

// ---------------------------------------------------------------- real R_C
// Real arguments x >= 0, y != 0 (principal value for y < 0).
template <typename T> __device__ T rc_r(T x, T y) {
    T scale = T(1);
    if (y < T(0)) {
        scale = Fp<T>::sqrt(Fp<T>::div(x, x - y));
        x = x - y;
        y = -y;
    }
    T A0 = (x + T(2) * y) * T(1.0 / 3.0);
    T dy = y - A0;
    T Q = Fp<T>::abs(A0 - x);
    T A = A0, f = T(1);
    for (int m = 0; m < kMaxDup && Q * f > Fp<T>::tau7 * Fp<T>::abs(A); ++m) {
        T lam = T(2) * Fp<T>::sqrt(x) * Fp<T>::sqrt(y) + y;
        x = (x + lam) * T(0.25);
        y = (y + lam) * T(0.25);
        A = (A + lam) * T(0.25);
        f *= T(0.25);
    }
    T s = dy * f * Fp<T>::rcp(A);
    return rc_tail(s) * Fp<T>::rsqrt(A) * scale;
}

template <typename T> __device__ __forceinline__ T rc1_r(T e) {
    if (Fp<T>::abs(e) < Fp<T>::rc_series_max) {
        T s = T(0), t = T(1);
#pragma unroll
        for (int n = 0; n < Fp<T>::rc_series_terms; ++n) {
            s += t * T(1.0 / (2 * n + 1));
            t *= -e;
        }
        return s;
    }
    return rc_r(T(1), T(1) + e);
}

// d R_C(1, 1 + e) / de: the derivative of the series above for small |e|, else the
// identity f'(e) = (1/(1 + e) - f(e)) / (2e) of f(e) = arctan(sqrt e)/sqrt e.
template <typename T> __device__ __forceinline__ T rc1_dr(T e, T f) {
    if (Fp<T>::abs(e) < Fp<T>::rc_series_max) {
        T s = T(0), t = T(-1);
#pragma unroll
        for (int n = 1; n < Fp<T>::rc_series_terms; ++n) {
            s += t * T(double(n) / (2 * n + 1));
            t *= -e;
        }
        return s;
    }
    return (Fp<T>::rcp(T(1) + e) - f) * Fp<T>::rcp(T(2) * e);
}

// ---------------------------------------------------------------- structured
// One duplication step on a structured triple; returns lambda.  For PAIR also
// returns Re sqrt(y) and |y| (reused by R_J's d_m).
template <typename T, bool PAIR>
__device__ __forceinline__ T dup_lambda(T x, T a, T b, T &sx, T &sy_re, T &sy_abs2, T &sz) {
    sx = Fp<T>::sqrt(x);
    if (PAIR) {
        T r;
        sy_re = csqrt_re(a, b, r);
        sy_abs2 = r;
        sz = T(0);
        return sx * (T(2) * sy_re) + r;
    } else {
        sy_re = Fp<T>::sqrt(a);
        sz = Fp<T>::sqrt(b);
        sy_abs2 = T(0);
        return sx * (sy_re + sz) + sy_re * sz;
    }
}

template <typename T, bool PAIR> __device__ __forceinline__ T mean3(T x, T a, T b) {
    return PAIR ? (x + T(2) * a) * T(1.0 / 3.0) : (x + a + b) * T(1.0 / 3.0);
}

// Spread of a structured triple about A0, in the measure the duplication tests
// compare: max_i |A0 - x_i| (not PAIR), or its square (PAIR: no square root).
template <typename T, bool PAIR> __device__ __forceinline__ T spread3(T A0, T x, T a, T b) {
    if (PAIR) {
        T dx = A0 - x, da = A0 - a;
        return tmax(dx * dx, da * da + b * b);
    }
    return tmax(tmax(Fp<T>::abs(A0 - x), Fp<T>::abs(A0 - a)), Fp<T>::abs(A0 - b));
}
// |d| in the same measure
template <typename T, bool PAIR> __device__ __forceinline__ T spread1(T d) { return PAIR ? d * d : Fp<T>::abs(d); }
// Duplication test: is the spread Q of the initial arguments, scaled by f = 4^-m,
// still above tau |A| (A the current mean)?
template <typename T, bool PAIR> __device__ __forceinline__ bool spread_above(T Q, T f, T tau, T A) {
    return PAIR ? Q * (f * f) > (tau * tau) * (A * A) : Q * f > tau * Fp<T>::abs(A);
}

// Symmetric functions of the deviations of (y, z) about A0, scaled by g:
// s = Y + Z and q = Y Z.
template <typename T, bool PAIR>
__device__ __forceinline__ void yz_sym(T A0, T a, T b, T g, T &s, T &q) {
    if (PAIR) {
        T u = (A0 - a) * g, v = b * g;
        s = T(2) * u;
        q = u * u + v * v;
    } else {
        T Y = (A0 - a) * g, Z = (A0 - b) * g;
        s = Y + Z;
        q = Y * Z;
    }
}

// FP32 lanes rarely duplicate at all (the expansion is accurate to the FP32 rounding
// level from the tau7 deviation down), and neighbouring redshifts agree on it: a wave
// none of whose lanes needs a step evaluates the tail at m = 0 directly, without the
// sequence's bookkeeping (f = 1, the mean A = A0, no accumulated terms).
template <typename T, bool PAIR> __device__ __forceinline__ bool wave_no_dup(T Q, T A0) {
    return sizeof(T) == 4 && __ballot(spread_above<T, PAIR>(Q, T(1), Fp<T>::tau7, A0)) == 0;
}

template <typename T, bool PAIR> __device__ T rf_s(T x, T a, T b) {
    const T A0 = mean3<T, PAIR>(x, a, b);
    const T x0 = x, a0 = a, b0 = b;
    const T Q = spread3<T, PAIR>(A0, x, a, b);
    if (wave_no_dup<T, PAIR>(Q, A0)) {
        const T ra = Fp<T>::rsqrt(A0), g = ra * ra;
        T s, q;
        const T X = (A0 - x0) * g;
        yz_sym<T, PAIR>(A0, a0, b0, g, s, q);
        return rf_tail(q - X * X, X * q) * ra;
    }
    T A = A0, f = T(1);
    for (int m = 0; m < kMaxDup && spread_above<T, PAIR>(Q, f, Fp<T>::tau7, A); ++m) {
        T sx, syr, sya, sz;
        T lam = dup_lambda<T, PAIR>(x, a, b, sx, syr, sya, sz);
        x = (x + lam) * T(0.25);
        a = (a + lam) * T(0.25);
        b = PAIR ? b * T(0.25) : (b + lam) * T(0.25);
        A = (A + lam) * T(0.25);
        f *= T(0.25);
    }
    const T ra = Fp<T>::rsqrt(A); // 1/A = ra^2 (A > 0 on the structured triples)
    T g = f * (ra * ra);
    T X = (A0 - x0) * g, s, q;
    yz_sym<T, PAIR>(A0, a0, b0, g, s, q);
    // with X + s = 0: E2 = XY + XZ + YZ = q - X^2, E3 = XYZ = X q
    return rf_tail(q - X * X, X * q) * ra;
}

// R_F(x, y, z) and R_J(x, y, z, p) from one shared duplication sequence
// (p real > 0; p <= 0 would need the principal-value transformation and yields NaN).
template <typename T, bool PAIR>
__device__ void rfj_s(T x, T a, T b, T p, T &rf, T &rj) {
    const T AF0 = mean3<T, PAIR>(x, a, b);
    const T AJ0 = (T(3) * AF0 + T(2) * p) * T(0.2);
    const T x0 = x, a0 = a, b0 = b, p0 = p;
    const T QF = spread3<T, PAIR>(AF0, x, a, b);
    const T QJ = tmax(spread3<T, PAIR>(AJ0, x, a, b), spread1<T, PAIR>(AJ0 - p));
    T delta = PAIR ? (p - x) * ((p - a) * (p - a) + b * b) : (p - x) * (p - a) * (p - b);
    T AF = AF0, AJ = AJ0, f = T(1), acc = T(0);
    for (int m = 0; m < kMaxDup && (spread_above<T, PAIR>(QF, f, Fp<T>::tau7, AF) ||
                                   spread_above<T, PAIR>(QJ, f, Fp<T>::tau5, AJ)); ++m) {
        T sx, syr, sya, sz;
        T lam = dup_lambda<T, PAIR>(x, a, b, sx, syr, sya, sz);
        T sp = Fp<T>::sqrt(p);
        T d = (sp + sx) * (PAIR ? p + T(2) * sp * syr + sya : (sp + syr) * (sp + sz));
        T rd = Fp<T>::rcp(d);
        T e = delta * rd * rd * (f * f * f);
        acc += f * rc1_r(e) * rd;
        x = (x + lam) * T(0.25);
        a = (a + lam) * T(0.25);
        b = PAIR ? b * T(0.25) : (b + lam) * T(0.25);
        p = (p + lam) * T(0.25);
        AF = (AF + lam) * T(0.25);
        AJ = (AJ + lam) * T(0.25);
        f *= T(0.25);
    }
    {
        const T ra = Fp<T>::rsqrt(AF);
        T g = f * (ra * ra);
        T X = (AF0 - x0) * g, s, q;
        yz_sym<T, PAIR>(AF0, a0, b0, g, s, q);
        rf = rf_tail(q - X * X, X * q) * ra;
    }
    {
        const T rj_a = Fp<T>::rsqrt(AJ);
        T g = f * (rj_a * rj_a);
        T X = (AJ0 - x0) * g, s, q;
        yz_sym<T, PAIR>(AJ0, a0, b0, g, s, q);
        T P = (AJ0 - p0) * g;
        T sym2 = X * s + q, xyz = X * q, P2 = P * P;
        T E2 = sym2 - T(3) * P2;
        T E3 = xyz + T(2) * E2 * P + T(4) * P2 * P;
        T E4 = (T(2) * xyz + E2 * P + T(3) * P2 * P) * P;
        T E5 = xyz * P2;
        rj = rj_tail(E2, E3, E4, E5) * g * rj_a + T(6) * acc;
    }
    if (!(p0 > T(0))) rj = Fp<T>::nan();
}

// R_D(y, z, x): the real member x of the triple is the last argument.
template <typename T, bool PAIR> __device__ T rd_last_x(T x, T a, T b) {
    const T A0 = PAIR ? (T(2) * a + T(3) * x) * T(0.2) : (a + b + T(3) * x) * T(0.2);
    const T a0 = a, b0 = b;
    const T Q = spread3<T, PAIR>(A0, x, a, b);
    T A = A0, f = T(1), acc = T(0);
    for (int m = 0; m < kMaxDup && spread_above<T, PAIR>(Q, f, Fp<T>::tau5, A); ++m) {
        T sx, syr, sya, sz;
        T lam = dup_lambda<T, PAIR>(x, a, b, sx, syr, sya, sz);
        acc += f * Fp<T>::rcp(sx * (x + lam));
        x = (x + lam) * T(0.25);
        a = (a + lam) * T(0.25);
        b = PAIR ? b * T(0.25) : (b + lam) * T(0.25);
        A = (A + lam) * T(0.25);
        f *= T(0.25);
    }
    const T ra = Fp<T>::rsqrt(A);
    T g = f * (ra * ra);
    T s, q; // (Y + Z, Y Z) of the two leading arguments
    yz_sym<T, PAIR>(A0, a0, b0, g, s, q);
    T Z = s * T(-1.0 / 3.0);
    T Z2 = Z * Z;
    T E2 = q - T(6) * Z2, E3 = (T(3) * q - T(8) * Z2) * Z;
    T E4 = T(3) * (q - Z2) * Z2, E5 = q * Z2 * Z;
    return rj_tail(E2, E3, E4, E5) * g * ra + T(3) * acc;
}

// R_C(x, y) and R_D(y, y, x) = -6 dR_C/dx (x >= 0, y > 0: R_C = R_F(x, y, y), eq. 2.10).
// An FP32 wave none of whose lanes needs a duplication step (rc_r's test at m = 0) takes
// both from the m = 0 tail: with A = (x + 2y)/3, s = y/A - 1 and P the series of
// rc_tail, R_C = A^(-1/2) P(s), and since dA/dx = 1/3, ds/dx = -(1 + s)/(3A),
// R_D(y, y, x) = A^(-3/2) [P(s) + 2 (1 + s) P'(s)] (truncation of P' at |s| <= tau7/2:
// below 2e-7 relative).  Otherwise rc_r and rd_last_x.
template <typename T> __device__ __forceinline__ void rc_rd_r(T x, T y, T &rc, T &rd) {
    const T A0 = (x + T(2) * y) * T(1.0 / 3.0);
    if (sizeof(T) == 4 && __ballot(!(y > T(0)) || Fp<T>::abs(A0 - x) > Fp<T>::tau7 * Fp<T>::abs(A0)) == 0) {
        const T ra = Fp<T>::rsqrt(A0), ia = ra * ra;
        const T s = (y - A0) * ia;
        const T P = rc_tail(s);
        rc = P * ra;
        rd = (P + T(2) * (T(1) + s) * rc_tail_d(s)) * ia * ra;
        return;
    }
    rc = rc_r(x, y);
    rd = rd_last_x<T, false>(x, y, y);
}

// R_F together with the three R_D(., ., x_k) that give its partial derivatives,
// dR_F/dx_k = -R_D(., ., x_k)/6 (eq. 2.10), from one duplication sequence.
// Outputs: rf; rdx = R_D(y, z, x); rdy = R_D(x, z, y) (complex for PAIR; for a
// PAIR triple R_D(x, y, z) = conj(rdy)); rdz = R_D(x, y, z) for real triples.
// Each R_D(., ., x_k) is accumulated along the sequence (the tests check the three
// against the cyclic identity R_D(x,y,z) + R_D(y,z,x) + R_D(z,x,y) = 3/sqrt(xyz),
// DLMF 19.21.7).
// End of a structured duplication sequence for R_F and the three R_D(., ., x_k):
// R_F from its seventh-order expansion about the final mean A, and the R_D tails
// 4^-m R_D(x_m, y_m, z_m; last x_k) from the derivative of that same expansion
// through dR_F/dx_k = -R_D(., ., x_k)/6 (eq. 2.10).  With X_k = 1 - x_k/A
// (sum 0), E2, E3 their symmetric functions, P_k the product of the two
// deviations other than X_k, T(E2, E3) the expansion and T2, T3 its partials:
//   dE2/dx_k = (X_k - 2E2/3)/A,  dE3/dx_k = (E2/3 - E3 - P_k)/A,
//   R_D(., ., x_k) = A^(-3/2) [T - 6 T2 (X_k - 2E2/3) - 6 T3 (E2/3 - E3 - P_k)].
// At R_F's stopping deviation (tau7: 0.136 FP32, 0.0121 FP64) the truncation of
// this derivative is below 4e-7 (FP32) / 2e-14 (FP64) relative.
// Outputs: rf; tx, ty (PAIR: complex, last argument y = a + i b), tz (not PAIR).
template <typename T, bool PAIR>
__device__ __forceinline__ void rfd_tails(T AF0, T x0, T a0, T b0, T AF, T f, T &rf, T &tx, cx<T> &ty, T &tz,
                                          T rs = T(1)) {
    const T ra = Fp<T>::rsqrt(AF);
    const T g = f * (ra * ra);
    const T X = (AF0 - x0) * g;
    T s, q;
    yz_sym<T, PAIR>(AF0, a0, b0, g, s, q);
    const T E2 = q - X * X, E3 = X * q;
    const T tF = rf_tail(E2, E3);
    rf = tF * ra;
    T t2, t3;
    rf_tail_grad(E2, E3, t2, t3);
    const T sc = g * ra * rs; // 4^-m A^(-3/2), times the caller's scale of the R_D outputs
    const T c0 = tF + E2 * (T(4) * t2 - T(2) * t3) + kc<T>(6.0) * t3 * E3;
    const T m2 = kc<T>(-6.0) * t2, m3 = kc<T>(6.0) * t3;
    tx = sc * (c0 + m2 * X + m3 * q); // P_x = Y Z = q
    if (PAIR) {
        // Y = u - i v, Z = conj(Y); P_y = X Z
        const T u = (AF0 - a0) * g, v = b0 * g;
        ty = mkc(sc * (c0 + u * (m2 + m3 * X)), sc * v * (m3 * X - m2));
        tz = T(0);
    } else {
        const T Y = (AF0 - a0) * g, Z = (AF0 - b0) * g;
        ty = mkc(sc * (c0 + m2 * Y + m3 * X * Z), T(0));
        tz = sc * (c0 + m2 * Z + m3 * X * Y);
    }
}

// The R_D outputs come multiplied by rs (a constant the caller would otherwise apply to
// each of them).
template <typename T, bool PAIR>
__device__ void rfd_s(T x, T a, T b, T &rf, T &rdx, cx<T> &rdy, T &rdz, T rs = T(1)) {
    const T AF0 = mean3<T, PAIR>(x, a, b);
    const T x0 = x, a0 = a, b0 = b;
    const T QF = spread3<T, PAIR>(AF0, x, a, b);
    if (wave_no_dup<T, PAIR>(QF, AF0)) {
        T tx, tz;
        cx<T> ty;
        rfd_tails<T, PAIR>(AF0, x0, a0, b0, AF0, T(1), rf, tx, ty, tz, rs);
        rdx = tx;
        rdy = ty;
        rdz = tz;
        return;
    }
    // One duplication sequence, stopped on R_F's criterion; each R_D(., ., x_k) is
    // 3 sum_m 4^-m / (sqrt(x_k,m) (x_k,m + lambda_m)) plus the tail of rfd_tails.
    T AF = AF0, f = T(1), accx = T(0), accz = T(0);
    cx<T> accy = mkc(T(0), T(0));
    for (int m = 0; m < kMaxDup && spread_above<T, PAIR>(QF, f, Fp<T>::tau7, AF); ++m) {
        T sx = Fp<T>::sqrt(x);
        T lam;
        if (PAIR) {
            T r;
            cx<T> sy = csqrt(mkc(a, b), r);
            lam = sx * (T(2) * sy.re) + r;
            accy = accy + crcp(sy * (mkc(a, b) + lam)) * f;
        } else {
            T sy = Fp<T>::sqrt(a), sz = Fp<T>::sqrt(b);
            lam = sx * (sy + sz) + sy * sz;
            accy.re += f * Fp<T>::rcp(sy * (a + lam));
            accz += f * Fp<T>::rcp(sz * (b + lam));
        }
        accx += f * Fp<T>::rcp(sx * (x + lam));
        x = (x + lam) * T(0.25);
        a = (a + lam) * T(0.25);
        b = PAIR ? b * T(0.25) : (b + lam) * T(0.25);
        AF = (AF + lam) * T(0.25);
        f *= T(0.25);
    }
    T tx, tz;
    cx<T> ty;
    rfd_tails<T, PAIR>(AF0, x0, a0, b0, AF, f, rf, tx, ty, tz, rs);
    const T r3 = T(3) * rs;
    rdx = r3 * accx + tx;
    rdy = accy * r3 + ty;
    rdz = r3 * accz + tz;
}

// R_F(x, y, z), R_J(x, y, z, p) and jx = dR_J/dx from one duplication sequence (p real
// > 0).  The derivative is carried through every step of the recursion (forward
// mode: the iterates' derivatives in the initial x, the R_C terms' and the fifth-order
// tail's), so it stays accurate where p is close to x -- where the form that eq. 2.11
// gives, (R_J - R_D(y, z, x)) / (2 (p - x)), cancels.  Along the sequence the
// derivatives of y, z and p are equal (each moves by lambda/4 per step; for PAIR the
// imaginary part b is not moved by lambda), so two tracks suffice: dx and dy.  The
// J criterion stops at taujx < tau5: the derivative of the truncated expansion loses
// one order of the deviation.
template <typename T, bool PAIR>
__device__ void rfjx_s(T x, T a, T b, T p, T &rf, T &rj, T &jx) {
    const T AF0 = mean3<T, PAIR>(x, a, b);
    const T AJ0 = (T(3) * AF0 + T(2) * p) * T(0.2);
    const T x0 = x, a0 = a, b0 = b, p0 = p;
    const T QF = spread3<T, PAIR>(AF0, x, a, b);
    const T QJ = tmax(spread3<T, PAIR>(AJ0, x, a, b), spread1<T, PAIR>(AJ0 - p));
    const T pyz = PAIR ? (p - a) * (p - a) + b * b : (p - a) * (p - b);
    const T delta = (p - x) * pyz, ddelta = -pyz;
    T AF = AF0, AJ = AJ0, f = T(1), acc = T(0), dacc = T(0);
    T dx = T(1), dy = T(0), dAJ = T(0.2);
    for (int m = 0; m < kMaxDup && (spread_above<T, PAIR>(QF, f, Fp<T>::tau7, AF) ||
                                   spread_above<T, PAIR>(QJ, f, Fp<T>::taujx, AJ)); ++m) {
        const T rsx = Fp<T>::rsqrt(x), rsp = Fp<T>::rsqrt(p);
        const T sx = x * rsx, sp = p * rsp;
        const T dsx = T(0.5) * dx * rsx, dsp = T(0.5) * dy * rsp;
        T lam, dlam, d, dd;
        if (PAIR) {
            T r;
            const T syr = csqrt_re(a, b, r);
            const T ir = Fp<T>::rcp(r);
            lam = T(2) * sx * syr + r;
            const T dsyr = T(0.5) * dy * syr * ir, dr = a * dy * ir;
            dlam = T(2) * (dsx * syr + sx * dsyr) + dr;
            const T g2 = p + T(2) * sp * syr + r;
            const T dg2 = dy + T(2) * (dsp * syr + sp * dsyr) + dr;
            d = (sp + sx) * g2;
            dd = (dsp + dsx) * g2 + (sp + sx) * dg2;
        } else {
            const T rsy = Fp<T>::rsqrt(a), rsz = Fp<T>::rsqrt(b);
            const T sy = a * rsy, sz = b * rsz;
            const T dsy = T(0.5) * dy * rsy, dsz = T(0.5) * dy * rsz;
            lam = sx * (sy + sz) + sy * sz;
            dlam = dsx * (sy + sz) + sx * (dsy + dsz) + dsy * sz + sy * dsz;
            const T py = sp + sy, pz = sp + sz, px = sp + sx;
            d = px * py * pz;
            dd = (dsp + dsx) * py * pz + px * ((dsp + dsy) * pz + py * (dsp + dsz));
        }
        const T rdd = Fp<T>::rcp(d);
        const T f3 = f * f * f;
        const T e = delta * rdd * rdd * f3;
        const T de = f3 * rdd * rdd * (ddelta - T(2) * delta * dd * rdd);
        const T rc = rc1_r(e);
        acc += f * rc * rdd;
        dacc += f * (rc1_dr(e, rc) * de * rdd - rc * rdd * rdd * dd);
        x = (x + lam) * T(0.25);
        a = (a + lam) * T(0.25);
        b = PAIR ? b * T(0.25) : (b + lam) * T(0.25);
        p = (p + lam) * T(0.25);
        AF = (AF + lam) * T(0.25);
        AJ = (AJ + lam) * T(0.25);
        dx = (dx + dlam) * T(0.25);
        dy = (dy + dlam) * T(0.25);
        dAJ = (dAJ + dlam) * T(0.25);
        f *= T(0.25);
    }
    {
        const T raF = Fp<T>::rsqrt(AF);
        const T gF = f * (raF * raF);
        const T X = (AF0 - x0) * gF;
        T s, q;
        yz_sym<T, PAIR>(AF0, a0, b0, gF, s, q);
        rf = rf_tail(q - X * X, X * q) * raF;
    }
    const T ra = Fp<T>::rsqrt(AJ);
    const T iA = ra * ra;
    const T g = f * iA, dg = -g * dAJ * iA, dra = T(-0.5) * ra * dAJ * iA;
    const T X = (AJ0 - x0) * g, dX = T(-0.8) * g + (AJ0 - x0) * dg;
    T s, q, ds, dq;
    if (PAIR) {
        const T u = (AJ0 - a0) * g, v = b0 * g;
        const T du = T(0.2) * g + (AJ0 - a0) * dg, dv = b0 * dg;
        s = T(2) * u; q = u * u + v * v;
        ds = T(2) * du; dq = T(2) * (u * du + v * dv);
    } else {
        const T Y = (AJ0 - a0) * g, Z = (AJ0 - b0) * g;
        const T dY = T(0.2) * g + (AJ0 - a0) * dg, dZ = T(0.2) * g + (AJ0 - b0) * dg;
        s = Y + Z; q = Y * Z;
        ds = dY + dZ; dq = dY * Z + Y * dZ;
    }
    const T P = (AJ0 - p0) * g, dP = T(0.2) * g + (AJ0 - p0) * dg;
    const T sym2 = X * s + q, xyz = X * q, P2 = P * P;
    const T dsym2 = dX * s + X * ds + dq, dxyz = dX * q + X * dq, dP2 = T(2) * P * dP;
    const T E2 = sym2 - T(3) * P2, dE2 = dsym2 - T(3) * dP2;
    const T P3 = P2 * P, dP3 = dP2 * P + P2 * dP;
    const T E3 = xyz + T(2) * E2 * P + T(4) * P3;
    const T dE3 = dxyz + T(2) * (dE2 * P + E2 * dP) + T(4) * dP3;
    const T B4 = T(2) * xyz + E2 * P + T(3) * P3;
    const T dB4 = T(2) * dxyz + dE2 * P + E2 * dP + T(3) * dP3;
    const T E4 = B4 * P, dE4 = dB4 * P + B4 * dP;
    const T E5 = xyz * P2, dE5 = dxyz * P2 + xyz * dP2;
    const T tail = rj_tail(E2, E3, E4, E5);
    const T dtail = dE2 * (T(-3.0 / 14.0) + T(9.0 / 44.0) * E2 - T(9.0 / 52.0) * E3) +
                    dE3 * (T(1.0 / 6.0) - T(9.0 / 52.0) * E2) - T(3.0 / 22.0) * dE4 + T(3.0 / 26.0) * dE5;
    rj = tail * g * ra + T(6) * acc;
    jx = dtail * g * ra + tail * (dg * ra + g * dra) + T(6) * dacc;
    if (!(p0 > T(0))) rj = jx = Fp<T>::nan();
}

// R_F, R_J(x, y, z, p) and the R_D(., ., x_k) of the triple, from one duplication
// sequence (the adjoint of the time coordinate).  p real > 0.  Output conventions
// as rfd_s.
template <typename T, bool PAIR>
__device__ void rfjd_s(T x, T a, T b, T p, T &rf, T &rj, T &rdx, cx<T> &rdy, T &rdz) {
    const T AF0 = mean3<T, PAIR>(x, a, b);
    const T AJ0 = (T(3) * AF0 + T(2) * p) * T(0.2);
    const T x0 = x, a0 = a, b0 = b, p0 = p;
    const T QF = spread3<T, PAIR>(AF0, x, a, b);
    const T QJ = tmax(spread3<T, PAIR>(AJ0, x, a, b), spread1<T, PAIR>(AJ0 - p));
    const T delta = PAIR ? (p - x) * ((p - a) * (p - a) + b * b) : (p - x) * (p - a) * (p - b);
    T AF = AF0, AJ = AJ0, f = T(1), acc = T(0), accz = T(0);
    cx<T> accy = mkc(T(0), T(0));
    for (int m = 0; m < kMaxDup && (spread_above<T, PAIR>(QF, f, Fp<T>::tau7, AF) ||
                                   spread_above<T, PAIR>(QJ, f, Fp<T>::tau5, AJ)); ++m) {
        T sx = Fp<T>::sqrt(x), sp = Fp<T>::sqrt(p);
        T lam, d;
        if (PAIR) {
            T r;
            cx<T> sy = csqrt(mkc(a, b), r);
            lam = sx * (T(2) * sy.re) + r;
            d = (sp + sx) * (p + T(2) * sp * sy.re + r);
            accy = accy + crcp(sy * (mkc(a, b) + lam)) * f;
        } else {
            T sy = Fp<T>::sqrt(a), sz = Fp<T>::sqrt(b);
            lam = sx * (sy + sz) + sy * sz;
            d = (sp + sx) * (sp + sy) * (sp + sz);
            accy.re += f * Fp<T>::rcp(sy * (a + lam));
            accz += f * Fp<T>::rcp(sz * (b + lam));
        }
        T rdd = Fp<T>::rcp(d);
        acc += f * rc1_r(delta * rdd * rdd * (f * f * f)) * rdd;
        x = (x + lam) * T(0.25);
        a = (a + lam) * T(0.25);
        b = PAIR ? b * T(0.25) : (b + lam) * T(0.25);
        p = (p + lam) * T(0.25);
        AF = (AF + lam) * T(0.25);
        AJ = (AJ + lam) * T(0.25);
        f *= T(0.25);
    }
    T tx, tz;
    cx<T> ty;
    rfd_tails<T, PAIR>(AF0, x0, a0, b0, AF, f, rf, tx, ty, tz);
    rdy = accy * T(3) + ty;
    rdz = T(3) * accz + tz;
    // R_D(y, z, x) from the cyclic identity R_D(x,y,z) + R_D(y,z,x) + R_D(z,x,y) =
    // 3/sqrt(xyz) (DLMF 19.21.7) instead of a third accumulation (on the time
    // coordinate's triples the terms are of one size; tested against the oracle)
    if (PAIR) rdx = T(3) * Fp<T>::rsqrt(x0 * (a0 * a0 + b0 * b0)) - T(2) * rdy.re;
    else rdx = T(3) * Fp<T>::rsqrt(x0 * a0 * b0) - rdy.re - rdz;
    {
        const T rj_a = Fp<T>::rsqrt(AJ);
        T g = f * (rj_a * rj_a);
        T X = (AJ0 - x0) * g, s, q;
        yz_sym<T, PAIR>(AJ0, a0, b0, g, s, q);
        T P = (AJ0 - p0) * g;
        T sym2 = X * s + q, xyz = X * q, P2 = P * P;
        T E2 = sym2 - T(3) * P2;
        T E3 = xyz + T(2) * E2 * P + T(4) * P2 * P;
        T E4 = (T(2) * xyz + E2 * P + T(3) * P2 * P) * P;
        T E5 = xyz * P2;
        rj = rj_tail(E2, E3, E4, E5) * g * rj_a + T(6) * acc;
    }
    if (!(p0 > T(0))) rj = Fp<T>::nan();
}

} // namespace cosmo
