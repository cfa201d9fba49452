// lane.hpp -- per-(cosmology, redshift) formulas, one GPU lane each.
//
// Notation (x = 1 + z, integration from x1 = 1 to x2 = 1 + z, dz = z):
//   X_n = sqrt(x2 - rho_n) = sqrt(z + w_n),  Y_n = sqrt(1 - rho_n)     (roots of Q)
//   Xt  = sqrt(1 - sigma x2),                Yt  = sqrt(1 - sigma)       (radiation factor)
//   U_m = Xt X_m Y_a Y_b + Yt Y_m X_a X_b    ({m, a, b} = {0, 1, 2})
// U_m is the paper's u_{lm} of sec. 3.1 (pairing the radiation root l with root
// m; the complementary pairs coincide, u_{ij} = u_{kl}) divided by sqrt(|rho_l|).
// For Or = 0 the radiation factor is one and U_m is the u_m of app. B.1.
//
//   D_C = (c/H0) beta^(-1/2) 2 dz R_F(U_0^2, U_1^2, U_2^2)                (eqs. 3.7, B.1)
//   T   = (1/H0) beta^(-1/2) 2 dz { (dz^2/3) prod_n(1 - s rho_n) R_J(U^2, W5)
//                                   + R_C(S5, Q5) + sigma R_F(U^2) }       (eqs. 3.8, B.2)
//         with j = 0 the real root of Q:  W5 = U_0^2 + dz^2 (1-s rho_1)(1-s rho_2) rho_0,
//         Q5 = x2 W5 / ((1-s)(1-s x2)),  S5 = Q5 - dz^2 rho_0 rho_1 rho_2
//   X   = (c/H0) beta^(-1/2) ...  (eq. 3.9 with i = 0 the real root of Q and l the
//         radiation root; eq. B.3 for Or = 0), with a Gauss-Legendre route for
//         lanes where eq. 3.9 cancels (see x_hat).
// The expressions in sigma are eqs. 3.7-3.9 after the substitution
// sqrt(z - r_l) = sqrt(|rho_l|) sqrt(1 - sigma x) and the homogeneity of the
// Carlson integrals; at sigma = 0 they are literally eqs. B.1-B.3.
#pragma once

#include "carlson.hpp"
#include "gl_tables.hpp"
#include "setup.hpp"

namespace cosmo {

template <typename T> __device__ __forceinline__ const LaneConst<T> &lane_of(const CosmoRec &r);
template <> __device__ __forceinline__ const LaneConst<float> &lane_of<float>(const CosmoRec &r) { return r.f; }
template <> __device__ __forceinline__ const LaneConst<double> &lane_of<double>(const CosmoRec &r) { return r.d; }

// Geometry of one lane.  For PAIR, slot 1 is complex and slot 2 its conjugate.
template <typename T, bool PAIR> struct Geo {
    T Xt, Xt2, X0, X02;
    T X1re, X1im, X1abs;   // X_1 (PAIR: complex; |X_1|^2 = |z + w_1| in X1abs); REAL: X1re
    T X2;                  // REAL only
    T U0, U1re, U1im, U2;  // U_m (PAIR: U_1 complex, U_2 = conj)
    T T1_0, T2_0;          // the two products making U_0
    T T1_1re, T1_1im, T2_1re, T2_1im; // same for U_1 (PAIR) ; REAL: T1_1re, T2_1re
    T T1_2, T2_2;          // REAL only
    T va, vb;              // structured second/third Carlson arguments
    // INV builds only: 1/Xt^2, 1/X_0^2 and 1/X_1^2 (PAIR: complex; REAL: also 1/X_2^2),
    // and 1/(Xt X_0 |X_1|^2) (REAL: 1/(Xt X_0 X_1 X_2)) = beta^(1/2) / E(z)
    T iXt2, iX02, iX1re, iX1im, iX2, iXprod;
};

// INV: the square roots come from reciprocal square roots (s = v rsqrt(v)), which
// also give the reciprocals 1/v the adjoint's chain needs, one transcendental per
// root instead of two.
template <typename T, bool PAIR, bool INV = false>
__device__ __forceinline__ void build_u(const LaneConst<T> &k, T z, Geo<T, PAIR> &g) {
    g.Xt2 = k.yt2 - k.sigma * z; // 1 - sigma (1 + z)
    g.X02 = z + k.w0;
    if (INV) {
        const T rt = Fp<T>::rsqrt(g.Xt2), r0 = Fp<T>::rsqrt(g.X02);
        g.Xt = g.Xt2 * rt; g.iXt2 = rt * rt;
        g.X0 = g.X02 * r0; g.iX02 = r0 * r0;
        g.iXprod = rt * r0;
    } else {
        g.Xt = Fp<T>::sqrt(g.Xt2);
        g.X0 = Fp<T>::sqrt(g.X02);
    }
    if (PAIR) {
        T ab;
        const T w1re = z + k.w1re;
        cx<T> X1;
        if (INV) {
            T iab;
            X1 = csqrt_uim_inv(w1re, k.w1im2, k.hw1im, k.sw1im, ab, iab);
            const T i2 = iab * iab;
            g.iX1re = w1re * i2; g.iX1im = -k.w1im * i2;
            g.iXprod *= iab;
        } else {
            X1 = csqrt(mkc(w1re, k.w1im), ab);
        }
        g.X1re = X1.re; g.X1im = X1.im; g.X1abs = ab;
        // U_0 = Xt X_0 |Y_1|^2 + Yt Y_0 |X_1|^2
        g.T1_0 = g.Xt * g.X0 * k.y1abs2;
        g.T2_0 = k.yty0 * ab;
        g.U0 = g.T1_0 + g.T2_0;
        // U_1 = Xt Y_0 w + Yt X_0 conj(w),  w = X_1 conj(Y_1)
        cx<T> w = X1 * mkc(k.y1re, -k.y1im);
        T cA = g.Xt * k.y0, cB = k.yt * g.X0;
        g.T1_1re = cA * w.re; g.T1_1im = cA * w.im;
        g.T2_1re = cB * w.re; g.T2_1im = -cB * w.im;
        g.U1re = g.T1_1re + g.T2_1re;
        g.U1im = g.T1_1im + g.T2_1im;
        g.va = g.U1re * g.U1re - g.U1im * g.U1im;
        g.vb = T(2) * g.U1re * g.U1im;
    } else {
        const T v1 = z + k.w1re, v2 = z + k.w2;
        if (INV) {
            const T r1 = Fp<T>::rsqrt(v1), r2 = Fp<T>::rsqrt(v2);
            g.X1re = v1 * r1; g.iX1re = r1 * r1;
            g.X2 = v2 * r2; g.iX2 = r2 * r2;
            g.iXprod *= r1 * r2;
        } else {
            g.X1re = Fp<T>::sqrt(v1);
            g.X2 = Fp<T>::sqrt(v2);
        }
        g.X1im = T(0); g.X1abs = T(0);
        g.T1_0 = g.Xt * g.X0 * k.y1y2;
        g.T2_0 = k.yty0 * (g.X1re * g.X2);
        g.T1_1re = g.Xt * g.X1re * k.y0y2;
        g.T2_1re = k.yty1 * (g.X0 * g.X2);
        g.T1_2 = g.Xt * g.X2 * k.y0y1;
        g.T2_2 = k.yty2 * (g.X0 * g.X1re);
        g.T1_1im = g.T2_1im = T(0);
        g.U0 = g.T1_0 + g.T2_0;
        g.U1re = g.T1_1re + g.T2_1re;
        g.U1im = T(0);
        g.U2 = g.T1_2 + g.T2_2;
        g.va = g.U1re * g.U1re;
        g.vb = g.U2 * g.U2;
    }
}

// chi / D_H (dimensionless comoving distance), eqs. 3.7 / B.1
template <typename T, bool PAIR> __device__ __forceinline__ T chi_hat(const LaneConst<T> &k, T z) {
    Geo<T, PAIR> g;
    build_u<T, PAIR>(k, z, g);
    return k.pre2 * z * rf_s<T, PAIR>(g.U0 * g.U0, g.va, g.vb);
}

// Arguments of the time coordinate's integrals (eqs. 3.8 / B.2): the U_m of build_u,
// V0 = U_0^2, W5, Q5 = x2 W5 / ((1 - s)(1 - s x2)) and S5 = Q5 - dz^2 rho_0 rho_1 rho_2.
// W5 = U_j^2 + dz^2 (1 - s rho_k)(1 - s rho_l) rho_j is the same for every j; its terms
// cancel when rho_j < 0 (at large z, by up to the ratio of the terms), so the j with
// the smallest terms is used (for a pair, the real part of the slot-1 form).
template <typename Q, bool PAIR>
__device__ __forceinline__ void t_args_in(const LaneConst<Q> &k, Q z, Geo<Q, PAIR> &g, Q &V0, Q &W, Q &Qv, Q &S) {
    build_u<Q, PAIR>(k, z, g);
    V0 = g.U0 * g.U0;
    const Q z2 = z * z;
    W = V0 + z2 * k.c5;
    Q m0 = V0 + Fp<Q>::abs(z2 * k.c5);
    const Q w1 = g.va + z2 * k.c5b;
    const Q m1 = (PAIR ? g.U1re * g.U1re + g.U1im * g.U1im : g.va) + Fp<Q>::abs(z2 * k.c5b);
    if (m1 < m0) { W = w1; m0 = m1; }
    if (!PAIR) {
        const Q w2 = g.vb + z2 * k.c5c, m2 = g.vb + Fp<Q>::abs(z2 * k.c5c);
        if (m2 < m0) W = w2;
    }
    Qv = (Q(1) + z) * W * Fp<Q>::rcp(k.yt2 * g.Xt2);
    S = Qv - z2 * k.rprod;
}

template <typename T, bool PAIR> struct TArgs {
    Geo<T, PAIR> g;
    T V0, W, Q, S;
};

template <typename A, typename B, bool PAIR> __device__ __forceinline__ void geo_cast(const Geo<A, PAIR> &a, Geo<B, PAIR> &b) {
    b.Xt = B(a.Xt); b.Xt2 = B(a.Xt2); b.X0 = B(a.X0); b.X02 = B(a.X02);
    b.X1re = B(a.X1re); b.X1im = B(a.X1im); b.X1abs = B(a.X1abs); b.X2 = B(a.X2);
    b.U0 = B(a.U0); b.U1re = B(a.U1re); b.U1im = B(a.U1im); b.U2 = B(a.U2);
    b.T1_0 = B(a.T1_0); b.T2_0 = B(a.T2_0);
    b.T1_1re = B(a.T1_1re); b.T1_1im = B(a.T1_1im); b.T2_1re = B(a.T2_1re); b.T2_1im = B(a.T2_1im);
    b.T1_2 = B(a.T1_2); b.T2_2 = B(a.T2_2); b.va = B(a.va); b.vb = B(a.vb);
}

// The FP32 path forms these arguments in FP64 from the FP64 lane constants and rounds
// once: in FP32 the products of square roots making U_m, and W5, accumulate a dozen
// roundings, which at large z is the leading error of t (FP64 multiplies and FMAs
// issue at the FP32 rate on this hardware; the Carlson iterations stay in FP32).
template <typename T, bool PAIR> __device__ __forceinline__ void t_args(const CosmoRec &r, T z, TArgs<T, PAIR> &a);
template <> __device__ __forceinline__ void t_args<double, true>(const CosmoRec &r, double z, TArgs<double, true> &a) {
    t_args_in<double, true>(r.d, z, a.g, a.V0, a.W, a.Q, a.S);
}
template <> __device__ __forceinline__ void t_args<double, false>(const CosmoRec &r, double z, TArgs<double, false> &a) {
    t_args_in<double, false>(r.d, z, a.g, a.V0, a.W, a.Q, a.S);
}
template <bool PAIR> __device__ __forceinline__ void t_args_f32(const CosmoRec &r, float z, TArgs<float, PAIR> &a) {
    Geo<double, PAIR> gd;
    double V0, W, Qv, S;
    t_args_in<double, PAIR>(r.d, (double)z, gd, V0, W, Qv, S);
    geo_cast<double, float, PAIR>(gd, a.g);
    a.V0 = float(V0); a.W = float(W); a.Q = float(Qv); a.S = float(S);
}
template <> __device__ __forceinline__ void t_args<float, true>(const CosmoRec &r, float z, TArgs<float, true> &a) {
    t_args_f32<true>(r, z, a);
}
template <> __device__ __forceinline__ void t_args<float, false>(const CosmoRec &r, float z, TArgs<float, false> &a) {
    t_args_f32<false>(r, z, a);
}

// t / (1/H0), eqs. 3.8 / B.2
template <typename T, bool PAIR> __device__ __forceinline__ T t_hat(const CosmoRec &r, T z) {
    const LaneConst<T> &k = lane_of<T>(r);
    TArgs<T, PAIR> a;
    t_args<T, PAIR>(r, z, a);
    const T z2 = z * z;
    T rf, rj;
    rfj_s<T, PAIR>(a.V0, a.g.va, a.g.vb, a.W, rf, rj);
    T rc = rc_r(a.S, a.Q);
    return k.pre2 * z * (z2 * T(1.0 / 3.0) * k.pre3 * rj + rc + k.sigma * rf);
}

// sqrt(Q(x)) at x2 = 1 + z and at x1 = 1 (products of the X_n / Y_n)
template <typename T, bool PAIR>
__device__ __forceinline__ void sqrtQ(const LaneConst<T> &k, const Geo<T, PAIR> &g, T &f2, T &f1) {
    if (PAIR) {
        f2 = g.X0 * g.X1abs;
        f1 = k.y0 * k.y1abs2;
    } else {
        f2 = g.X0 * g.X1re * g.X2;
        f1 = k.y0 * k.y1re * k.y2;
    }
}

// Gauss-Legendre nodes and weights: literal tables (gl_tables.hpp, 20 nodes FP64, 8
// FP32), so the quadrature routes need no run-time initialisation.
constexpr int kGlNp = 4;         // panels in u = ln(1+z)

template <typename Q> struct GlRule;
template <> struct GlRule<double> {
    static constexpr int n = kGlN64;
    static __device__ __forceinline__ double x(int i) { return c_gl64_x[i]; }
    static __device__ __forceinline__ double w(int i) { return c_gl64_w[i]; }
    static __device__ __forceinline__ double expm1_small(double u) { return ::expm1(u); }
};
template <> struct GlRule<float> {
    static constexpr int n = kGlN32;
    static __device__ __forceinline__ float x(int i) { return c_gl32_x[i]; }
    static __device__ __forceinline__ float w(int i) { return c_gl32_w[i]; }
    // e^u - 1 for 0 <= u <= 1/2: Taylor polynomial to u^8 (remainder below 6e-9 relative)
    static __device__ __forceinline__ float expm1_small(float u) {
        float p = 1.0f / 40320.0f;
        p = p * u + 1.0f / 5040.0f;
        p = p * u + 1.0f / 720.0f;
        p = p * u + 1.0f / 120.0f;
        p = p * u + 1.0f / 24.0f;
        p = p * u + 1.0f / 6.0f;
        p = p * u + 0.5f;
        p = p * u + 1.0f;
        return p * u;
    }
};

// Composite Gauss-Legendre quadrature in u = ln(1+z) of the defining integrals
// (eqs. 2.3-2.5): power 0 -> int x/E du (D_C), 1 -> int 1/E du (T), 2 -> int x^3/E du
// (X).  With grad, also the Leibniz derivatives -1/2 int f dP/dtheta / E^3 du for
// theta = (Om, OL, Or).  E^2 = beta (1 - sigma x) Q(x) in factored form.
// The number of equal panels is max(min_np, U / dpath) (capped at 64; min_np = 4 by
// default): every panel is then no wider than the distance d of the nearest
// singularity of the integrand from the path.  In units of the half-width h <= d/2 such
// a singularity lies outside the stadium of radius 2 about the panel; the smallest
// Bernstein-ellipse parameter on that stadium is 2 + sqrt(5) = 4.24 (abreast of the
// panel's centre), so the Gauss-Legendre error is of order 4.24^(-2n): below 1e-25 with
// 20 nodes, 1e-10 with 8.
// Nodes: for U > 1/2 they are placed from the upper limit down, x = (1+z) exp(-(U - u)):
// the integrands grow with x, and measuring from the top keeps the rounding of the node
// abscissae (absolute, ~eps times the distance from the anchor) smallest where the
// weight is.  For U <= 1/2 they are placed from x = 1 with x - 1 = expm1(u), which
// keeps x - 1 (a factor of every derivative integrand) accurate relative to itself.
template <typename Q, bool PAIR>
__device__ void gl_integral(const LaneConst<Q> &k, Q z, int power, bool grad, Q &val, Q gth[3], int min_np = kGlNp) {
    const Q U = Fp<Q>::log1p(z);
    const Q want = U * Fp<Q>::rcp(k.dpath);
    const int np = want > Q(64) ? 64 : (want > Q(min_np) ? (int)__builtin_ceil((double)want) : min_np);
    const Q h = U * Fp<Q>::rcp(Q(np));
    const Q x2 = Q(1) + z;
    const bool low = U <= Q(0.5);
    Q s = Q(0), g0 = Q(0), g1 = Q(0), g2 = Q(0);
    for (int p = 0; p < np; ++p) {
        const Q vmid = h * (Q(np - p) - Q(0.5)); // U - (panel midpoint)
        const Q umid = h * (Q(p) + Q(0.5));
        for (int i = 0; i < GlRule<Q>::n; ++i) {
            Q x, xm1;
            if (low) {
                xm1 = GlRule<Q>::expm1_small(umid + Q(0.5) * h * GlRule<Q>::x(i));
                x = Q(1) + xm1;
            } else {
                x = x2 * Fp<Q>::exp_fast(-(vmid - Q(0.5) * h * GlRule<Q>::x(i)));
                xm1 = x - Q(1);
            }
            Q q = PAIR ? (xm1 + k.w0) * ((xm1 + k.w1re) * (xm1 + k.w1re) + k.w1im * k.w1im)
                       : (xm1 + k.w0) * (xm1 + k.w1re) * (xm1 + k.w2);
            Q e2 = k.beta * (k.yt2 - k.sigma * xm1) * q;
            Q ie = Fp<Q>::rsqrt(e2);
            Q fx = power == 0 ? x : (power == 1 ? Q(1) : x * x * x);
            Q wf = GlRule<Q>::w(i) * fx * ie;
            s += wf;
            if (grad) {
                Q c = Q(-0.5) * wf * ie * ie;
                Q xx = x * x;
                g0 += c * xx * xm1;                      // x^3 - x^2
                g1 += c * (-xm1 * (Q(2) + xm1));        // 1 - x^2
                g2 += c * xx * xm1 * (Q(2) + xm1);      // x^4 - x^2
            }
        }
    }
    const Q hh = Q(0.5) * h;
    val = s * hh;
    if (grad) { gth[0] = g0 * hh; gth[1] = g1 * hh; gth[2] = g2 * hh; }
}

// Absorption distance (eqs. 3.9, B.3): X / (c/H0) = pre * z * B, returned as B together
// with the size M of its terms for the rounding check.
//
// Eq. 3.9 in the normalised form (i = 0 the real root of Q, (j, k) = slots 1, 2, l the
// radiation root) reads B = A + t2 + L (B1 - B2) with L = -1/sigma = |rho_l|:
//   B1 = (1 - s r1)(1 - s r2) [ (dz^2/3) d01 d02 R_D(U1^2, U2^2, U0^2) + X0 Y0 / (Xt Yt U0) ]
//   B2 = (1 + s S3) [ (dz^2/3) d01 d02 (1 - s r0) R_J(U^2, p) + R_C(q - s dz^2, q) ]
// with p = U0^2 + s dz^2 d01 d02 (the paper's u_i0^2 in these units) and q = p/(X0 Y0)^2.
// B1 and B2 agree to O(sigma), so the printed form loses ~|rho_l| ~ Om/Or digits.  It
// is rearranged so that the 1/sigma cancels analytically:
//  * R_D(U1^2, U2^2, U0^2) = R_J(U^2, U0^2), and with F(w) = R_J(U^2, w) the exact
//    divided difference F(U0^2) - F(p) = 2 (U0^2 - p) dR_J/dx (U^2, p) (from R_J's
//    integral representation; x its first argument), where U0^2 - p = -s dz^2 d01 d02:
//    that pair of terms becomes 2 (dz^2/3) d01 d02 (1 - s r1)(1 - s r2) dz^2 d01 d02
//    dR_J/dx, the derivative from rfjx_s, plus e1 (dz^2/3) d01 d02 R_J(U^2, p) with
//    e1 = [(1 - s r1)(1 - s r2) - (1 + s S3)(1 - s r0)] / s, a polynomial in sigma;
//  * R_C(q(1 - tau), q) = q^(-1/2) sum_n c_n tau^n, tau = s dz^2/q, c_n = (1/2)_n^2 /
//    ((3/2)_n n!) (R_C's hypergeometric series), whose n >= 1 part carries a factor
//    sigma; the remaining algebraic pair [(1 - s r1)(1 - s r2) / (Xt Yt U0) - (1 + s S3)
//    / sqrt(p)] / sigma is formed from sqrt(p) - U0 = s dz^2 d01 d02 / (sqrt(p) + U0) and
//    (Xt - 1)/s = -x2/(Xt + 1), (Yt - 1)/s = -1/(Yt + 1).
// Every term of the result is a regular function of sigma; at sigma = 0 it is the value
// of eq. B.3 (X is continuous in Or), so one form serves both degrees.  It is used
// while |tau| is small enough for the series (there the printed form cancels by
// ~1/(|s| x2) >= 1/tau_max); beyond, eq. 3.9 is evaluated as printed, its R_D from the
// same duplication sequence as F(U0^2) = F(p) + 2 (U0^2 - p) dR_J/dx.  Both are the
// paper's Carlson reduction; only the order of the algebra differs.  A milder
// cancellation at small z between terms of size ~r0^2 remains in either form (up to
// ~20 on the non-flat workload): M / |B| is returned for the caller's check.
template <typename Q> struct XSeries;
template <> struct XSeries<float> {
    static constexpr int n = 8;           // c_1 .. c_8: truncation below 4e-9 relative at |tau| = tau_max
    static constexpr float tau_max = 0.125f;
};
template <> struct XSeries<double> {
    static constexpr int n = 16;          // below 1e-17
    static constexpr double tau_max = 0.1;
};
constexpr double rc_series_coef(int n) { // c_n = (1/2)_n^2 / ((3/2)_n n!)
    double c = 1.0;
    for (int k = 0; k < n; ++k) c = c * (k + 0.5) * (k + 0.5) / ((k + 1.5) * (k + 1.0));
    return c;
}

// Q: precision of the Carlson integrals; G: precision of the geometry, the algebraic
// terms and the sum (the FP32 path forms them in FP64 and rounds the Carlson arguments
// once, as for the time coordinate: the algebraic terms are the largest, and FP32
// products of square roots would put a few ulp of error into each).
// The R_F term is returned apart (t2 = xc2 R_F with its FP64 Carlson arguments): at small
// z it is one of the two largest terms, so an FP32 lane whose terms cancel can refine it
// alone in FP64.
template <typename G> struct XRf {
    G V0, va, vb, t2;
};
template <typename Q, typename G, bool PAIR> __device__ G x_terms(const CosmoRec &r, G z, G &mag, XRf<G> &xr) {
    const LaneConst<G> &k = lane_of<G>(r);
    Geo<G, PAIR> g;
    build_u<G, PAIR>(k, z, g);
    const G s = k.sigma;
    const G V0 = g.U0 * g.U0;
    const G z2 = z * z;
    const G x2 = G(1) + z;
    const G cc = z2 * G(1.0 / 3.0) * k.d0102;
    const G p = V0 + s * z2 * k.d0102;
    const G iq = g.X02 * k.w0 * Fp<G>::rcp(p); // 1/q
    const G tau = s * z2 * iq;
    const G xy = g.X0 * k.y0;
    G f2, f1;
    sqrtQ<G, PAIR>(k, g, f2, f1);
    // (Q(x2) - Q(1))/dz as a divided difference (no cancellation at small z)
    const G DQ = G(3) + z * (G(3) + z) + k.q2 * (G(2) + z) + k.q1;
    const G num = DQ - s * (x2 * (G(1) + x2) + k.q2 * x2 - k.q0);
    const G fq2 = f2 * Fp<G>::rsqrt(g.Xt2), fq1 = f1 * Fp<G>::rsqrt(k.yt2);
    const G A = num * Fp<G>::rcp(k.yt2 * g.Xt2 * (fq2 + fq1));
    const bool regular = Fp<G>::abs(tau) <= G(XSeries<Q>::tau_max);
    // the algebraic terms first (few values stay live across the Carlson sequence)
    G alg, amag;
    if (regular) {
        const G rs = Fp<G>::rsqrt(p), su = p * rs;
        const G D1 = z2 * k.d0102 * Fp<G>::rcp(su + g.U0);     // (sqrt(p) - U0)/s
        const G xm = -x2 * Fp<G>::rcp(g.Xt + G(1));             // (Xt - 1)/s
        const G D2 = s * xm * k.xym + xm + k.xym;               // (Xt Yt - 1)/s
        const G b = k.xs3;
        const G Np = D1 + k.xa * g.U0 + k.xa * s * D1 - D2 * g.U0 - b * g.U0 - b * s * D2 * g.U0;
        const G tN = -xy * Np * Fp<G>::rcp(g.Xt * k.yt * g.U0 * su);
        G S1 = G(rc_series_coef(XSeries<Q>::n));
#pragma unroll
        for (int n = XSeries<Q>::n - 1; n >= 1; --n) S1 = S1 * tau + G(rc_series_coef(n));
        const G tS = k.op1s3 * xy * rs * z2 * iq * S1;
        alg = A + tN + tS;
        amag = Fp<G>::abs(A) + Fp<G>::abs(tN) + Fp<G>::abs(tS);
    } else {
        const G q = Fp<G>::rcp(iq);
        const G L = -Fp<G>::rcp(s);
        const G a1 = L * k.om1s12 * xy * Fp<G>::rcp(g.Xt * k.yt * g.U0);
        const G a2 = -L * k.op1s3 * G(rc_r(Q(q - s * z2), Q(q)));
        alg = A + a1 + a2;
        amag = Fp<G>::abs(A) + Fp<G>::abs(a1) + Fp<G>::abs(a2);
    }
    Q rf, rj, jx;
    rfjx_s<Q, PAIR>(Q(V0), Q(g.va), Q(g.vb), Q(p), rf, rj, jx);
    const G t2 = k.xc2 * G(rf);
    xr.V0 = V0; xr.va = g.va; xr.vb = g.vb; xr.t2 = t2;
    G t3, t4;
    if (regular) {
        t3 = G(2) * cc * k.om1s12 * z2 * k.d0102 * G(jx);
        t4 = -cc * k.xe1 * G(rj);
    } else {
        const G L = -Fp<G>::rcp(s);
        const G rd = G(rj) - G(2) * s * z2 * k.d0102 * G(jx); // R_D(U1^2, U2^2, U0^2)
        t3 = L * k.om1s12 * cc * rd;
        t4 = -L * k.op1s3 * cc * k.om1s0 * G(rj);
    }
    mag = amag + Fp<G>::abs(t2) + Fp<G>::abs(t3) + Fp<G>::abs(t4);
    return alg + t2 + t3 + t4;
}

// Rounding bounds on the cancellation M/|B| of x_terms.  FP32 lanes beyond kXCancel32
// refine the R_F term in FP64 (the algebraic terms are FP64 already; the R_J terms are
// small where the terms cancel, at small z), which leaves an FP64-sized error in every
// large term.  Lanes beyond kXCancel64 (none on the workloads: the matter-poor open
// cosmologies of the non-flat workload reach ~300 at z = 1e-3, where the real root of Q
// is ~ -15 and the terms are ~r0^2) take the Gauss-Legendre quadrature of eq. 2.5.
constexpr double kXCancel32 = 8.0;
constexpr double kXCancel64 = 1024.0;
enum { kXRouteCarlson = 0, kXRouteFp64 = 1, kXRouteQuad = 2 };

// X / (c/H0) for one lane; route: one of kXRoute* (1: the FP32 lane's R_F term refined
// in FP64).
template <typename T, bool PAIR> __device__ T x_hat(const CosmoRec &r, T z, int &route) {
    route = kXRouteCarlson;
    const double zd = (double)z;
    double mag, B;
    XRf<double> xr;
    if (sizeof(T) == 4) {
        B = x_terms<float, double, PAIR>(r, zd, mag, xr);
        if (!(mag <= kXCancel32 * __builtin_fabs(B))) {
            route = kXRouteFp64;
            B += r.d.xc2 * rf_s<double, PAIR>(xr.V0, xr.va, xr.vb) - xr.t2;
        }
    } else {
        B = x_terms<double, double, PAIR>(r, zd, mag, xr);
    }
    if (mag <= kXCancel64 * __builtin_fabs(B)) return T(r.d.pre * zd * B);
    route = kXRouteQuad;
    T v, gd[3];
    gl_integral<T, PAIR>(lane_of<T>(r), z, 2, false, v, gd);
    return v;
}

// Curvature transform: S = sinn(chi) (sec. 2.1.1; sinh for Ok > 0, sin for Ok < 0),
// C = dS/dchi, dS = dS/dOk.  The power series in t = Ok chi^2 (one entire function
// for both signs of Ok) is used for |t| < 1, where its terms stay below one (no
// cancellation in S or C) and N terms reach the type's precision; the closed forms
// beyond.
template <typename T>
__device__ __forceinline__ void sinn(T chi, T ok, T sk, T &S, T &C, T &dS) {
    const T t = ok * chi * chi;
    if (Fp<T>::abs(t) < T(1)) {
        // first omitted terms at |t| = 1: FP64 (N = 10) below 1e-20; FP32 (N = 4)
        // 2.5e-8 in S/chi, 2.8e-7 in C and 7.5e-7 relative in dS (C and dS enter only
        // derivatives)
        constexpr int N = sizeof(T) == 4 ? 4 : 10;
        // u(t) = S/chi = sum a_n t^n with a_n = 1/(2n+1)!, and u'(t) from the same
        // Horner pass (one set of coefficients): C = dS/dchi = u + 2 t u' and
        // dS/dOk = chi^3 u'
        T a[N + 1];
        a[0] = T(1);
#pragma unroll
        for (int n = 1; n <= N; ++n) a[n] = a[n - 1] / T((2 * n) * (2 * n + 1));
        T u = kc<T>(a[N]), du = T(0);
#pragma unroll
        for (int n = N - 1; n >= 0; --n) {
            du = du * t + u;
            u = u * t + (n == 0 ? T(1) : kc<T>(a[n]));
        }
        S = chi * u;
        C = u + T(2) * t * du;
        dS = chi * chi * chi * du;
        return;
    }
    if (ok > T(0)) {
        T e = Fp<T>::exp_fast(sk * chi), ie = Fp<T>::rcp(e);
        S = T(0.5) * (e - ie) * Fp<T>::rcp(sk);
        C = T(0.5) * (e + ie);
    } else {
        T sn;
        sincos_red(sk * chi, sn, C);
        S = sn * Fp<T>::rcp(sk);
    }
    dS = (chi * C - S) * Fp<T>::rcp(T(2) * ok);
}

// Comoving-volume factor G(chi) = int_0^chi sinn(u)^2 du (all-sky comoving volume
// V_C = 4 pi D_H^3 G, sec. 2.1: dV_C = 4 pi D_M^2 dD_C) and dG/dOk at fixed chi.
// With t = Ok chi^2 the series G / chi^3 = sum_{n>=1} 2^(2n-1) t^(n-1) / (2n+1)! (one
// entire function for both signs of Ok) is used for |t| < 1; beyond, the closed forms
// with a = sqrt|Ok|, s2, c2 = sinh, cosh (Ok > 0) or sin, cos (Ok < 0) of 2 a chi and
// h = s2 / (2a):  G = +-(h - chi) / (2|Ok|),  dG/dOk = h'/(4 |Ok|^(3/2)) - G/Ok with
// h' = dh/da = chi c2 / a - s2 / (2 a^2).
template <typename T>
__device__ __forceinline__ void vol_g(T chi, T ok, T sk, T &G, T &dG) {
    const T chi2 = chi * chi;
    const T t = ok * chi2;
    if (Fp<T>::abs(t) < T(1)) {
        // first omitted term at |t| = 1, relative to G/chi^3 = 1/3: 1.6e-18 (FP64, N = 11),
        // 2.8e-10 (FP32, N = 7)
        constexpr int N = sizeof(T) == 4 ? 7 : 11;
        T c[N + 1];
        double inv_fact = 1.0 / 6.0, p2 = 2.0; // 1/(2n+1)!, 2^(2n-1) at n = 1
        c[0] = T(0);
#pragma unroll
        for (int n = 1; n <= N; ++n) {
            c[n] = T(p2 * inv_fact);
            inv_fact /= double((2 * n + 2) * (2 * n + 3));
            p2 *= 4.0;
        }
        T g = T(0), d = T(0);
#pragma unroll
        for (int n = N; n >= 1; --n) {
            g = g * t + c[n];
            if (n >= 2) d = d * t + T(n - 1) * c[n];
        }
        G = chi2 * chi * g;
        dG = chi2 * chi2 * chi * d;
        return;
    }
    const T a = sk, x2 = T(2) * a * chi;
    T s2, c2;
    if (ok > T(0)) {
        const T e = Fp<T>::exp_fast(x2), ie = Fp<T>::rcp(e);
        s2 = T(0.5) * (e - ie);
        c2 = T(0.5) * (e + ie);
    } else {
        sincos_red(x2, s2, c2);
    }
    const T ia = Fp<T>::rcp(a), aok = Fp<T>::abs(ok);
    const T h = T(0.5) * s2 * ia;
    G = (ok > T(0) ? h - chi : chi - h) * Fp<T>::rcp(T(2) * aok);
    const T hp = chi * c2 * ia - T(0.5) * s2 * ia * ia;
    dG = hp * Fp<T>::rcp(T(4) * aok * a) - G * Fp<T>::rcp(ok);
}

// Observable from chi/D_H for the comoving-distance family.  Also returns the
// partials needed by the adjoint: dout/dchi, dout/dOk at fixed chi, dout/dz at
// fixed chi, dout/dH0.
template <typename T>
__device__ __forceinline__ T observable(int kind, const LaneConst<T> &k, T chi, T z, T H0inv,
                                        T &d_chi, T &d_ok, T &d_z, T &d_h) {
    if (kind == COSMO_DC) {
        T v = k.dh * chi;
        d_chi = k.dh; d_ok = T(0); d_z = T(0); d_h = -v * H0inv;
        return v;
    }
    T S, C, dS;
    sinn(chi, k.ok, k.sk, S, C, dS);
    const T x = T(1) + z;
    if (kind == COSMO_VC) {
        // V_C = 4 pi D_H^3 G(chi): dV/dchi = 4 pi D_H^3 sinn(chi)^2
        T G, dG;
        vol_g(chi, k.ok, k.sk, G, dG);
        const T v4 = T(12.566370614359172) * k.dh * k.dh * k.dh;
        const T v = v4 * G;
        d_chi = v4 * S * S; d_ok = v4 * dG; d_z = T(0); d_h = T(-3) * v * H0inv;
        return v;
    }
    if (kind == COSMO_DM) {
        T v = k.dh * S;
        d_chi = k.dh * C; d_ok = k.dh * dS; d_z = T(0); d_h = -v * H0inv;
        return v;
    }
    if (kind == COSMO_DA) {
        T ix = Fp<T>::rcp(x);
        T v = k.dh * S * ix;
        d_chi = k.dh * C * ix; d_ok = k.dh * dS * ix; d_z = -v * ix; d_h = -v * H0inv;
        return v;
    }
    const T DL = x * k.dh * S;
    if (kind == COSMO_DL) {
        d_chi = x * k.dh * C; d_ok = x * k.dh * dS; d_z = k.dh * S; d_h = -DL * H0inv;
        return DL;
    }
    // COSMO_MU: 5 log10(D_L / Mpc) + 25 (fn. 22)
    const T k5 = T(2.1714724095162591); // 5 / ln 10
    const T u = k5 * Fp<T>::rcp(S);
    d_chi = C * u; d_ok = dS * u; d_z = k5 * Fp<T>::rcp(x); d_h = -k.k5hinv;
    return T(5) * Fp<T>::log10_fast(DL) + T(25);
}

// E(z) from eq. 2.2 (for the fundamental-theorem z-derivatives) and its inverse
template <typename T> __device__ __forceinline__ T E2z(const LaneConst<T> &k, T z) {
    const T x = T(1) + z;
    const T x2 = x * x;
    return (k.Or * x2 + k.Om * x + k.ok) * x2 + k.OL;
}
template <typename T> __device__ __forceinline__ T Ez(const LaneConst<T> &k, T z) { return Fp<T>::sqrt(E2z(k, z)); }
template <typename T> __device__ __forceinline__ T iEz(const LaneConst<T> &k, T z) { return Fp<T>::rsqrt(E2z(k, z)); }

// ---------------------------------------------------------------- adjoint
// Gradient of chi/D_H with respect to the per-cosmology root parameters
// (sigma, rho_0, rho_1[, rho_2]), by the chain rule through the Carlson
// arguments: dR_F/d(U_m^2) = -R_D(., ., U_m^2)/6 (eq. 2.10).
template <typename T, bool PAIR> struct ChiGrad {
    T chi;
    T dsig, dr0, dr1re, dr1im, dr2; // the partials divided by kr (one factor shared by all four)
    T kr;
    T iE; // 1/E(z), from the lane's geometry (E^2 = beta Xt^2 X_0^2 |X_1^2|^2)
};

template <typename T, bool PAIR>
__device__ __forceinline__ void chi_grad(const LaneConst<T> &k, T z, ChiGrad<T, PAIR> &o) {
    Geo<T, PAIR> g;
    build_u<T, PAIR, true>(k, z, g);
    T rf, rdx, rdz;
    cx<T> rdy;
    // the R_D outputs as -R_D/3 (rs), the factor of G_m below
    rfd_s<T, PAIR>(g.U0 * g.U0, g.va, g.vb, rf, rdx, rdy, rdz, T(-1.0 / 3.0));
    const T scale = k.pre2 * z;
    o.chi = scale * rf;
    o.iE = k.pre * g.iXprod;
    o.kr = scale * T(-0.5);
    // G_m = dR_F/dU_m = -U_m R_D(., ., U_m^2)/3 ; a_m = G_m T1_m, b_m = G_m T2_m
    const T G0 = g.U0 * rdx;
    const T a0 = G0 * g.T1_0, b0 = G0 * g.T2_0;
    // derivative of X_n, Y_n in rho_n: -1/(2 X_n), -1/(2 Y_n); of Xt, Yt in sigma: -x/(2 Xt)
    if (PAIR) {
        cx<T> G1 = mkc(g.U1re, g.U1im) * rdy;
        cx<T> a1 = G1 * mkc(g.T1_1re, g.T1_1im), b1 = G1 * mkc(g.T2_1re, g.T2_1im);
        const T A = a0 + T(2) * a1.re, B = b0 + T(2) * b1.re;
        o.dsig = ((T(1) + z) * A * g.iXt2 + B * k.iyt2);
        o.dr0 = ((a0 + B - b0) * g.iX02 + (b0 + A - a0) * k.iw0);
        const cx<T> iX1sq = mkc(g.iX1re, g.iX1im);
        const cx<T> iW1 = mkc(k.iw1re, k.iw1im);
        // (a1 + B - b1)/X1^2 + (b1 + A - a1)/W1
        cx<T> d1 = (a1 + B - b1) * iX1sq + (b1 + A - a1) * iW1;
        o.dr1re = d1.re;
        o.dr1im = d1.im;
        o.dr2 = T(0);
    } else {
        const T G1 = g.U1re * rdy.re, G2 = g.U2 * rdz;
        const T a1 = G1 * g.T1_1re, b1 = G1 * g.T2_1re, a2 = G2 * g.T1_2, b2 = G2 * g.T2_2;
        const T A = a0 + a1 + a2, B = b0 + b1 + b2;
        o.dsig = ((T(1) + z) * A * g.iXt2 + B * k.iyt2);
        o.dr0 = ((a0 + B - b0) * g.iX02 + (b0 + A - a0) * k.iw0);
        o.dr1re = ((a1 + B - b1) * g.iX1re + (b1 + A - a1) * k.iw1re);
        o.dr2 = ((a2 + B - b2) * g.iX2 + (b2 + A - a2) * k.iw2);
        o.dr1im = T(0);
    }
}

// Chain from dF/dV_m (V_m = U_m^2) to the root parameters through the U-products:
// with G_m = dF/dV_m 2 U_m, a_m = G_m T1_m, b_m = G_m T2_m, A = sum a, B = sum b:
//   dF/dsigma += -1/2 [ x2 A / Xt^2 + B / Yt^2 ],
//   dF/drho_n += -1/2 [ (a_n + B - b_n)/X_n^2 + (b_n + A - a_n)/Y_n^2 ].
// For PAIR the slot-1 quantities are complex and slot 2 is their conjugate.
template <typename T, bool PAIR>
__device__ __forceinline__ void u_chain(const LaneConst<T> &k, const Geo<T, PAIR> &g, T z, T dV0, cx<T> dV1,
                                        T dV2, T &dsig, T &dr0, cx<T> &dr1, T &dr2) {
    const T G0 = dV0 * T(2) * g.U0;
    const T a0 = G0 * g.T1_0, b0 = G0 * g.T2_0;
    if (PAIR) {
        cx<T> G1 = dV1 * mkc(g.U1re, g.U1im) * T(2);
        cx<T> a1 = G1 * mkc(g.T1_1re, g.T1_1im), b1 = G1 * mkc(g.T2_1re, g.T2_1im);
        const T A = a0 + T(2) * a1.re, B = b0 + T(2) * b1.re;
        dsig += T(-0.5) * ((T(1) + z) * A * Fp<T>::rcp(g.Xt2) + B * k.iyt2);
        dr0 += T(-0.5) * ((a0 + B - b0) * Fp<T>::rcp(g.X02) + (b0 + A - a0) * k.iw0);
        cx<T> iX1sq = crcp(mkc(z + k.w1re, k.w1im));
        const cx<T> iW1 = mkc(k.iw1re, k.iw1im);
        dr1 = dr1 + ((a1 + B - b1) * iX1sq + (b1 + A - a1) * iW1) * T(-0.5);
    } else {
        const T G1 = dV1.re * T(2) * g.U1re, G2 = dV2 * T(2) * g.U2;
        const T a1 = G1 * g.T1_1re, b1 = G1 * g.T2_1re, a2 = G2 * g.T1_2, b2 = G2 * g.T2_2;
        const T A = a0 + a1 + a2, B = b0 + b1 + b2;
        dsig += T(-0.5) * ((T(1) + z) * A * Fp<T>::rcp(g.Xt2) + B * k.iyt2);
        dr0 += T(-0.5) * ((a0 + B - b0) * Fp<T>::rcp(g.X02) + (b0 + A - a0) * k.iw0);
        dr1.re += T(-0.5) * ((a1 + B - b1) * Fp<T>::rcp(z + k.w1re) + (b1 + A - a1) * k.iw1re);
        dr2 += T(-0.5) * ((a2 + B - b2) * Fp<T>::rcp(z + k.w2) + (b2 + A - a2) * k.iw2);
    }
}

// Gradient of t/(1/H0) (eq. 3.8 / B.2 in the normalised form of t_hat) with respect
// to (sigma, rho_0, rho_1[, rho_2]) at fixed beta:
//   B = (dz^2/3) P3 R_J(V, W) + R_C(S, Q) + sigma R_F(V),  t_hat = beta^(-1/2) 2 dz B.
// Carlson derivatives: dR_F/dV_m = -R_D(., ., V_m)/6 (eq. 2.10); dR_J/dV_m =
// (R_J - R_D(., ., V_m)) / (2 (W - V_m)) (eq. 2.11); dR_J/dW from Euler's relation
// for the degree -3/2 homogeneous R_J (W dR_J/dW = -3/2 R_J - sum V_m dR_J/dV_m);
// dR_C(S, Q)/dS = -R_D(Q, Q, S)/6 and Q dR_C/dQ = -R_C/2 - S dR_C/dS.
template <typename T, bool PAIR> struct TGrad {
    T t, dsig, dr0, dr1re, dr1im, dr2;
};

template <typename T, bool PAIR>
__device__ void t_grad(const CosmoRec &r, T z, TGrad<T, PAIR> &o) {
    const LaneConst<T> &k = lane_of<T>(r);
    TArgs<T, PAIR> ta;
    t_args<T, PAIR>(r, z, ta);
    const Geo<T, PAIR> &g = ta.g;
    const T V0 = ta.V0, W = ta.W, Qv = ta.Q, S = ta.S;
    const T z2 = z * z, x2 = T(1) + z;
    const T C5 = k.c5;
    const T iD = Fp<T>::rcp(k.yt2 * g.Xt2);
    T rf, rj, rdx, rdz;
    cx<T> rdy;
    rfjd_s<T, PAIR>(V0, g.va, g.vb, W, rf, rj, rdx, rdy, rdz);
    const T rc = rc_r(S, Qv);
    const T dRC_S = rd_last_x<T, false>(S, Qv, Qv) * T(-1.0 / 6.0); // -R_D(Q, Q, S)/6
    const T dRC_Q = (T(-0.5) * rc - S * dRC_S) * Fp<T>::rcp(Qv);
    const T P3 = k.pre3;
    const T c3 = z2 * T(1.0 / 3.0) * P3;
    // R_J partials in its three triple arguments (eq. 2.11); W - V0 = dz^2 C5 exactly
    const T dJ0 = (rj - rdx) * Fp<T>::rcp(T(2) * z2 * C5);
    cx<T> dJ1;
    T dJ2 = T(0), sumVdJ;
    if (PAIR) {
        dJ1 = (mkc(rj, T(0)) - rdy) * crcp(mkc(W - g.va, -g.vb) * T(2));
        sumVdJ = V0 * dJ0 + T(2) * (g.va * dJ1.re - g.vb * dJ1.im);
    } else {
        dJ1 = mkc((rj - rdy.re) * Fp<T>::rcp(T(2) * (W - g.va)), T(0));
        dJ2 = (rj - rdz) * Fp<T>::rcp(T(2) * (W - g.vb));
        sumVdJ = V0 * dJ0 + g.va * dJ1.re + g.vb * dJ2;
    }
    const T dJW = (T(-1.5) * rj - sumVdJ) * Fp<T>::rcp(W);
    const T dRC_sum = dRC_S + dRC_Q; // S = Q - dz^2 Rp moves with Q
    const T dB_dW = c3 * dJW + dRC_sum * x2 * iD;
    const T dB_dV0 = c3 * dJ0 - k.sigma * rdx * T(1.0 / 6.0) + dB_dW;
    const cx<T> dB_dV1 = dJ1 * c3 - rdy * (k.sigma * T(1.0 / 6.0));
    const T dB_dV2 = PAIR ? T(0) : c3 * dJ2 - k.sigma * rdz * T(1.0 / 6.0);
    // explicit dependence of P3, C5, Rp and Q on sigma and the roots
    const T s = k.sigma;
    const cx<T> om1 = mkc(T(1) - s * k.r1re, -s * k.r1im);
    const cx<T> om2 = PAIR ? conj(om1) : mkc(T(1) - s * k.r2, T(0));
    const T om0 = T(1) - s * k.r0;
    const cx<T> r1 = mkc(k.r1re, k.r1im);
    const cx<T> r2 = PAIR ? conj(r1) : mkc(k.r2, T(0));
    const T om12 = (om1 * om2).re;
    // rho_1 om_2 + rho_2 om_1 (real in both root structures)
    const T r1o2_r2o1 = (r1 * om2).re + (r2 * om1).re;
    const T dP3_ds = -(k.r0 * om12 + om0 * r1o2_r2o1);
    const T dC5_ds = -k.r0 * r1o2_r2o1;
    const T dQ_ds = Qv * (k.iyt2 + x2 * Fp<T>::rcp(g.Xt2));
    T dsig = (z2 * T(1.0 / 3.0)) * rj * dP3_ds + dB_dW * z2 * dC5_ds + dRC_sum * dQ_ds + rf;
    // rho_0
    T dr0 = (z2 * T(1.0 / 3.0)) * rj * (-s * om12) + dB_dW * z2 * om12 + dRC_S * (-z2 * (r1 * r2).re);
    // rho_1 (complex for PAIR)
    cx<T> dr1 = (om0 * om2 * (-s)) * ((z2 * T(1.0 / 3.0)) * rj) + om2 * (-s * k.r0) * (dB_dW * z2) +
                (r2 * k.r0) * (-z2 * dRC_S);
    T dr2 = PAIR ? T(0)
                 : ((z2 * T(1.0 / 3.0)) * rj * (-s * om0 * om1.re) + dB_dW * z2 * (-s * om1.re * k.r0) +
                    dRC_S * (-z2 * k.r0 * k.r1re));
    // through the Carlson arguments V_m(U_m)
    u_chain<T, PAIR>(k, g, z, dB_dV0, dB_dV1, dB_dV2, dsig, dr0, dr1, dr2);
    const T scale = k.pre2 * z;
    const T Bv = c3 * rj + rc + s * rf;
    o.t = scale * Bv;
    o.dsig = scale * dsig;
    o.dr0 = scale * dr0;
    o.dr1re = scale * dr1.re;
    o.dr1im = scale * dr1.im;
    o.dr2 = scale * dr2;
}

} // namespace cosmo
