// between.hpp -- observables between two redshifts z1 and z2 (either order), and to
// an infinite upper limit: chi(z1, z2) (eq. 3.7), the transverse and angular
// diameter distances between the two (sec. 2.1: curvature transform of chi(z1, z2),
// and D_M(z1, z2)/(1 + z2)), and the time coordinate t(z1, z2) (eq. 3.8; with
// z2 = inf the age t(z1, inf) of sec. 2.1).
//
// The one-sided kernels fold the lower limit x1 = 1 into per-cosmology constants
// (the Y's of build_u); here both limits are per lane.  A limit is described by the
// square roots of the factors of P(x) = beta (1 - sigma x) Q(x) at x = 1 + z.  At
// x -> infinity each square root grows like sqrt(x): the limit side holds them
// divided by sqrt(x) (sqrt(1 - sigma x)/sqrt(x) -> sqrt(-sigma), sqrt(x - rho)/sqrt(x)
// -> 1), which scales every U_m by 1/x2; by the homogeneity of R_F (degree -1/2),
// R_J (-3/2) and R_C (-1/2) the prefactors 2 dz, dz^2 then become 2 and 1.
#pragma once

#include "adjoint.hpp"

namespace cosmo {

// One limit: t = sqrt(1 - sigma x), n_m = sqrt(x - rho_m) (PAIR: n_1 complex, with
// |n_1|^2 = |x - rho_1| in n1abs), x itself; at infinity the scaled values and x = 1.
template <typename T, bool PAIR> struct Side {
    T t, t2, n0, n1re, n1im, n1abs, n2, x;
};

template <typename T, bool PAIR> __device__ __forceinline__ void side_at(const LaneConst<T> &k, T z, Side<T, PAIR> &s) {
    s.x = T(1) + z;
    s.t2 = k.yt2 - k.sigma * z; // 1 - sigma (1 + z)
    s.t = Fp<T>::sqrt(s.t2);
    s.n0 = Fp<T>::sqrt(z + k.w0);
    if (PAIR) {
        T ab;
        const cx<T> n1 = csqrt(mkc(z + k.w1re, k.w1im), ab);
        s.n1re = n1.re; s.n1im = n1.im; s.n1abs = ab;
        s.n2 = T(0);
    } else {
        s.n1re = Fp<T>::sqrt(z + k.w1re);
        s.n1im = T(0); s.n1abs = T(0);
        s.n2 = Fp<T>::sqrt(z + k.w2);
    }
}

template <typename T, bool PAIR> __device__ __forceinline__ void side_inf(const LaneConst<T> &k, Side<T, PAIR> &s) {
    s.x = T(1);
    s.t2 = -k.sigma; // sigma <= 0 (sigma < 0 with radiation, 0 without)
    s.t = k.tinf;
    s.n0 = T(1);
    s.n1re = T(1); s.n1im = T(0); s.n1abs = T(1);
    s.n2 = T(1);
}

// The three Carlson arguments U_m^2 between limits a (upper) and b (lower): the U_m of
// eq. 3.7 in the normalised form of build_u, with the lower limit's square roots per
// lane.  Returns V0 = U_0^2, (va, vb) as build_u, and U_0, U_1 (re, im) [PAIR] or
// U_1, U_2 for the time coordinate's W.
template <typename T, bool PAIR> struct Args2 {
    T V0, va, vb, U0, U1re, U1im, U2;
};

template <typename T, bool PAIR>
__device__ __forceinline__ void args_between(const Side<T, PAIR> &a, const Side<T, PAIR> &b, Args2<T, PAIR> &o) {
    if (PAIR) {
        // U_0 = ta n0a |n1b|^2 + tb n0b |n1a|^2 ;  U_1 = ta n0b w + tb n0a conj(w), w = n1a conj(n1b)
        o.U0 = a.t * a.n0 * b.n1abs + b.t * b.n0 * a.n1abs;
        const cx<T> w = mkc(a.n1re, a.n1im) * mkc(b.n1re, -b.n1im);
        const T cA = a.t * b.n0, cB = b.t * a.n0;
        o.U1re = (cA + cB) * w.re;
        o.U1im = (cA - cB) * w.im;
        o.U2 = T(0);
        o.va = o.U1re * o.U1re - o.U1im * o.U1im;
        o.vb = T(2) * o.U1re * o.U1im;
    } else {
        o.U0 = a.t * a.n0 * b.n1re * b.n2 + b.t * b.n0 * a.n1re * a.n2;
        o.U1re = a.t * a.n1re * b.n0 * b.n2 + b.t * b.n1re * a.n0 * a.n2;
        o.U1im = T(0);
        o.U2 = a.t * a.n2 * b.n0 * b.n1re + b.t * b.n2 * a.n0 * a.n1re;
        o.va = o.U1re * o.U1re;
        o.vb = o.U2 * o.U2;
    }
    o.V0 = o.U0 * o.U0;
}

// ZINF: the upper limit is known to be infinite on every lane (otherwise tested per lane).
template <typename T, bool PAIR, bool ZINF = false>
__device__ __forceinline__ void sides(const LaneConst<T> &k, T z1, T z2, Side<T, PAIR> &a, Side<T, PAIR> &b, T &dz) {
    side_at<T, PAIR>(k, z1, b);
    if (ZINF || z2 == Fp<T>::inf()) {
        side_inf<T, PAIR>(k, a);
        dz = T(1);
    } else {
        side_at<T, PAIR>(k, z2, a);
        dz = z2 - z1;
    }
}

// chi(z1, z2) / D_H, eq. 3.7 (z2 = inf: the limit form).
template <typename T, bool PAIR> __device__ __forceinline__ T chi_between(const LaneConst<T> &k, T z1, T z2) {
    Side<T, PAIR> a, b;
    T dz;
    sides<T, PAIR>(k, z1, z2, a, b, dz);
    Args2<T, PAIR> u;
    args_between<T, PAIR>(a, b, u);
    return k.pre2 * dz * rf_s<T, PAIR>(u.V0, u.va, u.vb);
}

// Arguments of t(z1, z2) (eq. 3.8 in the normalised form of t_args_in), in the
// precision Q: W5 = U_j^2 + dz^2 c5_j (the least-cancelling root slot j, as in
// t_args_in), Q5 = x1 x2 W5 / ((1 - sigma x1)(1 - sigma x2)), S5 = Q5 - dz^2 rho0 rho1
// rho2.  At infinity x2/(1 - sigma x2) -> -1/sigma: the scaled side has x = 1 and
// t2 = -sigma, so the same expressions hold; without radiation Q5 is infinite there
// (R_C -> 0), flagged by rc_zero.
template <typename Q, bool PAIR> struct TArgs2 {
    Args2<Q, PAIR> u;
    Q dz, W, Qv, S;
    bool rc_zero;
};

template <typename Q, bool PAIR>
__device__ __forceinline__ void t_args_sides(const LaneConst<Q> &k, const Side<Q, PAIR> &a, const Side<Q, PAIR> &b,
                                             Q dz, TArgs2<Q, PAIR> &o) {
    o.dz = dz;
    args_between<Q, PAIR>(a, b, o.u);
    const Q d2 = o.dz * o.dz;
    Q W = o.u.V0 + d2 * k.c5;
    Q m0 = o.u.V0 + Fp<Q>::abs(d2 * k.c5);
    const Q w1 = o.u.va + d2 * k.c5b;
    const Q m1 = (PAIR ? o.u.U1re * o.u.U1re + o.u.U1im * o.u.U1im : o.u.va) + Fp<Q>::abs(d2 * k.c5b);
    if (m1 < m0) { W = w1; m0 = m1; }
    if (!PAIR) {
        const Q w2 = o.u.vb + d2 * k.c5c, m2 = o.u.vb + Fp<Q>::abs(d2 * k.c5c);
        if (m2 < m0) W = w2;
    }
    o.W = W;
    o.rc_zero = a.t2 == Q(0);
    o.Qv = o.rc_zero ? Q(1) : a.x * b.x * W * Fp<Q>::rcp(a.t2 * b.t2);
    o.S = o.Qv - d2 * k.rprod;
}

template <typename Q, bool PAIR, bool ZINF = false>
__device__ __forceinline__ void t_args_between(const LaneConst<Q> &k, Q z1, Q z2, TArgs2<Q, PAIR> &o) {
    Side<Q, PAIR> a, b;
    Q dz;
    sides<Q, PAIR, ZINF>(k, z1, z2, a, b, dz);
    t_args_sides<Q, PAIR>(k, a, b, dz, o);
}

// ---------------------------------------------------------------- limits with reciprocals
// (the adjoints' chain, and the FP32 time coordinate's FP64 arguments)
// One limit with the reciprocals the chain needs (square roots as v rsqrt(v), as in
// build_u's INV form): it2 = 1/t^2, i0 = 1/n0^2, i1 = 1/n1^2 (PAIR: the complex
// 1/(x - rho_1)), i2 = 1/n2^2, and ie = 1/(t n0 |n1|^2) (PAIR) or 1/(t n0 n1 n2), so that
// 1/E = beta^(-1/2) ie at that limit.  At infinity the scaled side does not depend on
// the roots: its reciprocal squares are zero, and with x = 1 the sigma term of the
// chain (d t^2/d sigma = -x) holds for t^2 = -sigma.
template <typename T, bool PAIR> struct SideG {
    Side<T, PAIR> s;
    T it2, i0, i1re, i1im, i2, ie;
};

template <typename T, bool PAIR> __device__ __forceinline__ void side_at_g(const LaneConst<T> &k, T z, SideG<T, PAIR> &o) {
    Side<T, PAIR> &s = o.s;
    s.x = T(1) + z;
    s.t2 = k.yt2 - k.sigma * z;
    const T v0 = z + k.w0;
    const T rt = Fp<T>::rsqrt(s.t2), r0 = Fp<T>::rsqrt(v0);
    s.t = s.t2 * rt; o.it2 = rt * rt;
    s.n0 = v0 * r0; o.i0 = r0 * r0;
    if (PAIR) {
        T ab, iab;
        const cx<T> w = mkc(z + k.w1re, k.w1im);
        const cx<T> n1 = csqrt_inv(w, ab, iab);
        s.n1re = n1.re; s.n1im = n1.im; s.n1abs = ab;
        const T i2v = iab * iab;
        o.i1re = w.re * i2v; o.i1im = -w.im * i2v;
        s.n2 = T(0); o.i2 = T(0);
        o.ie = rt * r0 * iab;
    } else {
        const T v1 = z + k.w1re, v2 = z + k.w2;
        const T r1 = Fp<T>::rsqrt(v1), r2 = Fp<T>::rsqrt(v2);
        s.n1re = v1 * r1; s.n1im = T(0); s.n1abs = T(0);
        s.n2 = v2 * r2;
        o.i1re = r1 * r1; o.i1im = T(0); o.i2 = r2 * r2;
        o.ie = rt * r0 * r1 * r2;
    }
}

template <typename T, bool PAIR> __device__ __forceinline__ void side_inf_g(const LaneConst<T> &k, SideG<T, PAIR> &o) {
    side_inf<T, PAIR>(k, o.s);
    o.it2 = k.itinf2; // 1/(-sigma): infinite without radiation (see chi_grad_between)
    o.i0 = T(0); o.i1re = T(0); o.i1im = T(0); o.i2 = T(0);
    o.ie = T(0);
}

// FP64 square root of x to about 1e-14 relative from the FP32 root s = xf rt (rt the FP32
// reciprocal square root of xf = (float)x) and one Newton step whose correction
// (x - s^2)/(2 s) is formed in FP32: the FP32 root is within ~1e-7, so the step leaves
// ~1e-14.
__device__ __forceinline__ double sqrt_nr(double x, float s, float rt) {
    const double sd = (double)s;
    return sd + (double)((float)__builtin_fma(-sd, sd, x) * (0.5f * rt));
}

// One finite limit of an FP32 lane of the time coordinate: the square roots as FP32 values
// with the reciprocals of the chain (side_at_g's, in o) and, refined by sqrt_nr, in FP64
// (d) for the FP64 arguments of eq. 3.8 -- one reciprocal square root per factor.
template <bool PAIR>
__device__ __forceinline__ void side_at_mixed(const LaneConst<double> &kd, const LaneConst<float> &kf, float z,
                                              Side<double, PAIR> &d, SideG<float, PAIR> &o) {
    Side<float, PAIR> &s = o.s;
    const double zd = (double)z;
    d.x = 1.0 + zd;
    s.x = 1.0f + z;
    d.t2 = kd.yt2 - kd.sigma * zd;
    s.t2 = (float)d.t2;
    const float rt = Fp<float>::rsqrt(s.t2);
    s.t = s.t2 * rt;
    o.it2 = rt * rt;
    d.t = sqrt_nr(d.t2, s.t, rt);
    const double v0 = zd + kd.w0;
    const float v0f = (float)v0, r0 = Fp<float>::rsqrt(v0f);
    s.n0 = v0f * r0;
    o.i0 = r0 * r0;
    d.n0 = sqrt_nr(v0, s.n0, r0);
    if (PAIR) {
        const double wre = zd + kd.w1re;
        const float wref = (float)wre;
        float ab, iab;
        const cx<float> n1 = csqrt_uim_inv(wref, kf.w1im2, kf.hw1im, kf.sw1im, ab, iab);
        s.n1re = n1.re; s.n1im = n1.im; s.n1abs = ab;
        const float i2v = iab * iab;
        o.i1re = wref * i2v; o.i1im = -kf.w1im * i2v;
        s.n2 = 0.0f; o.i2 = 0.0f;
        o.ie = rt * r0 * iab;
        // Newton step for the complex root: n1 + (w - n1^2) / (2 n1), with
        // 1/(2 n1) = conj(n1) / (2 |w|) and the residual in FP64
        const double nre = (double)n1.re, nim = (double)n1.im;
        const float rr = (float)__builtin_fma(-nre, nre, __builtin_fma(nim, nim, wre));
        const float ri = (float)__builtin_fma(-2.0 * nre, nim, kd.w1im);
        const float h = 0.5f * iab;
        d.n1re = nre + (double)((rr * n1.re + ri * n1.im) * h);
        d.n1im = nim + (double)((ri * n1.re - rr * n1.im) * h);
        d.n1abs = d.n1re * d.n1re + d.n1im * d.n1im;
        d.n2 = 0.0;
    } else {
        const double v1 = zd + kd.w1re, v2 = zd + kd.w2;
        const float v1f = (float)v1, v2f = (float)v2;
        const float r1 = Fp<float>::rsqrt(v1f), r2 = Fp<float>::rsqrt(v2f);
        s.n1re = v1f * r1; s.n1im = 0.0f; s.n1abs = 0.0f;
        s.n2 = v2f * r2;
        o.i1re = r1 * r1; o.i1im = 0.0f; o.i2 = r2 * r2;
        o.ie = rt * r0 * r1 * r2;
        d.n1re = sqrt_nr(v1, s.n1re, r1); d.n1im = 0.0; d.n1abs = 0.0;
        d.n2 = sqrt_nr(v2, s.n2, r2);
    }
}

// The FP64 arguments of eq. 3.8 for an FP32 lane (z2 = inf: the scaled side), with the
// FP32 sides of the chain in a (upper) and b (lower).
template <bool PAIR, bool ZINF>
__device__ __forceinline__ void t_args_mixed(const CosmoRec &r, float z1, float z2, TArgs2<double, PAIR> &o,
                                             SideG<float, PAIR> &a, SideG<float, PAIR> &b) {
    Side<double, PAIR> ad, bd;
    side_at_mixed<PAIR>(r.d, r.f, z1, bd, b);
    double dz;
    if (ZINF || z2 == Fp<float>::inf()) {
        side_inf<double, PAIR>(r.d, ad);
        side_inf_g<float, PAIR>(r.f, a);
        dz = 1.0;
    } else {
        side_at_mixed<PAIR>(r.d, r.f, z2, ad, a);
        dz = (double)z2 - (double)z1;
    }
    t_args_sides<double, PAIR>(r.d, ad, bd, dz, o);
}

// t(z1, z2) / (1/H0), eq. 3.8 (z2 = inf: the age t(z1, inf)).  The FP32 path forms
// the arguments in FP64 (square roots by sqrt_nr) and rounds them once.
template <typename T, bool PAIR, bool ZINF = false> __device__ __forceinline__ T t_between(const CosmoRec &r, T z1, T z2) {
    const LaneConst<T> &k = lane_of<T>(r);
    TArgs2<double, PAIR> ad;
    if constexpr (sizeof(T) == 4) {
        SideG<float, PAIR> a, b;
        t_args_mixed<PAIR, ZINF>(r, z1, z2, ad, a, b);
    } else {
        t_args_between<double, PAIR, ZINF>(r.d, z1, z2, ad);
    }
    const T V0 = T(ad.u.V0), va = T(ad.u.va), vb = T(ad.u.vb), W = T(ad.W);
    const T dz = T(ad.dz), d2 = dz * dz;
    T rf, rj;
    rfj_s<T, PAIR>(V0, va, vb, W, rf, rj);
    const T rc = ad.rc_zero ? T(0) : rc_r(T(ad.S), T(ad.Qv));
    return k.pre2 * dz * (d2 * T(1.0 / 3.0) * k.pre3 * rj + rc + k.sigma * rf);
}

// Observable KIND (COSMO_DC, COSMO_DM, COSMO_DA or COSMO_T) between z1 and z2.
template <typename T, int KIND, bool PAIR>
__device__ __forceinline__ T eval_between(const CosmoRec &r, T z1, T z2) {
    const LaneConst<T> &k = lane_of<T>(r);
    if (KIND == COSMO_T) {
        // the age t(z1, inf) on every lane of the wave: the upper side's constants fold
        if (__ballot(!(z2 == Fp<T>::inf())) == 0) return k.th * t_between<T, PAIR, true>(r, z1, z2);
        return k.th * t_between<T, PAIR>(r, z1, z2);
    }
    const T chi = chi_between<T, PAIR>(k, z1, z2);
    if (KIND == COSMO_DC) return k.dh * chi;
    T S, C, dS;
    sinn(chi, k.ok, k.sk, S, C, dS);
    if (KIND == COSMO_DM) return k.dh * S;
    return z2 == Fp<T>::inf() ? T(0) : k.dh * S * Fp<T>::rcp(T(1) + z2); // COSMO_DA
}


// ---------------------------------------------------------------- adjoint (D_C family)
// chi(z1, z2)/D_H and its partials in the root parameters (sigma, rho_0, rho_1 [re, im]
// or rho_1, rho_2) at fixed beta, through dR_F/d(U_m^2) = -R_D(., ., U_m^2)/6 (eq. 2.10)
// and the square roots of both limits (each U_m = T1_m + T2_m, T1 led by the upper
// limit's sqrt(1 - sigma x), T2 by the lower's):
//   d/dsigma  = -1/2 [x2 A / t2^2 + x1 B / t1^2],
//   d/drho_n  = -1/2 [(a_n + B - b_n) / (x2 - rho_n) + (b_n + A - a_n) / (x1 - rho_n)],
// a_m = G_m T1_m, b_m = G_m T2_m, G_m = dR_F/dU_m, A = sum a, B = sum b (the one-sided
// chi_grad with the lower limit per lane).  Also 1/E at both limits (0 at infinity).
// Without radiation the sigma partial diverges at an infinite upper limit (d chi/d Or0
// is -inf at Or0 = 0 there): it is returned as NaN.
template <typename T, bool PAIR> struct ChiGrad2 {
    T chi, dsig, dr0, dr1re, dr1im, dr2, iE1, iE2;
};

template <typename T, bool PAIR>
__device__ __forceinline__ void chi_grad_between(const LaneConst<T> &k, T z1, T z2, ChiGrad2<T, PAIR> &o) {
    SideG<T, PAIR> a, b;
    side_at_g<T, PAIR>(k, z1, b);
    const bool zinf = z2 == Fp<T>::inf();
    T dz;
    if (zinf) {
        side_inf_g<T, PAIR>(k, a);
        dz = T(1);
    } else {
        side_at_g<T, PAIR>(k, z2, a);
        dz = z2 - z1;
    }
    const Side<T, PAIR> &A_ = a.s, &B_ = b.s;
    T U0, va, vb, T1_0, T2_0;
    cx<T> U1, T1_1, T2_1;
    T U2 = T(0), T1_2 = T(0), T2_2 = T(0), T1_1r = T(0), T2_1r = T(0);
    if (PAIR) {
        T1_0 = A_.t * A_.n0 * B_.n1abs;
        T2_0 = B_.t * B_.n0 * A_.n1abs;
        const cx<T> w = mkc(A_.n1re, A_.n1im) * mkc(B_.n1re, -B_.n1im);
        T1_1 = w * (A_.t * B_.n0);
        T2_1 = conj(w) * (B_.t * A_.n0);
        U1 = T1_1 + T2_1;
        va = U1.re * U1.re - U1.im * U1.im;
        vb = T(2) * U1.re * U1.im;
    } else {
        T1_0 = A_.t * A_.n0 * B_.n1re * B_.n2;
        T2_0 = B_.t * B_.n0 * A_.n1re * A_.n2;
        T1_1r = A_.t * A_.n1re * B_.n0 * B_.n2;
        T2_1r = B_.t * B_.n1re * A_.n0 * A_.n2;
        T1_2 = A_.t * A_.n2 * B_.n0 * B_.n1re;
        T2_2 = B_.t * B_.n2 * A_.n0 * A_.n1re;
        U1 = mkc(T1_1r + T2_1r, T(0));
        U2 = T1_2 + T2_2;
        va = U1.re * U1.re;
        vb = U2 * U2;
    }
    U0 = T1_0 + T2_0;
    T rf, rdx, rdz;
    cx<T> rdy;
    rfd_s<T, PAIR>(U0 * U0, va, vb, rf, rdx, rdy, rdz, T(-1.0 / 3.0)); // -R_D/3
    const T scale = k.pre2 * dz;
    o.chi = scale * rf;
    o.iE1 = k.pre * b.ie;
    o.iE2 = k.pre * a.ie;
    const T h = scale * T(-0.5);
    const T G0 = U0 * rdx;
    const T a0 = G0 * T1_0, b0 = G0 * T2_0;
    if (PAIR) {
        const cx<T> G1 = U1 * rdy;
        const cx<T> a1 = G1 * T1_1, b1 = G1 * T2_1;
        const T Asum = a0 + T(2) * a1.re, Bsum = b0 + T(2) * b1.re;
        o.dsig = h * (A_.x * Asum * a.it2 + B_.x * Bsum * b.it2);
        o.dr0 = h * ((a0 + Bsum - b0) * a.i0 + (b0 + Asum - a0) * b.i0);
        const cx<T> d1 = (a1 + Bsum - b1) * mkc(a.i1re, a.i1im) + (b1 + Asum - a1) * mkc(b.i1re, b.i1im);
        o.dr1re = h * d1.re;
        o.dr1im = h * d1.im;
        o.dr2 = T(0);
    } else {
        const T G1 = U1.re * rdy.re, G2 = U2 * rdz;
        const T a1 = G1 * T1_1r, b1 = G1 * T2_1r, a2 = G2 * T1_2, b2 = G2 * T2_2;
        const T Asum = a0 + a1 + a2, Bsum = b0 + b1 + b2;
        o.dsig = h * (A_.x * Asum * a.it2 + B_.x * Bsum * b.it2);
        o.dr0 = h * ((a0 + Bsum - b0) * a.i0 + (b0 + Asum - a0) * b.i0);
        o.dr1re = h * ((a1 + Bsum - b1) * a.i1re + (b1 + Asum - a1) * b.i1re);
        o.dr2 = h * ((a2 + Bsum - b2) * a.i2 + (b2 + Asum - a2) * b.i2);
        o.dr1im = T(0);
    }
    if (zinf && k.sigma == T(0)) o.dsig = Fp<T>::nan();
}

// t(z1, z2)/(1/H0) and its partials in the root parameters (sigma, rho_0, rho_1 [re, im]
// or rho_1, rho_2) at fixed beta: eq. 3.8 between the two limits, differentiated as
// t_grad differentiates the one-sided form (R_F, R_J and R_C partials from eqs. 2.10 and
// 2.11, Euler's relation for R_J's last argument, R_C's homogeneity; the explicit sigma-
// and root-dependence of the coefficients), with the square roots of both limits in the
// chain through the U_m (as chi_grad_between) and Q5 = x1 x2 W5 / ((1 - sigma x1)(1 -
// sigma x2)), so dQ5/dsigma at fixed W5 = Q5 (x1/(1 - sigma x1) + x2/(1 - sigma x2)) (at
// an infinite upper limit the scaled side has x = 1 and 1 - sigma x -> -sigma).  The
// Carlson arguments are formed in FP64 on the FP32 path (as t_between); the chain's
// geometry in the lane precision.  Not for an infinite upper limit at small |sigma|
// (kAgeSigma32/64 below; the Leibniz route covers it).
// The age t(z, inf) through the chain: its sigma partials grow like powers of 1/|sigma|
// (the infinite side has 1 - sigma x -> -sigma) while d t/d Or0 stays finite, so the Or0
// component cancels, by ~|sigma|^(-1/2) (measured on the host build against the
// oracle: FP32 1e-4 relative at Or0 = 1e-5, FP64 6e-11 at Or0 = 1e-10).  Below these
// |sigma| the age takes the Leibniz route, whose Or0 derivative has no cancellation.
constexpr float kAgeSigma32 = 1e-4f;
constexpr double kAgeSigma64 = 1e-9;

template <typename T, bool PAIR> struct TGrad2 {
    T t, dsig, dr0, dr1re, dr1im, dr2, iE1, iE2;
};

template <typename T, bool PAIR, bool ZINF = false>
__device__ __forceinline__ void t_grad_between(const CosmoRec &r, T z1, T z2, TGrad2<T, PAIR> &o) {
    const LaneConst<T> &k = lane_of<T>(r);
    const bool zinf = ZINF || z2 == Fp<T>::inf();
    TArgs2<double, PAIR> ad;
    SideG<T, PAIR> a, b;
    if constexpr (sizeof(T) == 4) {
        t_args_mixed<PAIR, ZINF>(r, z1, z2, ad, a, b);
    } else {
        // the sides of the chain give the arguments' square roots (2 ulp)
        side_at_g<T, PAIR>(k, z1, b);
        if (zinf) side_inf_g<T, PAIR>(k, a);
        else side_at_g<T, PAIR>(k, z2, a);
        t_args_sides<double, PAIR>(r.d, a.s, b.s, zinf ? 1.0 : z2 - z1, ad);
    }
    const T V0 = T(ad.u.V0), va = T(ad.u.va), vb = T(ad.u.vb), W = T(ad.W), Qv = T(ad.Qv), S = T(ad.S);
    const T dz = T(ad.dz), d2 = dz * dz;
    o.iE1 = k.pre * b.ie;
    o.iE2 = k.pre * a.ie;
    const Side<T, PAIR> &A_ = a.s, &B_ = b.s;
    // the products making U_m: T1 led by the upper limit's sqrt(1 - sigma x), T2 by the lower's
    T U0, T1_0, T2_0, U2 = T(0), T1_2 = T(0), T2_2 = T(0);
    cx<T> U1, T1_1, T2_1;
    if (PAIR) {
        T1_0 = A_.t * A_.n0 * B_.n1abs;
        T2_0 = B_.t * B_.n0 * A_.n1abs;
        const cx<T> w = mkc(A_.n1re, A_.n1im) * mkc(B_.n1re, -B_.n1im);
        T1_1 = w * (A_.t * B_.n0);
        T2_1 = conj(w) * (B_.t * A_.n0);
    } else {
        T1_0 = A_.t * A_.n0 * B_.n1re * B_.n2;
        T2_0 = B_.t * B_.n0 * A_.n1re * A_.n2;
        T1_1 = mkc(A_.t * A_.n1re * B_.n0 * B_.n2, T(0));
        T2_1 = mkc(B_.t * B_.n1re * A_.n0 * A_.n2, T(0));
        T1_2 = A_.t * A_.n2 * B_.n0 * B_.n1re;
        T2_2 = B_.t * B_.n2 * A_.n0 * A_.n1re;
        U2 = T1_2 + T2_2;
    }
    U0 = T1_0 + T2_0;
    U1 = T1_1 + T2_1;
    T rf, rj, rdx, rdz;
    cx<T> rdy;
    rfjd_s<T, PAIR>(V0, va, vb, W, rf, rj, rdx, rdy, rdz);
    T rc = T(0), dRC_S = T(0), dRC_Q = T(0);
    if (!ad.rc_zero) {
        T rdq;
        rc_rd_r(S, Qv, rc, rdq);
        dRC_S = rdq * T(-1.0 / 6.0); // -R_D(Q, Q, S)/6
        dRC_Q = (T(-0.5) * rc - S * dRC_S) * Fp<T>::rcp(Qv);
    }
    const T c3 = d2 * T(1.0 / 3.0) * k.pre3;
    // R_J partials in its three triple arguments (eq. 2.11); W - V0 = dz^2 C5 exactly
    const T dJ0 = (rj - rdx) * Fp<T>::rcp(T(2) * d2 * k.c5);
    cx<T> dJ1;
    T dJ2 = T(0), sumVdJ;
    if (PAIR) {
        dJ1 = (mkc(rj, T(0)) - rdy) * crcp(mkc(W - va, -vb) * T(2));
        sumVdJ = V0 * dJ0 + T(2) * (va * dJ1.re - vb * dJ1.im);
    } else {
        dJ1 = mkc((rj - rdy.re) * Fp<T>::rcp(T(2) * (W - va)), T(0));
        dJ2 = (rj - rdz) * Fp<T>::rcp(T(2) * (W - vb));
        sumVdJ = V0 * dJ0 + va * dJ1.re + vb * dJ2;
    }
    const T dJW = (T(-1.5) * rj - sumVdJ) * Fp<T>::rcp(W);
    const T dRC_sum = dRC_S + dRC_Q;         // S = Q - dz^2 Rp moves with Q
    const T qw = ad.rc_zero ? T(0) : Qv * Fp<T>::rcp(W); // dQ/dW
    const T dB_dW = c3 * dJW + dRC_sum * qw;
    const T dB_dV0 = c3 * dJ0 - k.sigma * rdx * T(1.0 / 6.0) + dB_dW;
    const cx<T> dB_dV1 = dJ1 * c3 - rdy * (k.sigma * T(1.0 / 6.0));
    const T dB_dV2 = PAIR ? T(0) : c3 * dJ2 - k.sigma * rdz * T(1.0 / 6.0);
    // explicit dependence of P3, C5, Rp and Q on sigma and the roots (the coefficients
    // are per-cosmology constants of the set-up: tdp3 = dP3/dsigma, tdc5 = dC5/dsigma,
    // om1s12 = o1 o2, tso12 = -sigma o1 o2, tr12 = r1 r2, tq1..3 and, for three real roots,
    // tq4..6, with o_n = 1 - sigma r_n)
    const T dQ_ds = ad.rc_zero ? T(0) : Qv * (B_.x * b.it2 + A_.x * a.it2);
    const T jr = d2 * T(1.0 / 3.0) * rj, bw = dB_dW * d2, rs = -d2 * dRC_S;
    T dsig = jr * k.tdp3 + bw * k.tdc5 + dRC_sum * dQ_ds + rf;
    T dr0 = jr * k.tso12 + bw * k.om1s12 + rs * k.tr12;
    cx<T> dr1 = mkc(jr * k.tq1re + bw * k.tq2re + rs * k.tq3re, jr * k.tq1im + bw * k.tq2im + rs * k.tq3im);
    T dr2 = PAIR ? T(0) : jr * k.tq4 + bw * k.tq5 + rs * k.tq6;
    // through the Carlson arguments V_m = U_m^2, with both limits' square roots
    const T G0 = dB_dV0 * T(2) * U0;
    const T a0 = G0 * T1_0, b0 = G0 * T2_0;
    if (PAIR) {
        const cx<T> G1 = dB_dV1 * U1 * T(2);
        const cx<T> a1 = G1 * T1_1, b1 = G1 * T2_1;
        const T As = a0 + T(2) * a1.re, Bs = b0 + T(2) * b1.re;
        dsig += T(-0.5) * (A_.x * As * a.it2 + B_.x * Bs * b.it2);
        if (ZINF) { // the scaled side at infinity has zero reciprocal squares
            dr0 += T(-0.5) * ((b0 + As - a0) * b.i0);
            dr1 = dr1 + ((b1 + As - a1) * mkc(b.i1re, b.i1im)) * T(-0.5);
        } else {
            dr0 += T(-0.5) * ((a0 + Bs - b0) * a.i0 + (b0 + As - a0) * b.i0);
            dr1 = dr1 + ((a1 + Bs - b1) * mkc(a.i1re, a.i1im) + (b1 + As - a1) * mkc(b.i1re, b.i1im)) * T(-0.5);
        }
    } else {
        const T G1 = dB_dV1.re * T(2) * U1.re, G2 = dB_dV2 * T(2) * U2;
        const T a1 = G1 * T1_1.re, b1 = G1 * T2_1.re, a2 = G2 * T1_2, b2 = G2 * T2_2;
        const T As = a0 + a1 + a2, Bs = b0 + b1 + b2;
        dsig += T(-0.5) * (A_.x * As * a.it2 + B_.x * Bs * b.it2);
        if (ZINF) {
            dr0 += T(-0.5) * ((b0 + As - a0) * b.i0);
            dr1.re += T(-0.5) * ((b1 + As - a1) * b.i1re);
            dr2 += T(-0.5) * ((b2 + As - a2) * b.i2);
        } else {
            dr0 += T(-0.5) * ((a0 + Bs - b0) * a.i0 + (b0 + As - a0) * b.i0);
            dr1.re += T(-0.5) * ((a1 + Bs - b1) * a.i1re + (b1 + As - a1) * b.i1re);
            dr2 += T(-0.5) * ((a2 + Bs - b2) * a.i2 + (b2 + As - a2) * b.i2);
        }
    }
    const T scale = k.pre2 * dz;
    o.t = scale * (c3 * rj + rc + k.sigma * rf);
    o.dsig = scale * dsig;
    o.dr0 = scale * dr0;
    o.dr1re = scale * dr1.re;
    o.dr1im = scale * dr1.im;
    o.dr2 = scale * dr2;
}

// Parameter derivatives of the time coordinate between two redshifts, t/(1/H0) =
// int_{z1}^{z2} dz / ((1 + z) E(z)) (eq. 2.4), by the Leibniz rule in s = (1 + z)^(-1/2)
// (a = s^2 = 1/(1 + z)): the integral becomes int_{s2}^{s1} 2 s^3 ds / sqrt(R(s^2)) with
// R(a) = a^4 E^2(1/a) = Or + Om a + Ok a^2 + OL a^4 = beta (a - sigma) prod_j (1 - rho_j a),
// and z2 = inf is s2 = 0.  With Ok eliminated, dR/d(Om, OL, Or) = (a - a^2, a^4 - a^2,
// 1 - a^2), so d/dtheta = int -s^3 dR/dtheta R^(-3/2) ds.  Gauss-Legendre panels are laid
// from the upper end of the s-range down, each no wider than half the distance from its
// upper end to the nearest zero of R(s^2) in the complex s-plane (s = +-i sqrt(-sigma),
// s = +-rho_j^(-1/2)).  In units of the panel's half-width h every zero then lies at
// least 4h from the panel's upper end, so at least 3h from its centre when it is nearest,
// on the axis beyond the lower end: the Bernstein ellipse through it has parameter at
// least 3 + sqrt(8) = 5.83, and the Gauss-Legendre error is of order 5.83^(-2n): below
// 1e-30 with 20 nodes and 1e-12 with 8.  Towards z2 = inf the panels
// shrink geometrically onto the radiation zeros s = +-i sqrt(-sigma), which resolves the
// change of the integrand from radiation to matter domination even for Or0 ~ 1e-20
// (about 35 panels; at most 96).
// The zero s = +-sqrt(p) of R(s^2) for a = p = 1/rho (principal root; the real s-range
// is s >= 0, so the root with non-negative real part is the nearer one).
template <typename Q> struct SZero {
    Q re, im;
};
template <typename Q> __device__ __forceinline__ SZero<Q> sqrt_zero(Q pre, Q pim) {
    const Q m = Fp<Q>::sqrt(pre * pre + pim * pim);
    return SZero<Q>{Fp<Q>::sqrt(Q(0.5) * (m + pre)), Fp<Q>::sqrt(Q(0.5) * Fp<Q>::abs(m - pre))};
}
template <typename Q> __device__ __forceinline__ Q dist2_to(Q s, SZero<Q> z) {
    const Q dr = s - z.re;
    return dr * dr + z.im * z.im;
}

template <typename Q, bool PAIR>
__device__ void gl_time_between(const LaneConst<Q> &k, Q z1, Q z2, bool zinf, Q g[3]) {
    // the s-range [s_hi - width, s_hi]: s_hi at the lower redshift; the width as a divided
    // difference (close limits would cancel in s1 - s2), and every node and 1 - a = 1 - s^2
    // measured from s_hi (1 - s_hi^2 = z_lo/(1 + z_lo) exactly)
    const bool up = zinf || z2 >= z1; // z2 above z1: t > 0
    const Q zlo = up ? z1 : z2;
    const Q xlo = Q(1) + zlo;
    const Q shi = Fp<Q>::rsqrt(xlo);
    Q width;
    if (zinf) {
        width = shi;
    } else {
        const Q x1 = Q(1) + z1, x2 = Q(1) + z2;
        const Q r1 = Fp<Q>::sqrt(x1), r2 = Fp<Q>::sqrt(x2);
        width = Fp<Q>::abs(z2 - z1) * Fp<Q>::rcp(r1 * r2 * (r1 + r2));
    }
    const Q omhi = zlo * Fp<Q>::rcp(xlo);
    const Q sgn = up ? Q(1) : Q(-1);
    // zeros of R(s^2), once per lane: a = sigma (s = +-i sqrt(-sigma)) and a = 1/rho_j
    const Q sig2 = k.sigma == Q(0) ? Q(-1) : (-k.sigma > Q(1e-30) ? -k.sigma : Q(1e-30));
    const SZero<Q> e0 = sqrt_zero<Q>(Fp<Q>::rcp(k.r0), Q(0));
    const Q q1m2 = k.r1re * k.r1re + k.r1im * k.r1im;
    const SZero<Q> e1 = PAIR ? sqrt_zero<Q>(k.r1re * Fp<Q>::rcp(q1m2), -k.r1im * Fp<Q>::rcp(q1m2))
                             : sqrt_zero<Q>(Fp<Q>::rcp(k.r1re), Q(0));
    const SZero<Q> e2 = PAIR ? e1 : sqrt_zero<Q>(Fp<Q>::rcp(k.r2), Q(0));
    Q g0 = Q(0), g1 = Q(0), g2 = Q(0);
    Q done = Q(0); // offset from s_hi covered so far
    for (int p = 0; p < 96 && done < width; ++p) {
        const Q top = shi - done;
        Q d2 = dist2_to<Q>(top, e0);
        Q t = dist2_to<Q>(top, e1);
        d2 = t < d2 ? t : d2;
        t = dist2_to<Q>(top, e2);
        d2 = t < d2 ? t : d2;
        if (sig2 > Q(0)) {
            t = top * top + sig2;
            d2 = t < d2 ? t : d2;
        }
        Q w = Q(0.5) * Fp<Q>::sqrt(d2);
        if (w > width - done || p == 95) w = width - done;
        const Q half = Q(0.5) * w, cen = done + half;
        for (int i = 0; i < GlRule<Q>::n; ++i) {
            const Q off = cen + half * GlRule<Q>::x(i); // offset from s_hi
            const Q s = shi - off;
            const Q a = s * s;
            const Q om = omhi + off * (Q(2) * shi - off); // 1 - a
            const Q qa = PAIR ? (Q(1) - k.r0 * a) * ((Q(1) - Q(2) * k.r1re * a) + q1m2 * a * a)
                              : (Q(1) - k.r0 * a) * (Q(1) - k.r1re * a) * (Q(1) - k.r2 * a);
            const Q R = k.beta * (a - k.sigma) * qa;
            const Q ir = Fp<Q>::rsqrt(R);
            const Q c = -half * GlRule<Q>::w(i) * s * s * s * ir * ir * ir;
            g0 += c * a * om;                     // a - a^2
            g1 += c * (-a * a * om * (Q(1) + a)); // a^4 - a^2
            g2 += c * om * (Q(1) + a);            // 1 - a^2
        }
        done += w;
    }
    g[0] = sgn * g0; g[1] = sgn * g1; g[2] = sgn * g2;
}

// Derivatives of one lane between z1 and z2 for KIND = COSMO_DC, COSMO_DM, COSMO_DA or
// COSMO_T (the last by gl_time_between; the others as follows),
// in the layout of LaneGrad (root mode: p[0..4]; near-multiple roots: the Leibniz
// quadrature partials from 0 to each limit, differenced, in q[0..2]); dz1 and dz2 by the
// fundamental theorem of calculus.
template <typename T> struct LaneGrad2 {
    LaneGrad<T> g;
    T dz1;
};

// Every lane of cosmology r takes the root chain (no quadrature route): not near-multiple
// roots, and for the time coordinate a radiation root large enough for an infinite limit.
template <typename T, int KIND> __device__ __forceinline__ bool between_chain_only(const CosmoRec &r) {
    const bool fp32 = sizeof(T) == 4;
    if (direct_mode(KIND, r, fp32)) return false;
    return KIND != COSMO_T || -lane_of<T>(r).sigma >= T(fp32 ? kAgeSigma32 : kAgeSigma64);
}

// CO: the cosmology is known to satisfy between_chain_only (quadrature routes compiled out).
template <typename T, int KIND, bool PAIR, bool CO = false>
__device__ __forceinline__ void lane_grad_between(const CosmoRec &r, T z1, T z2, LaneGrad2<T> &o) {
    const LaneConst<T> &k = lane_of<T>(r);
    const bool fp32 = sizeof(T) == 4;
    const bool zinf = z2 == Fp<T>::inf();
    const bool t_direct = KIND == COSMO_T && direct_mode(KIND, r, fp32);
    const bool t_sig = -k.sigma >= T(fp32 ? kAgeSigma32 : kAgeSigma64);
    if (KIND == COSMO_T && (CO || !(t_direct || (zinf && !t_sig)))) {
        // time coordinate: eq. 3.8 with both limits through the Carlson derivatives (the
        // age t(z1, inf) on every lane of the wave: the upper side's constants fold)
        LaneGrad<T> &g = o.g;
        TGrad2<T, PAIR> tg;
        if (__ballot(!zinf) == 0) t_grad_between<T, PAIR, true>(r, z1, z2, tg);
        else t_grad_between<T, PAIR>(r, z1, z2, tg);
        g.quad = false;
        g.p[0] = tg.t; g.p[1] = tg.dsig; g.p[2] = tg.dr0; g.p[3] = tg.dr1re; g.p[4] = PAIR ? tg.dr1im : tg.dr2;
        g.val = k.th * tg.t;
        g.s = k.th;
        g.dok = T(0);
        g.dh = -g.val * k.hinv;
        o.dz1 = -k.th * Fp<T>::rcp(T(1) + z1) * tg.iE1;
        g.dz = zinf ? T(0) : k.th * Fp<T>::rcp(T(1) + z2) * tg.iE2;
        return;
    }
    if (KIND == COSMO_T) {
        // near-multiple roots, and the age without radiation: the value by eq. 3.8 with
        // both limits, the parameter derivatives by the Leibniz quadrature in
        // s = (1 + z)^(-1/2) (finite to z2 = inf)
        LaneGrad<T> &g = o.g;
        T q[3];
        gl_time_between<T, PAIR>(k, z1, z2, zinf, q);
        g.quad = true;
#pragma unroll
        for (int i = 0; i < 5; ++i) g.p[i] = T(0);
        g.q[0] = q[0]; g.q[1] = q[1]; g.q[2] = q[2];
        g.val = k.th * t_between<T, PAIR>(r, z1, z2);
        g.s = k.th;
        g.dok = T(0);
        g.dh = -g.val * k.hinv;
        o.dz1 = -k.th * Fp<T>::rcp(T(1) + z1) * iEz<T>(k, z1);
        g.dz = zinf ? T(0) : k.th * Fp<T>::rcp(T(1) + z2) * iEz<T>(k, z2);
        return;
    }
    ChiGrad2<T, PAIR> cg;
    chi_grad_between<T, PAIR>(k, z1, z2, cg);
    LaneGrad<T> &g = o.g;
    g.quad = !CO && direct_mode(KIND, r, fp32);
    g.p[0] = cg.chi; g.p[1] = cg.dsig; g.p[2] = cg.dr0; g.p[3] = cg.dr1re; g.p[4] = PAIR ? cg.dr1im : cg.dr2;
    if (g.quad) {
        // near-multiple roots: the root chain is ill conditioned; Leibniz quadrature from
        // 0 to each limit (not defined to an infinite limit)
        if (zinf) {
            g.q[0] = g.q[1] = g.q[2] = Fp<double>::nan();
        } else if (fp32) {
            T v, g1[3], g2[3];
            gl_integral<T, PAIR>(k, z2, 0, true, v, g2);
            gl_integral<T, PAIR>(k, z1, 0, true, v, g1);
            for (int i = 0; i < 3; ++i) g.q[i] = (double)g2[i] - (double)g1[i];
        } else {
            const GlChi c2 = gl_chi_grad<PAIR>(r, (double)z2), c1 = gl_chi_grad<PAIR>(r, (double)z1);
            g.q[0] = c2.g0 - c1.g0; g.q[1] = c2.g1 - c1.g1; g.q[2] = c2.g2 - c1.g2;
        }
    }
    const T H0inv = k.hinv;
    const T chi = cg.chi;
    if (KIND == COSMO_DC) {
        g.val = k.dh * chi; g.s = k.dh; g.dok = T(0);
    } else {
        T S, C, dS;
        sinn(chi, k.ok, k.sk, S, C, dS);
        const T f = KIND == COSMO_DA ? (zinf ? T(0) : Fp<T>::rcp(T(1) + z2)) : T(1);
        g.val = k.dh * S * f; g.s = k.dh * C * f; g.dok = k.dh * dS * f;
    }
    g.dh = -g.val * H0inv;
    o.dz1 = -g.s * cg.iE1;
    g.dz = g.s * cg.iE2;
    if (KIND == COSMO_DA && !zinf) g.dz -= g.val * Fp<T>::rcp(T(1) + z2);
}

} // namespace cosmo
