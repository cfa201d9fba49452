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

#include "lane.hpp"

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
    s.t = Fp<T>::sqrt(s.t2);
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

template <typename T, bool PAIR>
__device__ __forceinline__ void sides(const LaneConst<T> &k, T z1, T z2, Side<T, PAIR> &a, Side<T, PAIR> &b, T &dz) {
    side_at<T, PAIR>(k, z1, b);
    if (z2 == Fp<T>::inf()) {
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
    return k.pre * T(2) * dz * rf_s<T, PAIR>(u.V0, u.va, u.vb);
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
__device__ __forceinline__ void t_args_between(const LaneConst<Q> &k, Q z1, Q z2, TArgs2<Q, PAIR> &o) {
    Side<Q, PAIR> a, b;
    sides<Q, PAIR>(k, z1, z2, a, b, o.dz);
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

// t(z1, z2) / (1/H0), eq. 3.8 (z2 = inf: the age t(z1, inf)).  The FP32 path forms
// the arguments in FP64 and rounds once (as t_hat does).
template <typename T, bool PAIR> __device__ __forceinline__ T t_between(const CosmoRec &r, T z1, T z2) {
    const LaneConst<T> &k = lane_of<T>(r);
    TArgs2<double, PAIR> ad;
    t_args_between<double, PAIR>(r.d, (double)z1, z2 == Fp<T>::inf() ? Fp<double>::inf() : (double)z2, ad);
    const T V0 = T(ad.u.V0), va = T(ad.u.va), vb = T(ad.u.vb), W = T(ad.W);
    const T dz = T(ad.dz), d2 = dz * dz;
    T rf, rj;
    rfj_s<T, PAIR>(V0, va, vb, W, rf, rj);
    const T rc = ad.rc_zero ? T(0) : rc_r(T(ad.S), T(ad.Qv));
    return k.pre * T(2) * dz * (d2 * T(1.0 / 3.0) * k.pre3 * rj + rc + k.sigma * rf);
}

// Observable KIND (COSMO_DC, COSMO_DM, COSMO_DA or COSMO_T) between z1 and z2.
template <typename T, int KIND, bool PAIR>
__device__ __forceinline__ T eval_between(const CosmoRec &r, T z1, T z2) {
    const LaneConst<T> &k = lane_of<T>(r);
    if (KIND == COSMO_T) return k.th * t_between<T, PAIR>(r, z1, z2);
    const T chi = chi_between<T, PAIR>(k, z1, z2);
    if (KIND == COSMO_DC) return k.dh * chi;
    T S, C, dS;
    sinn(chi, k.ok, k.sk, S, C, dS);
    if (KIND == COSMO_DM) return k.dh * S;
    return z2 == Fp<T>::inf() ? T(0) : k.dh * S * Fp<T>::rcp(T(1) + z2); // COSMO_DA
}

} // namespace cosmo
