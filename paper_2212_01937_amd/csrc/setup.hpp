// setup.hpp -- per-cosmology preparation, FP64 (one lane per cosmology).
//
// Factorisation of E^2 (sec. 3, eq. 3.2), taken in x = 1 + z where the
// polynomial is P(x) = Or x^4 + Om x^3 + Ok x^2 + OL (no linear term).
//
// Normalised radiation factor.  When Or > 0 the quartic has a real root rho_l of
// large modulus (~ -Om/Or).  Instead of that root we carry sigma = 1/rho_l, the
// root of the reversed polynomial R(s) = OL s^4 + Ok s^2 + Om s + Or closest to 0
// from below, and beta = -Or rho_l:
//       P(x) = beta (1 - sigma x) Q(x),     Q(x) = x^3 + q2 x^2 + q1 x + q0,
//       beta = Om + sigma (Ok + sigma^2 OL),  q0 = OL/beta, q1 = sigma q0,
//       q2 = (Ok + sigma^2 OL)/beta.
// The factor z + a_l of eq. 3.1 becomes (1 - sigma x) with a general
// coefficient (the b_i of fn. 11); for Or = 0 it is identically one (sigma = 0,
// beta = Om), which is exactly the radiationless case of app. B.1 (the label l
// "changed to 0").  So one set of formulas covers eqs. 3.7-3.9 and B.1-B.3 and
// stays well conditioned as Or -> 0; the radiation root's sqrt(z - r_l) factors
// become sqrt(|rho_l|) sqrt(1 - sigma x), and by homogeneity of the Carlson
// integrals the powers of |rho_l| collect into beta^(-1/2) = (Or |rho_l|)^(-1/2).
//
// Roots of the cubic factor: one real root by safeguarded Newton, deflation to
// a quadratic (forward and backward deflation, keeping the one with the smaller
// residual), a stable quadratic formula, then Newton polishing on Q.  Numerical
// root finding, as the paper recommends over the algebraic formulae (sec. 3.2.1).
//
// Root gradients (app. A): every root rho_n of P satisfies P(rho_n; theta) = 0,
// so d rho_n / d theta = -(dP/d theta)(rho_n) / P'(rho_n), with
// P'(rho_n) = beta (1 - sigma rho_n) prod_{m != n} (rho_n - rho_m).  This is the
// solution of the Vieta system of eq. A.4 (C^T dr/dc = -1 with c the monic
// coefficients; the printed "+1" sign reading is the one of eqs. A.2/A.3), written
// per root.  theta = (Om0, OL0, Or0) with Ok0 = 1 - Om0 - OL0 - Or0 eliminated:
// dP/dOm = x^3 - x^2, dP/dOL = 1 - x^2, dP/dOr = x^4 - x^2.
#pragma once

#include "cmath.hpp"
#include "../../include/cosmo.h"

namespace cosmo {

constexpr double kC = 299792.458;               // km/s
constexpr double kMpcKm = 3.0856775814913673e19; // km
constexpr double kGyrS = 3.15576e16;            // s

// Per-lane constants of one cosmology in the arithmetic type T.
// Root slots: n = 0 is a real root of Q; slots 1, 2 are a conjugate pair
// (pair = 1: rho1 = r1re + i r1im, rho2 = conj) or two further real roots
// (pair = 0: rho1 = r1re, rho2 = r2).  w_n = 1 - rho_n = (Y_n)^2.
template <typename T> struct LaneConst {
    T sigma, yt, yt2;       // sigma, Ytilde = sqrt(1 - sigma), Ytilde^2
    T r0, r1re, r1im, r2;   // roots of Q
    T w0, w1re, w1im, w2;   // 1 - rho_n
    T y0, y1re, y1im, y2;   // Y_n = sqrt(1 - rho_n)
    T y1abs2;               // |Y_1|^2 = |1 - rho_1| (pair)
    T pre;                  // beta^(-1/2)
    T ok, sk;               // Ok0 and sqrt(|Ok0|)
    T dh, th;               // c/H0 [Mpc], 1/H0 [Gyr]
    T Or, Om, OL;           // for E(z) in the z-gradient
    T q0, q1, q2;           // cubic factor coefficients
    T c5, pre3, rprod;      // T: (1-s r1)(1-s r2) r0, prod(1 - s r_n), r0 r1 r2
    T c5b, c5c;             // T: the same coefficient for root slot 1 (real part for a pair) and slot 2
    T xc3, xc2, xs3;        // X: 3 r0^2 - d01 d02, 2 r0^2 - d01 d02, S3 = sum r_n
    T d0102;                // X: (r1 - r0)(r2 - r0)
    T om1s12, op1s3, om1s0; // X: (1-s r1)(1-s r2), 1 + s S3, 1 - s r0
    T d02re, d02im;         // X: r2 - r0
    T xe1, xa, xym;         // X, regular form: -2(r1 + r2) + s (r1 r2 + S3 r0), -(r1 + r2) + s r1 r2,
                            //   -1/(Yt + 1)
    T dpath;                // distance of the nearest singularity ln(rho_n) to the path u >= 0
    T iyt2, iw0, iw1re, iw1im, iw2; // 1/Yt^2, 1/w_0, 1/w_1 (complex for a pair), 1/w_2
    T hinv;                 // 1/H0 [s Mpc/km]
    T beta;                 // E^2 = beta (1 - sigma x) Q(x)
    // per-cosmology products the lanes would otherwise form on every evaluation
    T pre2;                 // 2 beta^(-1/2)
    T yty0;                 // Yt Y0
    T y1y2, y0y2, y0y1;     // three real roots: Y1 Y2, Y0 Y2, Y0 Y1
    T yty1, yty2;           //   Yt Y1, Yt Y2
    T w1im2, hw1im, sw1im;  // pair: Im(w_1)^2, |Im(w_1)|/2, sign of Im(w_1) (+-1)
    T k5hinv;               // (5 / ln 10) / H0: minus dmu/dH0
    T tinf, itinf2;         // sqrt(-sigma) and 1/(-sigma): an infinite limit's scaled sqrt(1 - sigma x)
    // T between two limits: the explicit sigma- and root-dependence of eq. 3.8's
    // coefficients (o_n = 1 - sigma r_n; slot 1 with its partner slot 2, and for three
    // real roots slot 2 with partner 1)
    T tdp3, tdc5;           // dP3/dsigma = -(r0 o1 o2 + o0 (r1 o2 + r2 o1)), dC5/dsigma = -r0 (r1 o2 + r2 o1)
    T tso12, tr12;          // -sigma o1 o2, r1 r2 (real parts)
    T tq1re, tq1im;         // -sigma o0 o2
    T tq2re, tq2im;         // -sigma r0 o2
    T tq3re, tq3im;         // r0 r2
    T tq4, tq5, tq6;        // three real roots: -sigma o0 o1, -sigma r0 o1, r0 r1
};

struct CosmoRec {
    int32_t info;  // COSMO_INFO_* bits
    int32_t valid; // 1: evaluate; 0: NaN outputs
    int32_t pair;  // slot structure of the cubic roots
    int32_t fallback_grad; // 1: parameter gradients by quadrature (near-multiple roots)
    double H0, beta, minsep;
    double dbeta[3], dsigma[3];       // d/d(Om, OL, Or)
    double drho_re[3][3], drho_im[3][3]; // [root slot][param]
    double rl;                         // radiation root in x (1/sigma), NaN if cubic
    float jc32[5][3];                  // root-Jacobian contraction coefficients in FP32 (root_contract's)
    LaneConst<double> d;
    LaneConst<float> f;
};

// ---------------------------------------------------------------- helpers (FP64)
__device__ __forceinline__ double cubic_at(double q2, double q1, double q0, double x) {
    return ((x + q2) * x + q1) * x + q0;
}
__device__ __forceinline__ cx<double> cubic_at(double q2, double q1, double q0, cx<double> x) {
    return ((x + q2) * x + q1) * x + q0;
}
__device__ __forceinline__ cx<double> cubic_d(double q2, double q1, cx<double> x) {
    return (x * 3.0 + 2.0 * q2) * x + q1;
}

// Largest negative root of R(s) = OL s^4 + Ok s^2 + Om s + Or (Or > 0), or NaN.
__device__ double sigma_root(double Om, double OL, double Or, double Ok, int &iters) {
    auto R = [&](double s) { return ((OL * s * s + Ok) * s + Om) * s + Or; };
    auto dR = [&](double s) { return (4.0 * OL * s * s + 2.0 * Ok) * s + Om; };
    double hi = 0.0;
    double lo = Om > 0.0 ? -2.0 * Or / Om : -1.0;
    if (!(lo < 0.0)) lo = -1.0;
    int k = 0;
    while (R(lo) >= 0.0 && k < 2100) { hi = lo; lo *= 2.0; ++k; }
    if (!(R(lo) < 0.0)) return __builtin_nan("");
    double s = (Om > 0.0 && -Or / Om > lo && -Or / Om < hi) ? -Or / Om : 0.5 * (lo + hi);
    iters = 0;
    for (int it = 0; it < 200; ++it) {
        ++iters;
        double r = R(s);
        if (r == 0.0) break;
        if (r > 0.0) hi = s; else lo = s;
        const double dn = r / dR(s);
        // converged: the Newton correction is below the resolution of s (tested before
        // the bracket safeguard, which a step that rounds to s itself would trip)
        if (__builtin_fabs(dn) <= 4e-16 * __builtin_fabs(s)) { s -= dn; break; }
        double sn = s - dn;
        if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
        s = sn;
        if (hi - lo <= 4e-16 * __builtin_fabs(s)) break;
    }
    return s;
}

// A real root of the monic cubic by safeguarded Newton on the Cauchy bracket
// [-M, M], started from one end (from_left: converges to the leftmost real root,
// otherwise to the rightmost one).
__device__ double cubic_real_root(double q2, double q1, double q0, bool from_left, int &iters) {
    double M = 1.0 + tmax(tmax(__builtin_fabs(q0), __builtin_fabs(q1)), __builtin_fabs(q2));
    double lo = -M, hi = M;
    double x = from_left ? -M : M;
    iters = 0;
    for (int it = 0; it < 300; ++it) {
        ++iters;
        double f = cubic_at(q2, q1, q0, x);
        if (f == 0.0) return x;
        if (f < 0.0) lo = x; else hi = x;
        const double dn = f / ((3.0 * x + 2.0 * q2) * x + q1);
        // converged (checked before the safeguard: a correction that rounds to x itself
        // fails the open-bracket test and would send the iterate to the bracket midpoint,
        // possibly towards another root)
        if (__builtin_fabs(dn) <= 2e-16 * tmax(1.0, __builtin_fabs(x))) return x - dn;
        double xn = x - dn;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        x = xn;
        if (hi - lo <= 4e-16 * tmax(1.0, __builtin_fabs(x))) break;
    }
    return x;
}

// Roots of x^2 + b1 x + b0 (real coefficients).  Returns true for a complex pair.
__device__ bool quad_roots(double b1, double b0, cx<double> &u, cx<double> &v) {
    double disc = b1 * b1 - 4.0 * b0;
    if (disc < 0.0) {
        double im = 0.5 * __builtin_sqrt(-disc);
        u = mkc(-0.5 * b1, im);
        v = mkc(-0.5 * b1, -im);
        return true;
    }
    double qq = -0.5 * (b1 + (b1 >= 0.0 ? 1.0 : -1.0) * __builtin_sqrt(disc));
    double r1 = qq, r2 = (qq != 0.0) ? b0 / qq : 0.0;
    u = mkc(r1, 0.0);
    v = mkc(r2, 0.0);
    return false;
}

__device__ double cubic_resid(double q2, double q1, double q0, cx<double> x) {
    // |Q(x)| relative to the size of its terms
    cx<double> v = cubic_at(q2, q1, q0, x);
    double ax = cabs(x);
    double sc = ((ax + __builtin_fabs(q2)) * ax + __builtin_fabs(q1)) * ax + __builtin_fabs(q0);
    return cabs(v) / (sc > 0.0 ? sc : 1.0);
}

__device__ cx<double> newton_polish(double q2, double q1, double q0, cx<double> x) {
    double rx = cubic_resid(q2, q1, q0, x); // carried over: the accepted step's residual
    for (int it = 0; it < 4; ++it) {
        cx<double> d = cubic_d(q2, q1, x);
        if (norm2(d) == 0.0) break;
        cx<double> xn = x - cdiv(cubic_at(q2, q1, q0, x), d);
        const double rn = cubic_resid(q2, q1, q0, xn);
        if (rn < rx) { x = xn; rx = rn; } else break;
    }
    return x;
}

template <typename T> __device__ void fill_lane(LaneConst<T> &L, const LaneConst<double> &D) {
    L.sigma = T(D.sigma); L.yt = T(D.yt); L.yt2 = T(D.yt2);
    L.r0 = T(D.r0); L.r1re = T(D.r1re); L.r1im = T(D.r1im); L.r2 = T(D.r2);
    L.w0 = T(D.w0); L.w1re = T(D.w1re); L.w1im = T(D.w1im); L.w2 = T(D.w2);
    L.y0 = T(D.y0); L.y1re = T(D.y1re); L.y1im = T(D.y1im); L.y2 = T(D.y2);
    L.y1abs2 = T(D.y1abs2); L.pre = T(D.pre); L.ok = T(D.ok); L.sk = T(D.sk);
    L.dh = T(D.dh); L.th = T(D.th); L.Or = T(D.Or); L.Om = T(D.Om); L.OL = T(D.OL);
    L.q0 = T(D.q0); L.q1 = T(D.q1); L.q2 = T(D.q2);
    L.c5 = T(D.c5); L.pre3 = T(D.pre3); L.rprod = T(D.rprod); L.c5b = T(D.c5b); L.c5c = T(D.c5c);
    L.xc3 = T(D.xc3); L.xc2 = T(D.xc2); L.xs3 = T(D.xs3); L.d0102 = T(D.d0102);
    L.om1s12 = T(D.om1s12); L.op1s3 = T(D.op1s3); L.om1s0 = T(D.om1s0);
    L.d02re = T(D.d02re); L.d02im = T(D.d02im);
    L.xe1 = T(D.xe1); L.xa = T(D.xa); L.xym = T(D.xym);
    L.dpath = T(D.dpath);
    L.iyt2 = T(D.iyt2); L.iw0 = T(D.iw0); L.iw1re = T(D.iw1re); L.iw1im = T(D.iw1im); L.iw2 = T(D.iw2);
    L.hinv = T(D.hinv);
    L.beta = T(D.beta);
    L.pre2 = T(D.pre2); L.yty0 = T(D.yty0);
    L.y1y2 = T(D.y1y2); L.y0y2 = T(D.y0y2); L.y0y1 = T(D.y0y1); L.yty1 = T(D.yty1); L.yty2 = T(D.yty2);
    L.w1im2 = T(D.w1im2); L.hw1im = T(D.hw1im); L.sw1im = T(D.sw1im);
    L.k5hinv = T(D.k5hinv);
    L.tinf = T(D.tinf); L.itinf2 = T(D.itinf2);
    L.tdp3 = T(D.tdp3); L.tdc5 = T(D.tdc5); L.tso12 = T(D.tso12); L.tr12 = T(D.tr12);
    L.tq1re = T(D.tq1re); L.tq1im = T(D.tq1im); L.tq2re = T(D.tq2re); L.tq2im = T(D.tq2im);
    L.tq3re = T(D.tq3re); L.tq3im = T(D.tq3im); L.tq4 = T(D.tq4); L.tq5 = T(D.tq5); L.tq6 = T(D.tq6);
}

// dP/dtheta at x for theta = Om, OL, Or (Ok eliminated)
__device__ __forceinline__ cx<double> dP_dtheta(int a, cx<double> x) {
    cx<double> x2 = x * x;
    if (a == 0) return x2 * x - x2;
    if (a == 1) return mkc(1.0, 0.0) - x2;
    return x2 * x2 - x2;
}

__device__ void setup_cosmo(const double *prm, CosmoRec &rec) {
    const double H0 = prm[0], Om = prm[1], OL = prm[2], Or = prm[3];
    const double Ok = 1.0 - Om - OL - Or;
    int info = 0;
    rec.valid = 0;
    rec.pair = 0;
    rec.fallback_grad = 0;
    rec.H0 = H0;
    // fields the early returns below leave unset (records of cosmologies outside the
    // method are never evaluated, but every field is defined)
    rec.beta = 0.0;
    rec.minsep = 0.0;
    for (int a = 0; a < 3; ++a) {
        rec.dbeta[a] = rec.dsigma[a] = 0.0;
        for (int n = 0; n < 3; ++n) rec.drho_re[n][a] = rec.drho_im[n][a] = 0.0;
        for (int q = 0; q < 5; ++q) rec.jc32[q][a] = 0.0f;
    }
    LaneConst<double> &D = rec.d;
    D = LaneConst<double>{};
    bool finite = __builtin_isfinite(H0) && __builtin_isfinite(Om) && __builtin_isfinite(OL) &&
                  __builtin_isfinite(Or);
    if (!finite || !(H0 > 0.0) || Or < 0.0 || (Or == 0.0 && !(Om > 0.0))) {
        rec.info = COSMO_INFO_DOMAIN;
        rec.rl = __builtin_nan("");
        fill_lane(rec.f, D);
        return;
    }
    double sigma = 0.0, beta = Om;
    int it_s = 0;
    if (Or > 0.0) {
        info |= COSMO_INFO_QUARTIC;
        sigma = sigma_root(Om, OL, Or, Ok, it_s);
        if (!(sigma < 0.0)) { // no negative real root: outside the method
            rec.info = info | COSMO_INFO_DOMAIN;
            rec.rl = __builtin_nan("");
            fill_lane(rec.f, D);
            return;
        }
        beta = Om + sigma * (Ok + sigma * sigma * OL);
        if (it_s >= 200) info |= COSMO_INFO_ROOT_NOCONV;
    } else {
        info |= COSMO_INFO_CUBIC;
    }
    if (!(beta > 0.0)) {
        rec.info = info | COSMO_INFO_DOMAIN;
        rec.rl = __builtin_nan("");
        fill_lane(rec.f, D);
        return;
    }
    const double q0 = OL / beta, q1 = sigma * q0, q2 = (Ok + sigma * sigma * OL) / beta;

    // --- roots of the cubic factor.  Deflate by the real root that is best
    // isolated (largest |Q'(r)|): deflating one member of a near-double pair would
    // pass its ~eps/separation error on to the quadratic.  The leftmost real root
    // comes from Newton started left of every root; when the quadratic left by it
    // has real roots, the best isolated of the three (by the product of distances,
    // |Q'|) is polished on Q and taken instead.
    int it_r = 0;
    double r = cubic_real_root(q2, q1, q0, true, it_r);
    if (it_r >= 300) info |= COSMO_INFO_ROOT_NOCONV;
    {
        cx<double> a, b;
        const double l1 = q2 + r, l0 = q1 + r * l1;
        if (!quad_roots(l1, l0, a, b)) {
            const double gr = __builtin_fabs((r - a.re) * (r - b.re));
            const double ga = __builtin_fabs((a.re - r) * (a.re - b.re));
            const double gb = __builtin_fabs((b.re - r) * (b.re - a.re));
            if (tmax(ga, gb) > gr) r = newton_polish(q2, q1, q0, mkc(ga >= gb ? a.re : b.re, 0.0)).re;
        }
    }
    // forward deflation: b1 = q2 + r, b0 = q1 + r b1;  backward: b0 = -q0/r, b1 = (b0 - q1)/r
    cx<double> u1, v1, u2, v2;
    double fb1 = q2 + r, fb0 = q1 + r * fb1;
    bool p1 = quad_roots(fb1, fb0, u1, v1);
    bool p2 = p1;
    double e1 = tmax(cubic_resid(q2, q1, q0, u1), cubic_resid(q2, q1, q0, v1));
    double e2 = 1e300;
    if (r != 0.0) {
        double bb0 = -q0 / r, bb1 = (bb0 - q1) / r;
        p2 = quad_roots(bb1, bb0, u2, v2);
        e2 = tmax(cubic_resid(q2, q1, q0, u2), cubic_resid(q2, q1, q0, v2));
    }
    bool pair = p1;
    cx<double> ra = u1, rb = v1;
    if (e2 < e1) { pair = p2; ra = u2; rb = v2; }
    // Polish only well separated roots: Newton on a near-double pair can merge the
    // two, whereas the deflated quadratic's roots are already backward stable.
    bool separated = cabs(ra - rb) > 1e-3 * tmax(cabs(ra), cabs(rb));
    if (pair) {
        if (separated) {
            cx<double> pa = newton_polish(q2, q1, q0, ra);
            if (pa.im != 0.0) ra = pa;
        }
        if (ra.im < 0.0) ra = conj(ra);
        rb = conj(ra); // exact conjugate symmetry: the factorisation is of a real polynomial
    } else {
        if (separated) {
            ra = newton_polish(q2, q1, q0, ra);
            rb = newton_polish(q2, q1, q0, rb);
        }
        ra.im = 0.0;
        rb.im = 0.0;
    }
    double rr = newton_polish(q2, q1, q0, mkc(r, 0.0)).re;
    // slot order: 0 = real root (for three real roots: the largest modulus first)
    double s0, s1re, s1im, s2;
    if (pair) {
        s0 = rr; s1re = ra.re; s1im = ra.im; s2 = rb.re;
    } else {
        double t[3] = {rr, ra.re, rb.re};
        for (int i = 0; i < 3; ++i)
            for (int j = i + 1; j < 3; ++j)
                if (__builtin_fabs(t[j]) > __builtin_fabs(t[i])) { double w = t[i]; t[i] = t[j]; t[j] = w; }
        s0 = t[0]; s1re = t[1]; s1im = 0.0; s2 = t[2];
        info |= COSMO_INFO_THREE_REAL;
    }
    rec.pair = pair ? 1 : 0;
    cx<double> rho[3] = {mkc(s0, 0.0), mkc(s1re, s1im), pair ? mkc(s1re, -s1im) : mkc(s2, 0.0)};

    // --- classification (Fig. 1): a real root in x >= 1 lies on the integration path
    double maxreal = s0;
    if (!pair) maxreal = tmax(maxreal, tmax(s1re, s2));
    if (maxreal >= 1.0) info |= COSMO_INFO_RED;
    if (pair && s1re > 1.0) info |= COSMO_INFO_YELLOW;

    // --- separation of the roots (conditioning of the root Jacobian).  Two roots
    // rho_i, rho_j enter the distance through their symmetric functions; the root
    // chain cancels by about |x - rho| / |rho_i - rho_j| with x on the integration
    // path, so the separation is measured against the distance to x = 1.
    double minsep = 1e300;
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j) {
            double sc = tmax(cabs(mkc(1.0, 0.0) - rho[i]), cabs(mkc(1.0, 0.0) - rho[j]));
            double dd = cabs(rho[i] - rho[j]);
            double sep = sc > 0.0 ? dd / sc : 0.0;
            minsep = sep < minsep ? sep : minsep;
        }
    if (Or > 0.0)
        for (int i = 0; i < 3; ++i) {
            double sep = cabs(mkc(1.0, 0.0) - rho[i] * sigma); // |rho_l - rho_i| / |rho_l|
            minsep = sep < minsep ? sep : minsep;
        }
    rec.minsep = minsep;
    if (minsep < 1e-4) info |= COSMO_INFO_NEAR_MULTIROOT;
    if (minsep < 2e-2) info |= COSMO_INFO_NEAR_MULTIROOT_F32;

    // --- lane constants
    D.sigma = sigma;
    D.yt2 = 1.0 - sigma;
    D.yt = __builtin_sqrt(D.yt2);
    D.r0 = s0; D.r1re = s1re; D.r1im = pair ? s1im : 0.0; D.r2 = pair ? s1re : s2;
    D.w0 = 1.0 - s0; D.w1re = 1.0 - s1re; D.w1im = pair ? -s1im : 0.0; D.w2 = pair ? 1.0 - s1re : 1.0 - s2;
    D.y0 = __builtin_sqrt(D.w0);
    if (pair) {
        double ab;
        cx<double> y1 = csqrt(mkc(D.w1re, D.w1im), ab);
        D.y1re = y1.re; D.y1im = y1.im; D.y2 = 0.0; D.y1abs2 = ab;
    } else {
        D.y1re = __builtin_sqrt(D.w1re); D.y1im = 0.0; D.y2 = __builtin_sqrt(D.w2); D.y1abs2 = 0.0;
    }
    D.iyt2 = 1.0 / D.yt2;
    D.iw0 = 1.0 / D.w0;
    if (pair) {
        cx<double> iw1 = cdiv(mkc(1.0, 0.0), mkc(D.w1re, D.w1im));
        D.iw1re = iw1.re; D.iw1im = iw1.im; D.iw2 = 0.0;
    } else {
        D.iw1re = 1.0 / D.w1re; D.iw1im = 0.0; D.iw2 = 1.0 / D.w2;
    }
    D.hinv = 1.0 / H0;
    D.beta = beta;
    D.pre = 1.0 / __builtin_sqrt(beta);
    D.pre2 = 2.0 * D.pre;
    D.yty0 = D.yt * D.y0;
    D.y1y2 = D.y1re * D.y2; D.y0y2 = D.y0 * D.y2; D.y0y1 = D.y0 * D.y1re;
    D.yty1 = D.yt * D.y1re; D.yty2 = D.yt * D.y2;
    D.w1im2 = D.w1im * D.w1im; D.hw1im = 0.5 * __builtin_fabs(D.w1im); D.sw1im = D.w1im >= 0.0 ? 1.0 : -1.0;
    D.k5hinv = 2.1714724095162591 * D.hinv;
    D.tinf = __builtin_sqrt(-sigma);
    D.itinf2 = 1.0 / -sigma; // infinite without radiation (sigma = 0)
    D.ok = Ok;
    D.sk = __builtin_sqrt(__builtin_fabs(Ok));
    D.dh = kC / H0;
    D.th = kMpcKm / (H0 * kGyrS);
    D.Or = Or; D.Om = Om; D.OL = OL;
    D.q0 = q0; D.q1 = q1; D.q2 = q2;
    cx<double> o1 = mkc(1.0, 0.0) - rho[1] * sigma, o2 = mkc(1.0, 0.0) - rho[2] * sigma;
    double o12 = (o1 * o2).re;
    D.c5 = o12 * s0;
    {   // (1 - s r_a)(1 - s r_b) r_m for m = 1, 2 ({a, b} the other slots); real parts
        cx<double> o0 = mkc(1.0 - sigma * s0, 0.0);
        D.c5b = (o0 * o2 * rho[1]).re;
        D.c5c = (o0 * o1 * rho[2]).re;
    }
    D.pre3 = o12 * (1.0 - sigma * s0);
    {   // explicit dependence of the time coordinate's coefficients (t_grad_between)
        const double o0 = 1.0 - sigma * s0;
        const double ro = (rho[1] * o2).re + (rho[2] * o1).re;
        D.tdp3 = -(s0 * o12 + o0 * ro);
        D.tdc5 = -s0 * ro;
        D.tso12 = -sigma * o12;
        D.tr12 = (rho[1] * rho[2]).re;
        const cx<double> q1 = o2 * (-sigma * o0), q2 = o2 * (-sigma * s0), q3 = rho[2] * s0;
        D.tq1re = q1.re; D.tq1im = q1.im; D.tq2re = q2.re; D.tq2im = q2.im; D.tq3re = q3.re; D.tq3im = q3.im;
        D.tq4 = -sigma * o0 * o1.re; D.tq5 = -sigma * s0 * o1.re; D.tq6 = s0 * rho[1].re;
    }
    D.rprod = (rho[0] * rho[1] * rho[2]).re;
    cx<double> d01 = rho[1] - rho[0], d02 = rho[2] - rho[0];
    double d0102 = (d01 * d02).re;
    D.d0102 = d0102;
    D.xc3 = 3.0 * s0 * s0 - d0102;
    D.xc2 = 2.0 * s0 * s0 - d0102;
    D.xs3 = (rho[0] + rho[1] + rho[2]).re;
    D.om1s12 = o12;
    D.op1s3 = 1.0 + sigma * D.xs3;
    D.om1s0 = 1.0 - sigma * s0;
    D.d02re = d02.re; D.d02im = d02.im;
    {   // the coefficients of the regular form of eq. 3.9, as polynomials in sigma
        const double sum12 = (rho[1] + rho[2]).re, prod12 = (rho[1] * rho[2]).re;
        D.xa = -sum12 + sigma * prod12;
        D.xe1 = -2.0 * sum12 + sigma * (prod12 + D.xs3 * s0);
        D.xym = -1.0 / (D.yt + 1.0);
    }
    // Quadrature routes integrate in u = ln x along the half-line u >= 0; the
    // integrand is singular at u = ln(rho_n) (complex log).  Distance of the nearest
    // singularity to that half-line sizes the quadrature panels.
    {
        double dmin = 1e300;
        // (a panel-sizing heuristic: single precision is ample)
        for (int n = 0; n < 3; ++n) {
            double mag = cabs(rho[n]);
            if (!(mag > 0.0)) continue;
            double lr = logf((float)mag), li = atan2f((float)rho[n].im, (float)rho[n].re);
            double d = lr >= 0.0 ? __builtin_fabs(li) : __builtin_sqrt(lr * lr + li * li);
            dmin = d < dmin ? d : dmin;
        }
        if (Or > 0.0) { // radiation root rho_l = 1/sigma < 0: ln rho_l = ln|rho_l| + i pi
            double lr = -logf((float)(-sigma));
            double d = lr >= 0.0 ? M_PI : __builtin_sqrt(lr * lr + M_PI * M_PI);
            dmin = d < dmin ? d : dmin;
        }
        D.dpath = dmin;
    }

    // --- root Jacobian (app. A), FP64
    const double Rp = (4.0 * OL * sigma * sigma + 2.0 * Ok) * sigma + Om; // R'(sigma)
    const double dRdth[3] = {sigma - sigma * sigma, sigma * sigma * sigma * sigma - sigma * sigma,
                             1.0 - sigma * sigma};
    const double dbdth_s[3] = {1.0 - sigma, -sigma + sigma * sigma * sigma, -sigma};
    for (int a = 0; a < 3; ++a) {
        double ds = (Or > 0.0 || a == 2) ? -dRdth[a] / Rp : 0.0;
        rec.dsigma[a] = ds;
        rec.dbeta[a] = dbdth_s[a] + (Ok + 3.0 * sigma * sigma * OL) * ds;
    }
    for (int n = 0; n < 3; ++n) {
        cx<double> den = (mkc(1.0, 0.0) - rho[n] * sigma) * beta;
        for (int m = 0; m < 3; ++m)
            if (m != n) den = den * (rho[n] - rho[m]);
        for (int a = 0; a < 3; ++a) {
            cx<double> v = -cdiv(dP_dtheta(a, rho[n]), den);
            rec.drho_re[n][a] = v.re;
            rec.drho_im[n][a] = v.im;
        }
    }
    rec.beta = beta;
    for (int a = 0; a < 3; ++a) {
        rec.jc32[0][a] = (float)(-rec.dbeta[a] / (2.0 * beta));
        rec.jc32[1][a] = (float)rec.dsigma[a];
        rec.jc32[2][a] = (float)rec.drho_re[0][a];
        rec.jc32[3][a] = (float)(pair ? 2.0 * rec.drho_re[1][a] : rec.drho_re[1][a]);
        rec.jc32[4][a] = (float)(pair ? -2.0 * rec.drho_im[1][a] : rec.drho_re[2][a]);
    }
    rec.rl = Or > 0.0 ? 1.0 / sigma : __builtin_nan("");
    rec.fallback_grad = (minsep < 1e-4) ? 1 : 0;
    bool ok_all = !(info & (COSMO_INFO_RED | COSMO_INFO_DOMAIN));
    // every constant must be finite
    ok_all = ok_all && __builtin_isfinite(D.pre) && __builtin_isfinite(D.y0) && __builtin_isfinite(D.yt);
    rec.valid = ok_all ? 1 : 0;
    rec.info = info;
    fill_lane(rec.f, D);
}

} // namespace cosmo
