// adjoint.hpp -- derivatives of one (cosmology, redshift) lane, shared by the
// adjoint (vector-Jacobian product) and the materialised-Jacobian kernels.
//
// Routes: the root chain (Carlson derivatives, eqs. 2.10-2.11, through the root
// Jacobian of app. A), or Leibniz-rule quadrature of the defining integrals
// (eqs. 2.3-2.5 differentiated under the integral) where the chain is ill
// conditioned: near-multiple roots, X, and FP32 lanes at small z.
#pragma once

#include "lane.hpp"

namespace cosmo {

// Route predicates of the adjoint (the kernels branch on exactly these; the route
// counts of cosmo_route_counts use them too).  Per cosmology: all gradients by
// quadrature for X and for roots closer than the precision's threshold (the
// COSMO_INFO_NEAR_MULTIROOT bits).
__device__ __forceinline__ bool direct_mode(int kind, const CosmoRec &r, bool fp32) {
    if (kind == COSMO_X) return true;
    // minsep below 2e-2 (FP32) / 1e-4 (FP64), as the set-up recorded it in the info bits
    // (an integer test on the record instead of an FP64 compare against a literal)
    return (r.info & (fp32 ? COSMO_INFO_NEAR_MULTIROOT_F32 : COSMO_INFO_NEAR_MULTIROOT)) != 0;
}

// Near-multiple roots (direct mode): chi and its parameter gradient by quadrature in
// the lane's precision (no cancellation on this route, so FP32 lanes keep FP32
// accuracy).  The FP32 kernels inline the FP32 quadrature: an out-of-line call makes a
// kernel reserve the callee's registers on every lane, which for the FP64 quadrature
// would cost the FP32 adjoint two fifths of its occupancy.  The FP64 kernels keep the
// quadrature out of line (their own register use is higher).  Results come back by
// value: an output array whose address escapes into the call would move the
// caller's per-lane state to scratch memory.
struct GlChi {
    double chi, g0, g1, g2;
};
template <bool PAIR> __device__ __attribute__((noinline)) GlChi gl_chi_grad(const CosmoRec &r, double z) {
    double chi, g[3];
    gl_integral<double, PAIR>(r.d, z, 0, true, chi, g);
    return GlChi{chi, g[0], g[1], g[2]};
}

// FP32 small-z lanes.  There the partials in the root parameters are O(z) while the
// parameter derivatives they contract to are O(z^2) (E(0) = 1 for every theta), so
// FP32 partials lose about eps_32 / z in the contraction.  Below kSmallZ32 the FP32
// path takes the Leibniz-rule quadrature in the lane's precision instead, which has
// no such cancellation; one 8-node panel suffices there (the panel is a fraction of
// the distance to the nearest singularity of the integrand).
constexpr float kSmallZ32 = 0.02f;
// Per lane, on root-chain cosmologies: the FP32 small-z quadrature.
template <typename T> __device__ __forceinline__ bool small_z_lane(T z) { return sizeof(T) == 4 && z < T(kSmallZ32); }
// Whether the adjoint of lane (r, z) takes the Leibniz quadrature.
template <typename T> __device__ __forceinline__ bool adjoint_quadrature_lane(int kind, const CosmoRec &r, T z) {
    return direct_mode(kind, r, sizeof(T) == 4) || small_z_lane<T>(z);
}

// Derivatives of one (cosmology, redshift) lane.  The observable is out = F(base, Ok, z,
// H0) with base = chi (D_C family), t (T) or X; s = dF/dbase.
//   root mode:   p[0..4] = base and its partials in the root parameters (sigma,
//                rho_0, rho_1 re/im for a pair or rho_1, rho_2), all at fixed beta:
//                dbase/dtheta = -p0/(2 beta) dbeta/dtheta + sum p_k drho_k/dtheta;
//   quadrature:  q[0..2] = dbase/d(Om, OL, Or) by Leibniz-rule quadrature (near-multiple
//                roots and X: FP64 / lane precision; FP32 lanes at z < kSmallZ32).
// dok = dF/dOk at fixed base (the curvature transform; dOk/dtheta = -1), dh = dF/dH0,
// dz = dF/dz (fundamental theorem of calculus).
template <typename T> struct LaneGrad {
    T val, s, dok, dh, dz;
    T p[5];
    double q[3];
    bool quad; // this lane's parameter partials are q (quadrature) rather than p
};

template <typename T, int KIND, bool PAIR>
__device__ __forceinline__ void lane_grad(const CosmoRec &r, T z, LaneGrad<T> &o, bool &used_gl) {
    const LaneConst<T> &k = lane_of<T>(r);
    const bool fp32 = sizeof(T) == 4;
    const T H0inv = k.hinv;
    o.dok = T(0);
    o.quad = false;
    const bool small = small_z_lane<T>(z);
    if (KIND == COSMO_T && !direct_mode(KIND, r, fp32)) {
        // time coordinate: Carlson derivatives (eqs. 2.10, 2.11) and the root chain
        if (small) {
            T tv, g[3];
            gl_integral<T, PAIR>(k, z, 1, true, tv, g, 1);
            o.p[0] = tv;
            o.q[0] = g[0]; o.q[1] = g[1]; o.q[2] = g[2];
            o.quad = true;
        } else {
            TGrad<T, PAIR> tg;
            t_grad<T, PAIR>(r, z, tg);
            o.p[0] = tg.t; o.p[1] = tg.dsig; o.p[2] = tg.dr0; o.p[3] = tg.dr1re; o.p[4] = PAIR ? tg.dr1im : tg.dr2;
        }
        o.s = k.th;
        o.val = k.th * o.p[0];
        o.dh = -o.val * H0inv;
        o.dz = k.th * Fp<T>::rcp(T(1) + z) * iEz<T>(k, z);
        return;
    }
    if (KIND == COSMO_T || KIND == COSMO_X) {
        T qv, g[3];
        gl_integral<T, PAIR>(k, z, KIND == COSMO_T ? 1 : 2, true, qv, g);
        o.s = KIND == COSMO_T ? k.th : k.dh;
        const T x = T(1) + z;
        const T e = Ez<T>(k, z);
        o.dz = o.s * (KIND == COSMO_T ? Fp<T>::rcp(x * e) : x * x * Fp<T>::rcp(e));
        // the value (also needed for the H0 derivative) by the forward's route
        if (KIND == COSMO_T) {
            o.val = k.th * t_hat<T, PAIR>(r, z);
        } else {
            int route;
            o.val = k.dh * x_hat<T, PAIR>(r, z, route);
            used_gl = route == kXRouteQuad;
        }
        o.q[0] = g[0]; o.q[1] = g[1]; o.q[2] = g[2];
        o.quad = true;
        o.dh = -o.val * H0inv;
        return;
    }
    T dzz, ie; // ie = 1/E(z)
    if (direct_mode(KIND, r, fp32)) {
        // near-multiple roots: chi and its parameter gradient by FP64 quadrature
        T chi;
        if (fp32) {
            T g[3];
            gl_integral<T, PAIR>(k, z, 0, true, chi, g);
            o.q[0] = g[0]; o.q[1] = g[1]; o.q[2] = g[2];
        } else {
            const GlChi gc = gl_chi_grad<PAIR>(r, (double)z);
            chi = T(gc.chi);
            o.q[0] = gc.g0; o.q[1] = gc.g1; o.q[2] = gc.g2;
        }
        o.quad = true;
        ie = iEz<T>(k, z);
        o.val = observable<T>(KIND, k, chi, z, H0inv, o.s, o.dok, dzz, o.dh);
    } else {
        if (small) {
            T cv, g[3];
            gl_integral<T, PAIR>(k, z, 0, true, cv, g, 1);
            o.p[0] = cv;
            o.q[0] = g[0]; o.q[1] = g[1]; o.q[2] = g[2];
            o.quad = true;
            ie = iEz<T>(k, z);
        } else {
            ChiGrad<T, PAIR> cg;
            chi_grad<T, PAIR>(k, z, cg);
            o.p[0] = cg.chi; o.p[1] = cg.kr * cg.dsig; o.p[2] = cg.kr * cg.dr0; o.p[3] = cg.kr * cg.dr1re;
            o.p[4] = cg.kr * (PAIR ? cg.dr1im : cg.dr2);
            ie = cg.iE;
        }
        o.val = observable<T>(KIND, k, o.p[0], z, H0inv, o.s, o.dok, dzz, o.dh);
    }
    o.dz = dzz + o.s * ie;
}

// The common lane of the adjoint: root-chain route (separated roots, KIND not X), and
// on the FP32 path z at or above kSmallZ32.  The same arithmetic as lane_grad's
// root-chain branches, without the quadrature routes (which the kernels run in a
// separate pass over the few lanes that need them, so their registers and branches
// stay out of the main loop).
template <typename T> struct RootGrad {
    T val, s, dok, dh, dz;
    T p[5]; // p[1..4] divided by ps: the partials are (p[0], ps p[1], ..., ps p[4])
    T ps;
};

template <typename T, int KIND, bool PAIR>
__device__ __forceinline__ void lane_grad_root(const CosmoRec &r, T z, RootGrad<T> &o) {
    const LaneConst<T> &k = lane_of<T>(r);
    const T H0inv = k.hinv;
    if (KIND == COSMO_T) {
        TGrad<T, PAIR> tg;
        t_grad<T, PAIR>(r, z, tg);
        o.p[0] = tg.t; o.p[1] = tg.dsig; o.p[2] = tg.dr0; o.p[3] = tg.dr1re; o.p[4] = PAIR ? tg.dr1im : tg.dr2;
        o.ps = T(1);
        o.s = k.th;
        o.val = k.th * o.p[0];
        o.dok = T(0);
        o.dh = -o.val * H0inv;
        o.dz = k.th * Fp<T>::rcp(T(1) + z) * iEz<T>(k, z);
        return;
    }
    ChiGrad<T, PAIR> cg;
    chi_grad<T, PAIR>(k, z, cg);
    o.p[0] = cg.chi; o.p[1] = cg.dsig; o.p[2] = cg.dr0; o.p[3] = cg.dr1re; o.p[4] = PAIR ? cg.dr1im : cg.dr2;
    o.ps = cg.kr;
    T dzz;
    o.val = observable<T>(KIND, k, o.p[0], z, H0inv, o.s, o.dok, dzz, o.dh);
    o.dz = dzz + o.s * cg.iE;
}

// FP32 lanes below kSmallZ32 on root-chain cosmologies: lane_grad's one-panel
// Leibniz quadrature (chi family and T).  Parameter partials in q (d/d(Om, OL, Or)).
template <typename T, int KIND, bool PAIR>
__device__ __forceinline__ void lane_grad_small(const CosmoRec &r, T z, LaneGrad<T> &o) {
    const LaneConst<T> &k = lane_of<T>(r);
    const T H0inv = k.hinv;
    T v, g[3];
    gl_integral<T, PAIR>(k, z, KIND == COSMO_T ? 1 : 0, true, v, g, 1);
    o.q[0] = g[0]; o.q[1] = g[1]; o.q[2] = g[2];
    o.quad = true;
    o.p[0] = v;
    if (KIND == COSMO_T) {
        o.s = k.th;
        o.val = k.th * v;
        o.dok = T(0);
        o.dh = -o.val * H0inv;
        o.dz = k.th * Fp<T>::rcp(T(1) + z) * iEz<T>(k, z);
        return;
    }
    T dzz;
    o.val = observable<T>(KIND, k, v, z, H0inv, o.s, o.dok, dzz, o.dh);
    o.dz = dzz + o.s * iEz<T>(k, z);
}

// Contraction of root-space partials with the root Jacobian (app. A), FP64:
// d base / d theta for theta = (Om, OL, Or).  a[0..4] as LaneGrad::p (or their
// cotangent-weighted sums).
__device__ __forceinline__ double root_contract(const CosmoRec &r, const double a[5], int th, double *mag = nullptr) {
    double t[5];
    t[0] = -a[0] / (2.0 * r.beta) * r.dbeta[th];
    t[1] = a[1] * r.dsigma[th];
    t[2] = a[2] * r.drho_re[0][th];
    if (r.pair) {
        t[3] = 2.0 * a[3] * r.drho_re[1][th];
        t[4] = -2.0 * a[4] * r.drho_im[1][th];
    } else {
        t[3] = a[3] * r.drho_re[1][th];
        t[4] = a[4] * r.drho_re[2][th];
    }
    if (mag) *mag = __builtin_fabs(t[0]) + __builtin_fabs(t[1]) + __builtin_fabs(t[2]) + __builtin_fabs(t[3]) +
                    __builtin_fabs(t[4]);
    return t[0] + t[1] + t[2] + t[3] + t[4];
}

// The contraction above cancels when beta is small and at small z (E(0) = 1 for every
// theta: the O(z) parts of the root partials sum to zero), by up to ~1e3-1e4 on the
// workloads for the Om0 and Or0 components.  Per-lane consumers in FP32 (the
// materialised Jacobian) recompute a lane whose contraction cancels by more than
// kJacCancel32 by Leibniz-rule quadrature in FP32 (no cancellation there).
constexpr double kJacCancel32 = 64.0;

} // namespace cosmo
