// Host build of the per-lane forward formulas (D_C, T, X) for tests.
#include "../../paper_2212_01937_amd/csrc/between.hpp"
using namespace cosmo;
template <typename T, bool PAIR> static double one(const CosmoRec &r, int kind, T z) {
    const LaneConst<T> &k = lane_of<T>(r);
    int route = 0;
    if (kind == COSMO_T) return k.th * t_hat<T, PAIR>(r, z);
    if (kind == COSMO_X) return k.dh * x_hat<T, PAIR>(r, z, route);
    return k.dh * chi_hat<T, PAIR>(k, z);
}
// kind: COSMO_DC, COSMO_T or COSMO_X; dt: 0 FP32, 1 FP64.  NaN for invalid cosmologies.
extern "C" void host_eval(const double *prm, int kind, int dt, const double *z, long n, double *out) {
    CosmoRec r;
    setup_cosmo(prm, r);
    for (long i = 0; i < n; ++i) {
        if (!r.valid) { out[i] = __builtin_nan(""); continue; }
        if (dt == 0) out[i] = r.pair ? one<float, true>(r, kind, (float)z[i]) : one<float, false>(r, kind, (float)z[i]);
        else out[i] = r.pair ? one<double, true>(r, kind, z[i]) : one<double, false>(r, kind, z[i]);
    }
}

// The FP32 time coordinate's FP64 square roots: sqrt_nr from the FP32 root v rsqrt(v) for
// n arguments; and one finite limit's FP64 sides (side_at_mixed) of cosmology prm at
// float z[i]: out[12 i ..] = (t, n0, n1re, n1im, n1abs, n2) and the same from FP64
// square roots of the record's constants.
extern "C" void host_sqrt_nr(const double *x, long n, double *out) {
    for (long i = 0; i < n; ++i) {
        const float xf = (float)x[i], rt = Fp<float>::rsqrt(xf);
        out[i] = sqrt_nr(x[i], xf * rt, rt);
    }
}
extern "C" void host_side_mixed(const double *prm, const double *z, long n, double *out) {
    CosmoRec r;
    setup_cosmo(prm, r);
    const LaneConst<double> &k = r.d;
    for (long i = 0; i < n; ++i) {
        double *o = out + 12 * i;
        const float zf = (float)z[i];
        const double zd = (double)zf;
        if (r.pair) {
            Side<double, true> d; SideG<float, true> g;
            side_at_mixed<true>(r.d, r.f, zf, d, g);
            o[0] = d.t; o[1] = d.n0; o[2] = d.n1re; o[3] = d.n1im; o[4] = d.n1abs; o[5] = d.n2;
        } else {
            Side<double, false> d; SideG<float, false> g;
            side_at_mixed<false>(r.d, r.f, zf, d, g);
            o[0] = d.t; o[1] = d.n0; o[2] = d.n1re; o[3] = d.n1im; o[4] = d.n1abs; o[5] = d.n2;
        }
        // FP64 references from the same record: correctly rounded square roots
        o[6] = __builtin_sqrt(k.yt2 - k.sigma * zd);
        o[7] = __builtin_sqrt(zd + k.w0);
        if (r.pair) {
            double ab;
            const cx<double> n1 = csqrt(mkc(zd + k.w1re, k.w1im), ab);
            o[8] = n1.re; o[9] = n1.im; o[10] = ab; o[11] = 0.0;
        } else {
            o[8] = __builtin_sqrt(zd + k.w1re); o[9] = 0.0; o[10] = 0.0; o[11] = __builtin_sqrt(zd + k.w2);
        }
    }
}

// R_C(x, y) and R_D(y, y, x) (rc_rd_r) for n pairs; out[2 i ..] = (rc, rd).  dt: 0 FP32
// (the host stand-in for the wave vote is the lane's own test), 1 FP64.
extern "C" void host_rc_rd(int dt, const double *x, const double *y, long n, double *out) {
    for (long i = 0; i < n; ++i) {
        if (dt == 0) {
            float rc, rd;
            rc_rd_r((float)x[i], (float)y[i], rc, rd);
            out[2 * i] = rc; out[2 * i + 1] = rd;
        } else {
            rc_rd_r(x[i], y[i], out[2 * i], out[2 * i + 1]);
        }
    }
}

// Structured R_F and R_D(., ., x_k) from one duplication sequence (rfd_s), for a
// triple (x, a, b): pair != 0 -> (x, a + i b, a - i b), else (x, a, b).
// out: rf, rdx, rdy.re, rdy.im, rdz.  dt: 0 FP32, 1 FP64.
extern "C" void host_rfd(int dt, int pair, double x, double a, double b, double *out) {
    if (dt == 0) {
        float rf, rdx, rdz;
        cx<float> rdy;
        if (pair) rfd_s<float, true>((float)x, (float)a, (float)b, rf, rdx, rdy, rdz);
        else rfd_s<float, false>((float)x, (float)a, (float)b, rf, rdx, rdy, rdz);
        out[0] = rf; out[1] = rdx; out[2] = rdy.re; out[3] = rdy.im; out[4] = rdz;
    } else {
        double rf, rdx, rdz;
        cx<double> rdy;
        if (pair) rfd_s<double, true>(x, a, b, rf, rdx, rdy, rdz);
        else rfd_s<double, false>(x, a, b, rf, rdx, rdy, rdz);
        out[0] = rf; out[1] = rdx; out[2] = rdy.re; out[3] = rdy.im; out[4] = rdz;
    }
}

// Observables between z1[i] and z2[i] (between.hpp) for one cosmology; kind:
// COSMO_DC, COSMO_DM, COSMO_DA or COSMO_T; dt: 0 FP32, 1 FP64.
template <typename T, bool PAIR> static double btw(const CosmoRec &r, int kind, T z1, T z2) {
    switch (kind) {
    case COSMO_DC: return eval_between<T, COSMO_DC, PAIR>(r, z1, z2);
    case COSMO_DM: return eval_between<T, COSMO_DM, PAIR>(r, z1, z2);
    case COSMO_DA: return eval_between<T, COSMO_DA, PAIR>(r, z1, z2);
    default: return eval_between<T, COSMO_T, PAIR>(r, z1, z2);
    }
}
extern "C" void host_between(const double *prm, int kind, int dt, const double *z1, const double *z2, long n,
                             double *out) {
    CosmoRec r;
    setup_cosmo(prm, r);
    for (long i = 0; i < n; ++i) {
        if (!r.valid) { out[i] = __builtin_nan(""); continue; }
        if (dt == 0) out[i] = r.pair ? btw<float, true>(r, kind, (float)z1[i], (float)z2[i])
                                     : btw<float, false>(r, kind, (float)z1[i], (float)z2[i]);
        else out[i] = r.pair ? btw<double, true>(r, kind, z1[i], z2[i]) : btw<double, false>(r, kind, z1[i], z2[i]);
    }
}

// Leibniz-rule derivatives of t/(1/H0) between z1 and z2 (gl_time_between), d/d(Om, OL,
// Or) per pair into out[3 n].  dt: 0 FP32, 1 FP64; z2 = inf allowed.
template <typename T, bool PAIR> static void tgb(const CosmoRec &r, T z1, T z2, double *o) {
    T q[3];
    gl_time_between<T, PAIR>(lane_of<T>(r), z1, z2, z2 == Fp<T>::inf(), q);
    o[0] = q[0]; o[1] = q[1]; o[2] = q[2];
}
extern "C" void host_time_between_grad(const double *prm, int dt, const double *z1, const double *z2, long n,
                                       double *out) {
    CosmoRec r;
    setup_cosmo(prm, r);
    for (long i = 0; i < n; ++i) {
        double *o = out + 3 * i;
        if (!r.valid) { o[0] = o[1] = o[2] = __builtin_nan(""); continue; }
        if (dt == 0) {
            if (r.pair) tgb<float, true>(r, (float)z1[i], (float)z2[i], o);
            else tgb<float, false>(r, (float)z1[i], (float)z2[i], o);
        } else {
            if (r.pair) tgb<double, true>(r, z1[i], z2[i], o);
            else tgb<double, false>(r, z1[i], z2[i], o);
        }
    }
}

// R_F, R_J(x, y, z, p) and dR_J/dx from one duplication sequence (rfjx_s): triple as
// host_rfd.  out: rf, rj, jx.  dt: 0 FP32, 1 FP64.
extern "C" void host_rfjx(int dt, int pair, double x, double a, double b, double p, double *out) {
    if (dt == 0) {
        float rf, rj, jx;
        if (pair) rfjx_s<float, true>((float)x, (float)a, (float)b, (float)p, rf, rj, jx);
        else rfjx_s<float, false>((float)x, (float)a, (float)b, (float)p, rf, rj, jx);
        out[0] = rf; out[1] = rj; out[2] = jx;
    } else {
        double rf, rj, jx;
        if (pair) rfjx_s<double, true>(x, a, b, p, rf, rj, jx);
        else rfjx_s<double, false>(x, a, b, p, rf, rj, jx);
        out[0] = rf; out[1] = rj; out[2] = jx;
    }
}

// Route taken by x_hat per redshift (kXRoute*: 0 Carlson in the lane precision, 1 FP64
// re-evaluation of an FP32 lane, 2 quadrature), for one cosmology.
extern "C" void host_x_route(const double *prm, int dt, const double *z, long n, int *route) {
    CosmoRec r;
    setup_cosmo(prm, r);
    for (long i = 0; i < n; ++i) {
        route[i] = -1;
        if (!r.valid) continue;
        if (dt == 0) {
            if (r.pair) x_hat<float, true>(r, (float)z[i], route[i]);
            else x_hat<float, false>(r, (float)z[i], route[i]);
        } else {
            if (r.pair) x_hat<double, true>(r, z[i], route[i]);
            else x_hat<double, false>(r, z[i], route[i]);
        }
    }
}

// Value and derivatives of one lane between z1 and z2 (lane_grad_between, finished with
// the root-Jacobian contraction of app. A as k_finalize_params does): out[6 i ..] =
// (value, d/dOm0, d/dOL0, d/dOr0, d/dz1, d/dz2).  kind: COSMO_DC, COSMO_DM, COSMO_DA or
// COSMO_T; dt: 0 FP32, 1 FP64; z2 = inf allowed.
template <typename T, int KIND, bool PAIR> static void bgr(const CosmoRec &r, T z1, T z2, double *o) {
    LaneGrad2<T> g2;
    lane_grad_between<T, KIND, PAIR>(r, z1, z2, g2);
    const LaneGrad<T> &g = g2.g;
    double p[5];
    for (int i = 0; i < 5; ++i) p[i] = (double)g.p[i];
    o[0] = g.val;
    for (int th = 0; th < 3; ++th) {
        const double base = g.quad ? g.q[th] : root_contract(r, p, th);
        o[1 + th] = (double)g.s * base - (double)g.dok;
    }
    o[4] = g2.dz1;
    o[5] = g.dz;
}
template <typename T, bool PAIR> static void bgk(const CosmoRec &r, int kind, T z1, T z2, double *o) {
    switch (kind) {
    case COSMO_DC: bgr<T, COSMO_DC, PAIR>(r, z1, z2, o); break;
    case COSMO_DM: bgr<T, COSMO_DM, PAIR>(r, z1, z2, o); break;
    case COSMO_DA: bgr<T, COSMO_DA, PAIR>(r, z1, z2, o); break;
    default: bgr<T, COSMO_T, PAIR>(r, z1, z2, o); break;
    }
}
extern "C" void host_between_grad(const double *prm, int kind, int dt, const double *z1, const double *z2, long n,
                                  double *out) {
    CosmoRec r;
    setup_cosmo(prm, r);
    for (long i = 0; i < n; ++i) {
        double *o = out + 6 * i;
        if (!r.valid) { for (int q = 0; q < 6; ++q) o[q] = __builtin_nan(""); continue; }
        if (dt == 0) {
            const float a = (float)z1[i], b = z2[i] == __builtin_inf() ? __builtin_inff() : (float)z2[i];
            if (r.pair) bgk<float, true>(r, kind, a, b, o);
            else bgk<float, false>(r, kind, a, b, o);
        } else {
            if (r.pair) bgk<double, true>(r, kind, z1[i], z2[i], o);
            else bgk<double, false>(r, kind, z1[i], z2[i], o);
        }
    }
}

// sincos_red (the curvature transform's sin and cos) for n arguments; dt: 0 FP32, 1 FP64.
extern "C" void host_sincos(int dt, const double *x, long n, double *s, double *c) {
    for (long i = 0; i < n; ++i) {
        if (dt == 0) {
            float sf, cf;
            sincos_red<float>((float)x[i], sf, cf);
            s[i] = sf; c[i] = cf;
        } else {
            sincos_red<double>(x[i], s[i], c[i]);
        }
    }
}

// The FP64 lane path's log10 and exp (mu and the curvature transform's closed forms).
extern "C" void host_log10_exp(const double *x, long n, double *lg, double *ex) {
    for (long i = 0; i < n; ++i) {
        lg[i] = Fp<double>::log10_fast(x[i]);
        ex[i] = Fp<double>::exp_fast(x[i]);
    }
}
