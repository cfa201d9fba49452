/*
 * oracle.c -- plain, slow, FP64 reference for the distance integrals of
 * Karchev, "Analytic auto-differentiable LambdaCDM cosmography" (arXiv:2212.01937).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, constant table or helper with the
 * HIP library: it evaluates the *defining integrals* by adaptive quadrature,
 * whereas the library evaluates the paper's Carlson reductions.
 *
 * What it computes (all in FP64):
 *   E^2(z) = Or (1+z)^4 + Om (1+z)^3 + Ok (1+z)^2 + OL          (sec. 2.1, eq. 2.2)
 *   Ok     = 1 - Om - OL - Or                                     (sec. 2.1, closure)
 *   D_C    = (c/H0)  int_0^z dz'/E                                (eq. 2.3)
 *   T      = (1/H0)  int_0^z dz'/((1+z')E)   (lookback time)      (eq. 2.4)
 *   X      = (c/H0)  int_0^z (1+z')^2/E dz'  (absorption dist.)   (eq. 2.5)
 *   D_M    = curvature-modified comoving distance (sin/sinh of D_C), D_L = (1+z) D_M,
 *   D_A    = D_M/(1+z), mu = 5 log10(D_L / 10 pc)                  (sec. 2.1.1; fn. 22)
 * between two redshifts (oracle_between): chi(z1, z2), t(z1, z2), d_abs(z1, z2) of eqs.
 * 2.3-2.5 with both limits free (z2 = +inf for chi and t: the age t(z, inf), sec. 2.1),
 * D_M(z1, z2) = sinn of chi(z1, z2) and D_A(z1, z2) = D_M(z1, z2)/(1+z2);
 * and their gradients with respect to (H0, Om, OL, Or, z) by the Leibniz
 * integral rule (differentiation under the integral sign, as the HMC analyses
 * quoted in sec. 4, fn. 23 do), Ok being eliminated through the closure.
 *
 * Quadrature: global adaptive bisection driven by the 7-point Gauss / 15-point
 * Kronrod pair (the QUADPACK rule that scipy.integrate.quad uses, which is the
 * paper's own numerical baseline, sec. 3.2.1, fn. 18).  Error estimate of a
 * panel = |K15 - G7|, deliberately pessimistic.  The distance integrals are taken
 * in u = ln(1+z) (dz = (1+z) du), which keeps the integrands smooth.
 *
 * The Carlson symmetric integrals R_F, R_J (eqs. 2.6, 2.7) and their degenerate
 * forms R_C, R_D (eqs. 2.8, 2.9) are evaluated by the same quadrature of their
 * defining integrals (complex arguments off the non-positive real axis; the
 * Cauchy principal value for a negative real w is not covered and yields NaN).
 *
 * Units: c = 299792.458 km/s, H0 in km/s/Mpc, distances in Mpc, times in Gyr
 * (1 Mpc = 3.0856775814913673e19 km, 1 Gyr = 3.15576e16 s, Julian years),
 * mu in magnitudes.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define C_KMS 299792.458
#define MPC_KM 3.0856775814913673e19
#define GYR_S 3.15576e16
#define FOUR_PI 12.566370614359172953850573533118

/* ---------------------------------------------------------------------------
 * 7/15-point Gauss-Kronrod rule on [-1, 1] (nodes/weights of QUADPACK qk15).
 * Index 0 is the outermost node; XGK[7] = 0 is the centre.  The Gauss nodes are
 * XGK[1], XGK[3], XGK[5], XGK[7] with weights WG[0..3].
 * ------------------------------------------------------------------------- */
static const double XGK[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double WGK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

typedef double (*integrand_fn)(double t, const void *ctx);

/* One G7K15 panel on [a, b]: returns the Kronrod value, *err = |K15 - G7|. */
static double gk15(integrand_fn f, const void *ctx, double a, double b, double *err)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double fc = f(c, ctx);
    double resk = WGK[7] * fc, resg = WG[3] * fc;
    for (int j = 0; j < 7; ++j) {
        double dx = h * XGK[j];
        double f1 = f(c - dx, ctx), f2 = f(c + dx, ctx);
        resk += WGK[j] * (f1 + f2);
        if (j % 2 == 1) resg += WG[j / 2] * (f1 + f2);
    }
    *err = fabs((resk - resg) * h);
    return resk * h;
}

/* Exposed so that the rule itself can be pinned (polynomial exactness). */
double oracle_gk15_panel(int which_rule, int power, double a, double b);

struct panel { double a, b, r, e; };

#define QUAD_LIMIT 4000

/* Global adaptive quadrature: bisect the panel with the largest error estimate
 * until sum(err) <= max(epsabs, epsrel*|sum(result)|) or the panel budget is used.
 * Returns the integral; *abserr receives the summed error estimate (NaN result
 * if the integrand produced NaN). */
static double adapt(integrand_fn f, const void *ctx, double a, double b,
                    double epsabs, double epsrel, double *abserr)
{
    if (b < a) return -adapt(f, ctx, b, a, epsabs, epsrel, abserr); /* bisection needs a < b */
    struct panel *p = (struct panel *)malloc(sizeof(struct panel) * QUAD_LIMIT);
    int n = 1;
    p[0].a = a; p[0].b = b;
    p[0].r = gk15(f, ctx, a, b, &p[0].e);
    double res = p[0].r, err = p[0].e;
    while (n < QUAD_LIMIT) {
        if (!(err > fmax(epsabs, epsrel * fabs(res)))) break; /* also exits on NaN */
        int worst = 0;
        for (int k = 1; k < n; ++k)
            if (p[k].e > p[worst].e) worst = k;
        double m = 0.5 * (p[worst].a + p[worst].b);
        if (!(m > p[worst].a && m < p[worst].b)) break; /* panel at rounding level */
        struct panel L = {p[worst].a, m, 0, 0}, R = {m, p[worst].b, 0, 0};
        L.r = gk15(f, ctx, L.a, L.b, &L.e);
        R.r = gk15(f, ctx, R.a, R.b, &R.e);
        p[worst] = L;
        p[n++] = R;
        res = 0.0; err = 0.0; /* re-sum from scratch: no running-sum drift */
        for (int k = 0; k < n; ++k) { res += p[k].r; err += p[k].e; }
    }
    free(p);
    if (abserr) *abserr = err;
    return res;
}

/* ---------------------------------------------------------------------------
 * Cosmology and the distance integrands (in u = ln(1+z), x = 1+z = e^u).
 * ------------------------------------------------------------------------- */
struct cosmo { double H0, Om, OL, Or, Ok; };

/* eq. 2.2 written out term by term */
static double E2_of_x(const struct cosmo *c, double x)
{
    return c->Or * x * x * x * x + c->Om * x * x * x + c->Ok * x * x + c->OL;
}

/* Partial derivative of E^2 with respect to parameter a (1: Om, 2: OL, 3: Or) with
 * Ok = 1 - Om - OL - Or eliminated, i.e. dE2/dOm = x^3 - x^2, dE2/dOL = 1 - x^2,
 * dE2/dOr = x^4 - x^2.  Each has the factor x - 1, passed in as xm1 = expm1(u) so
 * that the differences do not cancel near x = 1 (low z). */
static double dE2_dparam(int a, double x, double xm1)
{
    switch (a) {
    case 1: return x * x * xm1;
    case 2: return -xm1 * (x + 1.0);
    case 3: return x * x * xm1 * (x + 1.0);
    }
    return 0.0;
}

/* Which of the three defining integrals: power of (1+z) multiplying 1/E in dz. */
enum { INT_CHI = 0, INT_T = 1, INT_ABS = 2 };

static double integrand_power(int which)
{
    return which == INT_CHI ? 0.0 : (which == INT_T ? -1.0 : 2.0);
}

/* x = x0 e^u: x0 = 1 for integrals from z = 0 (u = ln(1+z)); x0 = 1 + z1 from a lower
 * limit z1, which keeps the interval [0, ln((1+z2)/(1+z1))] exact for close limits. */
struct ictx { const struct cosmo *c; int which; int dparam; double x0; };

/* Integrand in u.  dparam == 0: (1+z)^p / E * dz/du.  dparam = a > 0: its partial
 * derivative with respect to parameter a, i.e. -(1/2) (1+z)^p (dE2/da) / E^3 * dz/du. */
static double dist_integrand(double u, const void *vctx)
{
    const struct ictx *k = (const struct ictx *)vctx;
    double x = k->x0 * exp(u);
    double e2 = E2_of_x(k->c, x);
    double e = sqrt(e2);
    double g = pow(x, integrand_power(k->which)) * x; /* (1+z)^p * dz/du */
    if (k->dparam == 0) return g / e;
    double xm1 = k->x0 == 1.0 ? expm1(u) : x - 1.0;
    return -0.5 * g * dE2_dparam(k->dparam, x, xm1) / (e2 * e);
}

static const double EPSREL = 1e-14;

/* Dimensionless integral int_0^z (1+z')^p / E dz' (dparam = 0) or its Leibniz
 * derivative (dparam = 1..3). */
static double dimless_integral(const struct cosmo *c, int which, int dparam, double z,
                               double *abserr)
{
    struct ictx k = {c, which, dparam, 1.0};
    if (z == 0.0) { if (abserr) *abserr = 0.0; return 0.0; }
    return adapt(dist_integrand, &k, 0.0, log1p(z), 0.0, EPSREL, abserr);
}

/* Integrand to an infinite upper limit.  With a = 1/x = s^2 (x = 1 + z):
 *   dz / E          = da / sqrt(P(a))          = 2 s ds / sqrt(P(s^2)),
 *   dz / ((1+z) E)  = a da / sqrt(P(a))        = 2 s^3 ds / sqrt(P(s^2)),
 * P(a) = a^4 E^2(1/a) = Or + Om a + Ok a^2 + OL a^4; s runs over [0, 1/sqrt(1+z1)].
 * (The s-form stays bounded at s -> 0 also for Or = 0.) */
static double inf_integrand(double s, const void *vctx)
{
    const struct ictx *k = (const struct ictx *)vctx;
    const struct cosmo *c = k->c;
    double a = s * s;
    double P = c->Or + c->Om * a + c->Ok * a * a + c->OL * a * a * a * a;
    double num = k->which == INT_CHI ? 2.0 * s : 2.0 * s * s * s;
    if (k->dparam == 0) return num / sqrt(P);
    /* Leibniz: -1/2 num (dP/dtheta) / P^(3/2), Ok eliminated: dP/dOm = a - a^2,
     * dP/dOL = a^4 - a^2, dP/dOr = 1 - a^2 */
    double dP = k->dparam == 1 ? a - a * a : (k->dparam == 2 ? a * a * a * a - a * a : 1.0 - a * a);
    return -0.5 * num * dP / (P * sqrt(P));
}

/* Dimensionless integral from z1 to z2 (either order; z2 = +inf for the comoving
 * distance and the time coordinate; the absorption distance diverges there). */
static double dimless_between(const struct cosmo *c, int which, int dparam, double z1, double z2, double *abserr)
{
    if (abserr) *abserr = 0.0;
    if (isinf(z2) && z2 > 0.0) {
        if (which == INT_ABS) return INFINITY;
        struct ictx k = {c, which, dparam, 1.0};
        /* panels [s1 10^-(j+1), s1 10^-j], j < 16, and [0, s1 1e-16]: the integrand has
         * structure at the scale sqrt(Or/Om) (where radiation takes over from matter),
         * which a single interval's first bisections would not sample */
        double s1 = 1.0 / sqrt(1.0 + z1), hi = s1, sum = 0.0, e = 0.0, ej;
        for (int j = 0; j < 16; ++j) {
            double lo = hi * 0.1;
            sum += adapt(inf_integrand, &k, lo, hi, 0.0, EPSREL, &ej);
            e += ej;
            hi = lo;
        }
        sum += adapt(inf_integrand, &k, 0.0, hi, 0.0, EPSREL, &ej);
        if (abserr) *abserr = e + ej;
        return sum;
    }
    if (z1 == z2) return 0.0;
    struct ictx k = {c, which, dparam, 1.0 + z1};
    return adapt(dist_integrand, &k, 0.0, log1p((z2 - z1) / (1.0 + z1)), 0.0, EPSREL, abserr);
}

/* ---------------------------------------------------------------------------
 * Output kinds (numbering matches the public ABI's enumeration of observables).
 * ------------------------------------------------------------------------- */
enum { K_DC = 0, K_DM = 1, K_DL = 2, K_MU = 3, K_T = 4, K_X = 5, K_DA = 6, K_VC = 7 };

/* Curvature transform S_k(chi) = sinh(sqrt(Ok) chi)/sqrt(Ok) (Ok > 0), chi (Ok = 0),
 * sin(sqrt(-Ok) chi)/sqrt(-Ok) (Ok < 0), with chi = D_C/D_H dimensionless.
 * Also returns dS/dchi and dS/dOk. */
static void curvature_transform(double ok, double chi, double *S, double *dS_dchi, double *dS_dok)
{
    if (ok > 0.0) {
        double s = sqrt(ok);
        *S = sinh(s * chi) / s;
        *dS_dchi = cosh(s * chi);
    } else if (ok < 0.0) {
        double s = sqrt(-ok);
        *S = sin(s * chi) / s;
        *dS_dchi = cos(s * chi);
    } else {
        *S = chi;
        *dS_dchi = 1.0;
    }
    /* dS/dOk from the power series S = sum_n Ok^n chi^(2n+1)/(2n+1)!, which holds for
     * both signs; the closed form (chi*cosh - sinh/s)/(2 Ok) cancels for small Ok chi^2. */
    double t = ok * chi * chi;
    if (fabs(t) < 1.0) {
        double term = chi * chi * chi / 6.0; /* n = 1 term of dS/dOk: chi^3/3! */
        double sum = 0.0;
        for (int n = 1; n < 40; ++n) {
            sum += term;
            /* next: (n+1) Ok^n chi^(2n+3)/(2n+3)!  from  n Ok^(n-1) chi^(2n+1)/(2n+1)! */
            term *= (double)(n + 1) / (double)n * t / ((2.0 * n + 2.0) * (2.0 * n + 3.0));
        }
        *dS_dok = sum;
    } else {
        /* dS/dOk = (chi dS/dchi - S) / (2 Ok) for Ok != 0 */
        *dS_dok = (chi * (*dS_dchi) - *S) / (2.0 * ok);
    }
}

static double volume_one(const double *prm, double z, double *grad, double *errest);

/* One evaluation: value of `kind` at (cosmology, z) and, if grad != NULL, its
 * gradient with respect to (H0, Om, OL, Or, z) in grad[0..4]. */
static double eval_one(int kind, const double *prm, double z, double *grad, double *errest)
{
    if (kind == K_VC) return volume_one(prm, z, grad, errest);
    struct cosmo c;
    c.H0 = prm[0]; c.Om = prm[1]; c.OL = prm[2]; c.Or = prm[3];
    c.Ok = 1.0 - c.Om - c.OL - c.Or;
    double DH = C_KMS / c.H0;               /* Hubble distance, Mpc */
    double tH = MPC_KM / (c.H0 * GYR_S);    /* Hubble time, Gyr */
    double x = 1.0 + z;
    double Ez = sqrt(E2_of_x(&c, x));
    double err = 0.0;

    if (kind == K_T || kind == K_X) {
        int which = kind == K_T ? INT_T : INT_ABS;
        double scale = kind == K_T ? tH : DH;
        double integ = dimless_integral(&c, which, 0, z, &err);
        double val = scale * integ;
        if (grad) {
            grad[0] = -val / c.H0;
            for (int a = 1; a <= 3; ++a) grad[a] = scale * dimless_integral(&c, which, a, z, NULL);
            grad[4] = scale * pow(x, integrand_power(which)) / Ez; /* fundamental theorem */
        }
        if (errest) *errest = scale * err;
        return val;
    }

    /* comoving-distance family */
    double chi = dimless_integral(&c, INT_CHI, 0, z, &err); /* D_C / D_H */
    double dchi[5] = {0, 0, 0, 0, 0};                          /* d chi / d(H0,Om,OL,Or,z) */
    if (grad) {
        for (int a = 1; a <= 3; ++a) dchi[a] = dimless_integral(&c, INT_CHI, a, z, NULL);
        dchi[4] = 1.0 / Ez;
    }
    if (kind == K_DC) {
        double val = DH * chi;
        if (grad) {
            grad[0] = -val / c.H0;
            for (int a = 1; a <= 4; ++a) grad[a] = DH * dchi[a];
        }
        if (errest) *errest = DH * err;
        return val;
    }
    double S, dS_dchi, dS_dok;
    curvature_transform(c.Ok, chi, &S, &dS_dchi, &dS_dok);
    double DM = DH * S;
    double dDM[5];
    dDM[0] = -DM / c.H0;
    for (int a = 1; a <= 3; ++a) dDM[a] = DH * (dS_dchi * dchi[a] - dS_dok); /* dOk/da = -1 */
    dDM[4] = DH * dS_dchi * dchi[4];
    if (errest) *errest = DH * fabs(dS_dchi) * err;

    double val;
    double dval[5];
    if (kind == K_DM) {
        val = DM;
        memcpy(dval, dDM, sizeof dval);
    } else if (kind == K_DA) {
        val = DM / x;
        for (int a = 0; a < 4; ++a) dval[a] = dDM[a] / x;
        dval[4] = dDM[4] / x - DM / (x * x);
        if (errest) *errest /= x;
    } else { /* D_L or mu */
        double DL = x * DM;
        double dDL[5];
        for (int a = 0; a < 4; ++a) dDL[a] = x * dDM[a];
        dDL[4] = DM + x * dDM[4];
        if (kind == K_DL) {
            val = DL;
            memcpy(dval, dDL, sizeof dval);
            if (errest) *errest *= x;
        } else {
            /* mu = 5 log10(D_L / 10 pc) = 5 log10(D_L / Mpc) + 25 (fn. 22) */
            val = 5.0 * log10(DL) + 25.0;
            double k = 5.0 / (log(10.0) * DL);
            for (int a = 0; a < 5; ++a) dval[a] = k * dDL[a];
            if (errest) *errest *= x * k;
        }
    }
    if (grad) memcpy(grad, dval, sizeof dval);
    return val;
}

/* All-sky comoving volume V_C(z) = 4 pi int_0^z D_M(z')^2 dD_C(z')  (sec. 2.1; dD_C =
 * (c/H0) dz'/E), by quadrature in u = ln(1+z') over this file's own D_M(z') (itself a
 * quadrature).  The parameter gradient is the same integral of the derivatives of the
 * integrand (Leibniz rule), with D_M's gradient from eval_one; d/dz by the fundamental
 * theorem of calculus. */
struct vctx { const double *prm; int a; }; /* a < 0: value; 0..3: d/d(H0, Om, OL, Or) */

static double vol_integrand(double u, const void *vctx)
{
    const struct vctx *k = (const struct vctx *)vctx;
    const double *prm = k->prm;
    struct cosmo c = {prm[0], prm[1], prm[2], prm[3], 1.0 - prm[1] - prm[2] - prm[3]};
    double x = exp(u), z = expm1(u);
    double g[5];
    double dm = eval_one(K_DM, prm, z, k->a >= 0 ? g : NULL, NULL);
    double e2 = E2_of_x(&c, x);
    double f = (C_KMS / c.H0) * x / sqrt(e2); /* dD_C/du */
    if (k->a < 0) return FOUR_PI * dm * dm * f;
    double df = k->a == 0 ? -f / c.H0 : -0.5 * f * dE2_dparam(k->a, x, z) / e2;
    return FOUR_PI * (2.0 * dm * g[k->a] * f + dm * dm * df);
}

static double volume_one(const double *prm, double z, double *grad, double *errest)
{
    double err = 0.0;
    if (z == 0.0) {
        if (grad) memset(grad, 0, 5 * sizeof(double));
        if (errest) *errest = 0.0;
        return 0.0;
    }
    struct vctx k = {prm, -1};
    double val = adapt(vol_integrand, &k, 0.0, log1p(z), 0.0, EPSREL, &err);
    if (errest) *errest = err;
    if (grad) {
        for (int a = 0; a < 4; ++a) {
            struct vctx ka = {prm, a};
            grad[a] = adapt(vol_integrand, &ka, 0.0, log1p(z), 0.0, EPSREL, NULL);
        }
        struct cosmo c = {prm[0], prm[1], prm[2], prm[3], 1.0 - prm[1] - prm[2] - prm[3]};
        double dm = eval_one(K_DM, prm, z, NULL, NULL);
        grad[4] = FOUR_PI * dm * dm * (C_KMS / c.H0) / sqrt(E2_of_x(&c, 1.0 + z));
    }
    return val;
}

/* Batched driver.  params: [n_cosmo][4] = (H0, Om, OL, Or); z[c*z_stride + i];
 * out[c*n_z + i]; grad (nullable): [n_cosmo][n_z][5]; errest (nullable): like out.
 * Returns 0, or -1 on bad arguments.  nthreads <= 0 means "all OpenMP threads". */
int oracle_eval(int kind, const double *params, long n_cosmo, const double *z, long n_z,
                long z_stride, double *out, double *grad, double *errest, int nthreads)
{
    if (kind < 0 || kind > 7 || n_cosmo < 0 || n_z < 0 || !params || !z || !out) return -1;
    long total = n_cosmo * n_z;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
#endif
    for (long idx = 0; idx < total; ++idx) {
        long ci = idx / n_z, i = idx % n_z;
        double e;
        out[idx] = eval_one(kind, params + 4 * ci, z[ci * z_stride + i],
                            grad ? grad + 5 * idx : NULL, &e);
        if (errest) errest[idx] = e;
    }
    (void)nthreads;
    return 0;
}

/* Between two redshifts: kind K_DC, K_DM, K_DA, K_T or K_X at (z1, z2) of one
 * cosmology.  D_M(z1, z2) = (c/H0) sinn(chi(z1, z2)), D_A(z1, z2) = D_M(z1, z2)/(1+z2).
 * grad (nullable): d/d(H0, Om, OL, Or, z1, z2) in grad[0..5] (Leibniz rule for the
 * parameters, the fundamental theorem for the limits; d/dz2 = 0 at z2 = inf). */
static double between_one(int kind, const double *prm, double z1, double z2, double *grad)
{
    struct cosmo c;
    c.H0 = prm[0]; c.Om = prm[1]; c.OL = prm[2]; c.Or = prm[3];
    c.Ok = 1.0 - c.Om - c.OL - c.Or;
    double DH = C_KMS / c.H0;
    double tH = MPC_KM / (c.H0 * GYR_S);
    int zinf = isinf(z2) && z2 > 0.0;
    double x1 = 1.0 + z1, x2 = 1.0 + z2;
    double iE1 = 1.0 / sqrt(E2_of_x(&c, x1)), iE2 = zinf ? 0.0 : 1.0 / sqrt(E2_of_x(&c, x2));
    if (kind == K_T || kind == K_X) {
        int which = kind == K_T ? INT_T : INT_ABS;
        double scale = kind == K_T ? tH : DH;
        double val = scale * dimless_between(&c, which, 0, z1, z2, NULL);
        if (grad) {
            grad[0] = -val / c.H0;
            for (int a = 1; a <= 3; ++a) grad[a] = scale * dimless_between(&c, which, a, z1, z2, NULL);
            double p = integrand_power(which);
            grad[4] = -scale * pow(x1, p) * iE1;
            grad[5] = zinf ? 0.0 : scale * pow(x2, p) * iE2;
        }
        return val;
    }
    double chi = dimless_between(&c, INT_CHI, 0, z1, z2, NULL);
    double dchi[6] = {0, 0, 0, 0, -iE1, iE2};
    if (grad)
        for (int a = 1; a <= 3; ++a) dchi[a] = dimless_between(&c, INT_CHI, a, z1, z2, NULL);
    if (kind == K_DC) {
        double val = DH * chi;
        if (grad) {
            grad[0] = -val / c.H0;
            for (int a = 1; a <= 5; ++a) grad[a] = DH * dchi[a];
        }
        return val;
    }
    double S, dS_dchi, dS_dok;
    curvature_transform(c.Ok, chi, &S, &dS_dchi, &dS_dok);
    double DM = DH * S;
    double g[6];
    g[0] = -DM / c.H0;
    for (int a = 1; a <= 3; ++a) g[a] = DH * (dS_dchi * dchi[a] - dS_dok); /* dOk/da = -1 */
    g[4] = DH * dS_dchi * dchi[4];
    g[5] = DH * dS_dchi * dchi[5];
    if (kind == K_DM) {
        if (grad) memcpy(grad, g, sizeof g);
        return DM;
    }
    /* K_DA */
    if (zinf) {
        if (grad) memset(grad, 0, 6 * sizeof(double));
        return 0.0;
    }
    double DA = DM / x2;
    if (grad) {
        for (int a = 0; a < 5; ++a) grad[a] = g[a] / x2;
        grad[5] = g[5] / x2 - DA / x2;
    }
    return DA;
}

/* Batched: out[c*n_z + i] for the pair (z1[c*z_stride + i], z2[c*z_stride + i]);
 * grad (nullable): [n_cosmo][n_z][6].  kind: K_DC, K_DM, K_DA, K_T or K_X.  Returns 0,
 * or -1 on bad arguments. */
int oracle_between(int kind, const double *params, long n_cosmo, const double *z1, const double *z2,
                   long n_z, long z_stride, double *out, double *grad, int nthreads)
{
    if (!(kind == K_DC || kind == K_DM || kind == K_DA || kind == K_T || kind == K_X)) return -1;
    if (n_cosmo < 0 || n_z < 0 || !params || !z1 || !z2 || !out) return -1;
    long total = n_cosmo * n_z;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
#endif
    for (long idx = 0; idx < total; ++idx) {
        long ci = idx / n_z, i = idx % n_z;
        out[idx] = between_one(kind, params + 4 * ci, z1[ci * z_stride + i], z2[ci * z_stride + i],
                               grad ? grad + 6 * idx : NULL);
    }
    (void)nthreads;
    return 0;
}

/* Number of OpenMP threads oracle_eval uses by default. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Carlson symmetric integrals by quadrature of their definitions (eqs. 2.6-2.9).
 *   R_F(x,y,z)   = 1/2 int_0^inf dt / sqrt((t+x)(t+y)(t+z))
 *   R_J(x,y,z,p) = 3/2 int_0^inf dt / ((t+p) sqrt((t+x)(t+y)(t+z)))
 *   R_C(x,y) = R_F(x,y,y),  R_D(x,y,z) = R_J(x,y,z,z)
 * The square root of the product is the product of principal square roots, which
 * is the branch continuous along t in [0, inf) for arguments off the cut.
 * Substitution t = (s/(1-s))^2, s in [0,1), makes the tails integrable on a
 * finite interval (the integrand times dt/ds stays bounded as s -> 1).
 * ------------------------------------------------------------------------- */
struct cctx { double complex x, y, z, p; int third; int imag; };

static double carlson_integrand(double s, const void *vctx)
{
    const struct cctx *k = (const struct cctx *)vctx;
    double r = s / (1.0 - s);
    double t = r * r;
    double dt = 2.0 * s / ((1.0 - s) * (1.0 - s) * (1.0 - s));
    double complex v = 1.0 / (csqrt(t + k->x) * csqrt(t + k->y) * csqrt(t + k->z));
    if (k->third) v = v / (t + k->p);
    v *= dt;
    return k->imag ? cimag(v) : creal(v);
}

static double complex carlson_quad(double complex x, double complex y, double complex z,
                                   double complex p, int third)
{
    struct cctx k = {x, y, z, p, third, 0};
    double re = adapt(carlson_integrand, &k, 0.0, 1.0, 0.0, 1e-13, NULL);
    k.imag = 1;
    double im = adapt(carlson_integrand, &k, 0.0, 1.0, 1e-300, 1e-13, NULL);
    return third ? 1.5 * (re + I * im) : 0.5 * (re + I * im);
}

static int on_cut(double complex v) { return cimag(v) == 0.0 && creal(v) <= 0.0; }

/* which: 0 R_F(x,y,z), 1 R_D(x,y,z), 2 R_J(x,y,z,p), 3 R_C(x,y).
 * args: [n][4][2] interleaved (re, im) of (x, y, z, p); unused slots ignored.
 * out: [n][2].  Arguments on the non-positive real axis give NaN (for R_F, R_D one
 * zero argument is admissible; the quadrature handles it). */
int oracle_carlson(int which, long n, const double *args, double *out)
{
    if (which < 0 || which > 3 || n < 0) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (long i = 0; i < n; ++i) {
        const double *a = args + 8 * i;
        double complex x = a[0] + I * a[1], y = a[2] + I * a[3], z = a[4] + I * a[5],
                       p = a[6] + I * a[7];
        double complex r;
        if (which == 0) r = carlson_quad(x, y, z, 0.0, 0);
        else if (which == 1) r = on_cut(z) ? NAN : carlson_quad(x, y, z, z, 1);
        else if (which == 2) r = on_cut(p) ? NAN : carlson_quad(x, y, z, p, 1);
        else r = on_cut(y) ? NAN : carlson_quad(x, y, y, 0.0, 0);
        out[2 * i] = creal(r);
        out[2 * i + 1] = cimag(r);
    }
    return 0;
}

/* Polynomial exactness probe of the G7K15 rule: integral of t^power over [a,b] by
 * the Kronrod rule (which_rule = 1) or the embedded Gauss rule (which_rule = 0). */
struct pctx { int power; };
static double mono(double t, const void *v) { return pow(t, ((const struct pctx *)v)->power); }

double oracle_gk15_panel(int which_rule, int power, double a, double b)
{
    struct pctx k = {power};
    double err;
    double rk = gk15(mono, &k, a, b, &err);
    if (which_rule == 1) return rk;
    /* recover G7 from K15 and |K15 - G7| is ambiguous in sign: recompute directly */
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double rg = WG[3] * mono(c, &k);
    for (int j = 1; j < 7; j += 2) {
        double dx = h * XGK[j];
        rg += WG[j / 2] * (mono(c - dx, &k) + mono(c + dx, &k));
    }
    return rg * h;
}
