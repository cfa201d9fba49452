/*
 * cosmo.h -- C ABI of libcosmo.so: batched, differentiable LambdaCDM+radiation
 * distances on MI355X (gfx950), after Karchev, "Analytic auto-differentiable
 * LambdaCDM cosmography" (arXiv:2212.01937).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller.  The library keeps
 *    no state between calls and needs no initialisation (its quadrature nodes are
 *    compile-time constants), never frees caller memory and is safe to call from
 *    several host threads.  With a caller-supplied workspace a call only enqueues
 *    kernel launches, so it can be captured in a HIP graph, the first call of a
 *    program included.  The one exception is cosmo_distance_vjp_noalloc, which
 *    works in a fixed device array of the library (see there).
 *  - Calls enqueue asynchronously on `stream` (a hipStream_t passed as void*;
 *    NULL is the default stream) and return a cosmo_status.  Argument errors
 *    (NULL pointers, negative sizes, unknown kind/dtype, workspace too small) are
 *    detected synchronously on the host and nothing is enqueued.  Launch failures
 *    return COSMO_E_HIP.  Per-cosmology domain problems never fail the call: they
 *    write NaN to the affected outputs and set bits in the optional `info` array.
 *  - Cosmological parameters are FP64 rows (H0 [km/s/Mpc], Om0, OL0, Or0); the
 *    curvature follows from the closure Ok0 = 1 - Om0 - OL0 - Or0 (sec. 2.1).
 *    E^2(z) = Or0 (1+z)^4 + Om0 (1+z)^3 + Ok0 (1+z)^2 + OL0 (eq. 2.2).
 *  - Redshifts z (> -1; all outputs are for the interval from 0 to z) and the
 *    outputs use the dtype argument: COSMO_F32 (float) or COSMO_F64 (double).
 *    Rows hold fewer than 2^29 - 2048 redshifts (n_z; the kernels address a row by
 *    32-bit byte offsets): COSMO_E_ARG beyond.
 *    Whatever the dtype, the per-cosmology root finding and the root Jacobian run
 *    in FP64.  Parameter-gradient reductions: each wave sums its lanes' terms (at
 *    most 512: 64 lanes x 8 redshifts) in the dtype; the sums over waves and the
 *    contraction with the root Jacobian are FP64.
 *  - Units: distances in Mpc, time in Gyr, distance modulus in magnitudes
 *    (c = 299792.458 km/s, 1 Mpc = 3.0856775814913673e19 km, 1 Gyr = 3.15576e16 s).
 */
#ifndef COSMO_H
#define COSMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    COSMO_OK = 0,
    COSMO_E_ARG = -1,       /* NULL pointer, negative size, bad stride          */
    COSMO_E_KIND = -2,      /* unknown cosmo_kind                                */
    COSMO_E_DTYPE = -3,     /* unknown cosmo_dtype                               */
    COSMO_E_HIP = -4,       /* a HIP runtime call or kernel launch failed       */
    COSMO_E_WORKSPACE = -5, /* workspace too small (see cosmo_workspace_size)   */
    COSMO_E_SCRATCH = -6    /* problem too large for the fixed device array of
                               cosmo_distance_vjp_noalloc                       */
} cosmo_status;

/* Size in bytes of the fixed device array that cosmo_distance_vjp_noalloc works in
 * (one per GPU, held until the process ends).                                    */
#define COSMO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

typedef enum { COSMO_F32 = 0, COSMO_F64 = 1 } cosmo_dtype;

/* Observables (sec. 2.1.1).  All from z1 = 0 to z2 = z.
 *  DC: comoving distance chi (eq. 2.3), Mpc
 *  DM: transverse comoving distance, curvature-modified chi, Mpc
 *  DL: luminosity distance (1+z) D_M, Mpc
 *  MU: distance modulus 5 log10(D_L / 10 pc) (fn. 22), mag
 *  T : time coordinate / lookback time t(0, z) (eq. 2.4), Gyr
 *  X : absorption distance d_abs (eq. 2.5), Mpc
 *  DA: angular-diameter distance D_M / (1+z), Mpc
 *  VC: all-sky comoving volume 4 pi int_0^z D_M^2 dD_C (sec. 2.1), Mpc^3          */
typedef enum {
    COSMO_DC = 0, COSMO_DM = 1, COSMO_DL = 2, COSMO_MU = 3,
    COSMO_T = 4, COSMO_X = 5, COSMO_DA = 6, COSMO_VC = 7
} cosmo_kind;

/* Bits of the per-cosmology `info` word (int32).                                */
#define COSMO_INFO_CUBIC          0x0001 /* Or0 == 0: radiationless cubic (app. B.1) */
#define COSMO_INFO_QUARTIC        0x0002 /* Or0 > 0: quartic E^2 (eqs. 3.7-3.9)     */
#define COSMO_INFO_THREE_REAL     0x0004 /* cubic factor has three real roots        */
#define COSMO_INFO_YELLOW         0x0008 /* complex pair with Re(r) > 0 (Fig. 1)     */
#define COSMO_INFO_RED            0x0010 /* a real root on the integration path: no Big Bang (Fig. 1, sec. 3) */
#define COSMO_INFO_DOMAIN         0x0020 /* outside the method (degree < 3, no negative real root, ...): NaN */
#define COSMO_INFO_ROOT_NOCONV    0x0040 /* root polishing hit its iteration cap     */
#define COSMO_INFO_NEAR_MULTIROOT 0x0080 /* two roots closer than 1e-4 (relative): gradients by quadrature */
#define COSMO_INFO_X_QUADRATURE   0x0100 /* some X lanes used the Gauss-Legendre route */
#define COSMO_INFO_NEAR_MULTIROOT_F32 0x0200 /* two roots closer than 2e-2 (relative): the FP32
                                                 path's gradients take the quadrature    */

/* Number of bytes of device workspace that cosmo_distance / cosmo_distance_vjp
 * need for this problem size.  A NULL workspace is also accepted by those calls:
 * the library then takes stream-ordered memory from HIP's default pool for the
 * duration of the call (hipMallocAsync / hipFreeAsync on `stream`).              */
int cosmo_workspace_size(int64_t n_cosmo, int64_t n_z, size_t *bytes);

/* cosmo_roots -- factorisation of E^2 (sec. 3, eq. 3.2; fn. 12/13), FP64.
 * params: [n_cosmo][4] FP64 (H0, Om0, OL0, Or0).
 * roots : [n_cosmo][4][2] FP64 out, z-roots r_j as (re, im).  Slots 0..2 are
 *         the roots of the cubic factor (slot 0 real; slots 1, 2 a conjugate pair
 *         with Im >= 0 first, or two further real roots), slot 3 the radiation
 *         root (the real root of largest modulus when Or0 > 0; NaN when Or0 == 0).
 * info  : [n_cosmo] int32 out, nullable.                                        */
int cosmo_roots(const double *params, int64_t n_cosmo, double *roots, int32_t *info,
                void *stream);

/* Carlson symmetric integrals (eqs. 2.6-2.9) for complex arguments, by the
 * duplication method; element-wise over n.  Every operand is interleaved
 * (re, im) of the given dtype, length 2n.  Arguments must avoid the cut of the
 * definitions (non-positive reals; R_F and R_D allow one zero argument); for a
 * negative real p (R_J) or y (R_C) the Cauchy principal value is returned.      */
int carlson_rf(cosmo_dtype dt, int64_t n, const void *x, const void *y, const void *z,
               void *out, void *stream);
int carlson_rd(cosmo_dtype dt, int64_t n, const void *x, const void *y, const void *z,
               void *out, void *stream);
int carlson_rj(cosmo_dtype dt, int64_t n, const void *x, const void *y, const void *z,
               const void *p, void *out, void *stream);
int carlson_rc(cosmo_dtype dt, int64_t n, const void *x, const void *y, void *out,
               void *stream);

/* cosmo_distance -- forward evaluation, sec. 3.1 eqs. 3.7-3.9 (Or0 > 0) and
 * app. B.1 eqs. B.1-B.3 (Or0 == 0), curvature transform and observables.
 * z     : element (c, i) at z[c * z_cosmo_stride + i]; z_cosmo_stride = 0 shares
 *         one row of n_z redshifts between all cosmologies.
 * out   : [n_cosmo][n_z] of dtype, row-major.
 * info  : [n_cosmo] int32, nullable.
 * workspace / workspace_bytes: see cosmo_workspace_size (NULL allowed).          */
int cosmo_distance(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo,
                   const void *z, int64_t n_z, int64_t z_cosmo_stride, void *out,
                   int32_t *info, void *workspace, size_t workspace_bytes, void *stream);

/* cosmo_distance_between -- observables between two redshifts, sec. 2.1 eqs.
 * 2.3-2.4 with both limits free, evaluated as eqs. 3.7-3.8 (app. B.1-B.2 for
 * Or0 == 0), whose Carlson arguments u_ij take both limits:
 *   COSMO_DC  chi(z1, z2)               comoving distance from z1 to z2 [Mpc]
 *   COSMO_DM  (c/H0) sinn(chi(z1, z2))  transverse comoving distance [Mpc]
 *   COSMO_DA  D_M(z1, z2) / (1 + z2)    angular diameter distance of z2 seen
 *                                       from z1 (lensing) [Mpc]
 *   COSMO_T   t(z1, z2)                 time coordinate from z1 to z2 [Gyr]
 * Other kinds return COSMO_E_KIND.  z1[c * z_cosmo_stride + i] and z2[...]: the
 * limits of element (c, i), either order (the result changes sign, D_A aside),
 * laid out like cosmo_distance's z; z2 = +inf gives the limits chi(z1, inf),
 * D_M(z1, inf), D_A = 0 and the age t(z1, inf).  out: [n_cosmo][n_z] of dtype.
 * info, workspace, workspace_bytes, stream: as cosmo_distance.  Adjoint:
 * cosmo_distance_between_vjp (distance kinds).                                      */
int cosmo_distance_between(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo,
                           const void *z1, const void *z2, int64_t n_z, int64_t z_cosmo_stride,
                           void *out, int32_t *info, void *workspace, size_t workspace_bytes,
                           void *stream);

/* cosmo_distance_between_vjp -- adjoint of cosmo_distance_between for COSMO_DC,
 * COSMO_DM, COSMO_DA and COSMO_T (other kinds: COSMO_E_KIND).  The distance kinds through
 * the Carlson derivatives of eq. 3.7 (eq. 2.10) and T through those of eq. 3.8 (R_F,
 * R_J and R_C partials, eqs. 2.10-2.11), with both limits' square roots per element and
 * the root Jacobian (app. A).  Near-multiple-root cosmologies, and for T with z2 = inf
 * a radiation root too small for the chain (|sigma| below 1e-4 FP32 / 1e-9 FP64, or no
 * radiation), take the parameter derivatives by the Leibniz rule (eq. 2.4
 * differentiated under the integral; for T by Gauss-Legendre quadrature in
 * s = (1+z)^(-1/2), finite for z2 = inf).  Limits by the fundamental theorem of
 * calculus.  cot: [n_cosmo][n_z] of dtype.
 * out        : nullable; the observable from the same pass.
 * grad_params: [n_cosmo][4] FP64, sum over elements of cot * d out/d(H0, Om0, OL0,
 *              Or0); nullable.  For the distance kinds NaN for a cosmology with an
 *              infinite upper limit and Or0 = 0 (d chi(z, inf)/d Or0 is -inf there),
 *              and for near-multiple-root cosmologies (whose gradient is the Leibniz
 *              quadrature from z = 0) with z2 = inf.
 * grad_z1, grad_z2: dtype, nullable; [n_z] summed over cosmologies when
 *              z_cosmo_stride == 0, else [n_cosmo][n_z]; d/dz2 is 0 where z2 = inf.
 * workspace  : cosmo_workspace_size(n_cosmo, n_z) bytes (NULL allowed).            */
int cosmo_distance_between_vjp(cosmo_kind kind, cosmo_dtype dt, const double *params,
                               int64_t n_cosmo, const void *z1, const void *z2, int64_t n_z,
                               int64_t z_cosmo_stride, const void *cot, void *out,
                               double *grad_params, void *grad_z1, void *grad_z2, int32_t *info,
                               void *workspace, size_t workspace_bytes, void *stream);

/* cosmo_route_counts -- which route each (cosmology, redshift) lane of `kind` takes,
 * counted per cosmology: the reductions of sec. 3.1 / app. B.1 (eqs. 3.7-3.9,
 * B.1-B.3) against the fallbacks of this implementation.  The routes are decided by
 * the same device functions the forward and adjoint kernels branch on; the values
 * themselves are evaluated (for X) and discarded.
 * counts: [n_cosmo][4] int64 out, overwritten (zero for cosmologies outside the
 *         method): [0] lanes whose value takes the Carlson reduction in the dtype's
 *         precision; [1] FP32 X lanes whose R_F term is refined in FP64 (the terms of
 *         eq. 3.9 cancel by more than 8); [2] lanes whose value takes Gauss-Legendre
 *         quadrature of eq. 2.5 (X only, beyond a cancellation of 1024); [3] lanes whose
 *         adjoint takes the Leibniz-rule quadrature (X; near-multiple roots, see the
 *         NEAR_MULTIROOT info bits; FP32 lanes below z = 0.02).
 * Other arguments as cosmo_distance (the workspace holds the records only).       */
int cosmo_route_counts(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo,
                       const void *z, int64_t n_z, int64_t z_cosmo_stride, int64_t *counts,
                       void *workspace, size_t workspace_bytes, void *stream);

/* cosmo_distance_vjp -- adjoint of cosmo_distance for a cotangent `cot`
 * ([n_cosmo][n_z], dtype).  Gradients through the Carlson derivatives (eqs.
 * 2.10-2.12) and the differentiated root finding (app. A, eqs. A.1-A.4); the
 * z-gradient by the fundamental theorem of calculus.
 * out        : [n_cosmo][n_z] of dtype, nullable.  When given, the observable
 *              itself is written as well (value and gradient from one pass over
 *              the lanes; the values agree with cosmo_distance within the
 *              precision of dt, and the X_QUADRATURE info bit is set as there).
 * grad_params: [n_cosmo][4] FP64 out, sum over z of cot * d out/d(H0, Om0, OL0,
 *              Or0); overwritten; nullable.
 * grad_z     : dtype out, nullable; [n_z] summed over cosmologies when
 *              z_cosmo_stride == 0, else [n_cosmo][n_z]; overwritten.           */
int cosmo_distance_vjp(cosmo_kind kind, cosmo_dtype dt, const double *params,
                       int64_t n_cosmo, const void *z, int64_t n_z, int64_t z_cosmo_stride,
                       const void *cot, void *out, double *grad_params, void *grad_z,
                       int32_t *info, void *workspace, size_t workspace_bytes, void *stream);

/* cosmo_distance_vjp_noalloc -- cosmo_distance_vjp for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that forbid
 * hipMalloc): the same kernels and results (bit for bit), with the per-cosmology
 * records and partial sums in a fixed device array of the library instead of a
 * workspace.  It calls no hipMalloc, hipFree or other allocating routine; the
 * caller passes every input and output as in cosmo_distance_vjp.
 *  - The array holds COSMO_NOALLOC_SCRATCH_BYTES per GPU.  A call needs the record
 *    table (1.2 KB per cosmology); with grad_params, 44 B (FP32) or 88 B (FP64)
 *    per cosmology per 512 redshifts (per 64 redshifts when n_z < 8192); with a
 *    shared-z grad_z and more than one tile of cosmologies (tiles of up to 8),
 *    one dtype element per redshift per tile.  It fits whenever
 *    cosmo_workspace_size(n_cosmo, n_z) <= COSMO_NOALLOC_SCRATCH_BYTES, and often
 *    beyond (1e6 shared redshifts: 64 cosmologies fit in FP32, 32 in FP64).  Larger
 *    problems return COSMO_E_SCRATCH, detected on the host before any HIP call.
 *  - The first call on a GPU resolves the array's device address there
 *    (hipGetSymbolAddress, with that GPU current); make that first call outside a
 *    graph capture if the capture must hold kernel launches only.
 *  - All calls on one GPU share its array: calls that overlap in time on one GPU
 *    (different streams or host threads without ordering) race and give wrong
 *    results.  Calls ordered on one stream are safe: each call writes every byte
 *    of the array it reads before reading it.
 * Arguments and errors otherwise as cosmo_distance_vjp.                         */
int cosmo_distance_vjp_noalloc(cosmo_kind kind, cosmo_dtype dt, const double *params,
                               int64_t n_cosmo, const void *z, int64_t n_z,
                               int64_t z_cosmo_stride, const void *cot, void *out,
                               double *grad_params, void *grad_z, int32_t *info,
                               void *stream);

/* cosmo_distance_jac -- the observable with its materialised per-evaluation
 * Jacobian: the same derivatives as cosmo_distance_vjp (Carlson derivatives,
 * eqs. 2.10-2.12; root Jacobian, app. A; z by the fundamental theorem of
 * calculus), not summed.
 * out : [n_cosmo][n_z] of dtype, nullable (the observable, as cosmo_distance).
 * jac : [5][n_cosmo][n_z] of dtype, five planes d out/d(H0, Om0, OL0, Or0, z);
 *       NaN rows for cosmologies outside the method.
 * info, workspace, workspace_bytes: as cosmo_distance.                          */
int cosmo_distance_jac(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo,
                       const void *z, int64_t n_z, int64_t z_cosmo_stride, void *out, void *jac,
                       int32_t *info, void *workspace, size_t workspace_bytes, void *stream);

/* cosmo_gaussian_loglike -- Gaussian log-likelihood of observed values of the
 * observable (sec. 4: the SN Ia likelihood, mu with Gaussian magnitude errors) and
 * its gradient, from one pass over the lanes:
 *   loglike[c] = -1/2 sum_i ivar_ci (obs_ci - out_ci)^2,
 * the gradient being that of cosmo_distance_vjp with the cotangent formed in each
 * lane, cot_ci = wc[c] ivar_ci (obs_ci - out_ci).
 * obs, ivar : dtype, laid out as z (element (c, i) at [c * z_cosmo_stride + i]: one
 *             row shared by every cosmology when z_cosmo_stride == 0); ivar = 1/sigma^2.
 * wc        : [n_cosmo] FP64 weights of the cosmologies in the gradient, nullable (1).
 * loglike   : [n_cosmo] FP64 out, nullable (unweighted; NaN for cosmologies outside
 *             the method and where out is undefined).
 * grad_params, grad_z, info, workspace, workspace_bytes: as cosmo_distance_vjp.    */
int cosmo_gaussian_loglike(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo,
                           const void *z, int64_t n_z, int64_t z_cosmo_stride, const void *obs,
                           const void *ivar, const double *wc, double *loglike, double *grad_params,
                           void *grad_z, int32_t *info, void *workspace, size_t workspace_bytes,
                           void *stream);

/* ---- the supernova model of sec. 4 (fig. 4b), the distance path as its inner loop ----
 * Latent redshifts of n_sn supernovae under n_draws reparametrised draws of the partial
 * multivariate normal guide (sec. 4): for draw s and supernova n
 *   zeta[s][n] = a[n] + dtheta[s][0] b[n][0] + dtheta[s][1] b[n][1] + exp(log_s[n]) eps[s][n],
 *   z[s][n]    = exp(zeta[s][n]), rounded once to dt.
 * a, log_s, zhat: [n_sn] FP64; b: [n_sn][2] FP64; dtheta: [n_draws][2] FP64 (the draw's
 * offset of (Om0, OL0) from the guide's mean); eps: [n_draws][n_sn] FP64 standard normals
 * drawn by the caller.  All device pointers, caller-owned; asynchronous on `stream`.
 * Errors: COSMO_E_DTYPE; COSMO_E_ARG for negative sizes, n_draws * n_sn beyond
 * 2^32 - 1 blocks of 256, or a NULL array that the sizes require.                    */
int snia_draw(cosmo_dtype dt, int64_t n_draws, int64_t n_sn, const double *a, const double *b,
              const double *log_s, const double *dtheta, const double *eps, void *z, void *stream);

/* snia_latent_vjp -- the per-supernova terms of the model's log joint density (sec. 4)
 * and their adjoint, summed over draws and supernovae:
 *   F = sum_{s,n} [ -1/2 ((zhat - z)/((1 + z) sigma_z))^2 - log((1 + z) sigma_z)
 *                   + (gamma_shape - 1) log z - gamma_rate z + zeta + eps^2 / 2 ]
 * (photometric redshift likelihood, Gamma redshift prior up to its constant, the
 * Jacobian of z = exp(zeta) and the eps^2/2 of the guide density), with z recomputed
 * as snia_draw does.  grad_z ([n_draws][n_sn] of dt, nullable) is an extra derivative
 * d G/dz of terms computed elsewhere (the distance likelihood of cosmo_gaussian_loglike);
 * the adjoint is that of F + G:
 *   value_dtheta[0]          = F (FP64),
 *   value_dtheta[1 + 2s + j] = d(F + G)/d dtheta[s][j],
 *   grad_a[n], grad_b[n][j], grad_log_s[n] = d(F + G)/d a[n], b[n][j], log_s[n]   (FP64).
 * value_dtheta: [1 + 2 n_draws]; overwritten (zeros for empty sizes).
 * workspace: snia_workspace_size(n_draws, n_sn) bytes, or NULL (allocated on stream).
 * Errors: as snia_draw; COSMO_E_ARG also unless sigma_z, gamma_shape and gamma_rate
 * are finite and positive; COSMO_E_WORKSPACE for a workspace below the size.          */
int snia_latent_vjp(cosmo_dtype dt, int64_t n_draws, int64_t n_sn, const double *a, const double *b,
                    const double *log_s, const double *dtheta, const double *eps, const double *zhat,
                    const void *grad_z, double sigma_z, double gamma_shape, double gamma_rate,
                    double *value_dtheta, double *grad_a, double *grad_b, double *grad_log_s,
                    void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes of snia_latent_vjp.  COSMO_E_ARG for invalid sizes or NULL bytes. */
int snia_workspace_size(int64_t n_draws, int64_t n_sn, size_t *bytes);

/* Library version string (static storage). */
const char *cosmo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COSMO_H */
