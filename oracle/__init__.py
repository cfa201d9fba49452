"""CPU oracle for the distance integrals -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library: distances come from
adaptive Gauss-Kronrod quadrature of the defining integrals (eqs. 2.3-2.5 of
arXiv:2212.01937), the Carlson integrals from quadrature of their definitions
(eqs. 2.6-2.9), and polynomial roots from mpmath's arbitrary-precision
polynomial solver (the factorisation of eq. 3.2).

Every function below is a thin ctypes/numpy wrapper; the arithmetic lives in
oracle.c (and, for the roots, in mpmath).
"""
import ctypes
import os

import numpy as np

from . import build as _build

KINDS = {"DC": 0, "DM": 1, "DL": 2, "MU": 3, "T": 4, "X": 5, "DA": 6, "VC": 7}
CARLSON = {"RF": 0, "RD": 1, "RJ": 2, "RC": 3}

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_eval.argtypes = [ctypes.c_int, dp, ctypes.c_long, dp, ctypes.c_long,
                                    ctypes.c_long, dp, dp, dp, ctypes.c_int]
        lib.oracle_eval.restype = ctypes.c_int
        lib.oracle_carlson.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp]
        lib.oracle_carlson.restype = ctypes.c_int
        lib.oracle_gk15_panel.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double]
        lib.oracle_gk15_panel.restype = ctypes.c_double
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_between.argtypes = [ctypes.c_int, dp, ctypes.c_long, dp, dp, ctypes.c_long, ctypes.c_long,
                                       dp, dp, ctypes.c_int]
        lib.oracle_between.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def distance(kind, params, z, shared_z=None, grad=False, errest=False, nthreads=0):
    """Evaluate observable `kind` ('DC','DM','DL','MU','T','X','DA').

    params: (n_cosmo, 4) array of (H0, Om0, OL0, Or0).
    z: (n_z,) shared by all cosmologies, or (n_cosmo, n_z) per cosmology.
    Returns out (n_cosmo, n_z) and, if requested, grad (n_cosmo, n_z, 5) with
    d/d(H0, Om0, OL0, Or0, z), and errest (n_cosmo, n_z) (quadrature estimate).
    """
    lib = _load()
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, 4))
    zz = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    n_c = p.shape[0]
    if shared_z is None:
        shared_z = zz.ndim == 1
    if shared_z:
        n_z, stride = zz.shape[-1], 0
    else:
        zz = np.ascontiguousarray(zz.reshape(n_c, -1))
        n_z, stride = zz.shape[1], zz.shape[1]
    out = np.empty((n_c, n_z))
    g = np.empty((n_c, n_z, 5)) if grad else None
    e = np.empty((n_c, n_z)) if errest else None
    rc = lib.oracle_eval(KINDS[kind], _ptr(p), n_c, _ptr(zz), n_z, stride, _ptr(out), _ptr(g),
                         _ptr(e), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_eval rejected its arguments")
    res = [out]
    if grad:
        res.append(g)
    if errest:
        res.append(e)
    return res[0] if len(res) == 1 else tuple(res)


def between(kind, params, z1, z2, grad=False, nthreads=0):
    """Observable `kind` ('DC', 'DM', 'DA', 'T', 'X') between redshifts z1 and z2:
    the integrals of eqs. 2.3-2.5 from z1 to z2 (either order; z2 = inf allowed for
    'DC', 'DM', 'DA' and 'T', the latter being the age t(z1, inf)).  D_M(z1, z2) is
    the curvature transform of chi(z1, z2) and D_A(z1, z2) = D_M(z1, z2)/(1 + z2).

    params: (n_cosmo, 4); z1, z2: broadcastable to (n_z,) (shared by all cosmologies)
    or (n_cosmo, n_z).  Returns out (n_cosmo, n_z) and, with grad, the derivatives
    (n_cosmo, n_z, 6) with respect to (H0, Om0, OL0, Or0, z1, z2)."""
    lib = _load()
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, 4))
    n_c = p.shape[0]
    a, b = np.broadcast_arrays(np.asarray(z1, dtype=np.float64), np.asarray(z2, dtype=np.float64))
    shared = a.ndim == 1
    if shared:
        n_z, stride = a.shape[0], 0
    else:
        a = a.reshape(n_c, -1)
        b = b.reshape(n_c, -1)
        n_z, stride = a.shape[1], a.shape[1]
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    out = np.empty((n_c, n_z))
    g = np.empty((n_c, n_z, 6)) if grad else None
    rc = lib.oracle_between(KINDS[kind], _ptr(p), n_c, _ptr(a), _ptr(b), n_z, stride, _ptr(out), _ptr(g),
                            int(nthreads))
    if rc != 0:
        raise ValueError("oracle_between rejected its arguments")
    return (out, g) if grad else out


def snia_log_joint(theta, z, zhat, muhat, h0=70.0, sigma_mu=0.14, sigma_z=0.04, beta=3.0, shape=3.0,
                   grad=False):
    """Log joint density of the supernova model of sec. 4, per sample, up to the
    constants of the two Gaussian likelihoods (written term by term):
        sum_s  -1/2 ((muhat_s - mu(z_s; theta)) / sigma_mu)^2
             + [-1/2 ((zhat_s - z_s) / ((1 + z_s) sigma_z))^2 - log((1 + z_s) sigma_z)]
             + [(shape - 1) log z_s - beta z_s + shape log beta - lgamma(shape)]
    with theta = (Om0, OL0), Or0 = 0, H0 fixed; mu from this oracle's quadrature.
    theta (S, 2), z (S, N), zhat and muhat (N,).  Returns lp (S,) and, with grad,
    (dlp/dtheta (S, 2), dlp/dz (S, N))."""
    import math
    th = np.asarray(theta, dtype=np.float64).reshape(-1, 2)
    zz = np.asarray(z, dtype=np.float64).reshape(th.shape[0], -1)
    zh = np.asarray(zhat, dtype=np.float64)
    mh = np.asarray(muhat, dtype=np.float64)
    S, N = zz.shape
    params = np.column_stack([np.full(S, h0), th[:, 0], th[:, 1], np.zeros(S)])
    if grad:
        mu, g = distance("MU", params, zz, shared_z=False, grad=True)
    else:
        mu = distance("MU", params, zz, shared_z=False)
    r = (mh - mu) / sigma_mu
    sd = (1.0 + zz) * sigma_z
    q = (zh - zz) / sd
    lp = (-0.5 * r ** 2 - 0.5 * q ** 2 - np.log(sd) + (shape - 1.0) * np.log(zz) - beta * zz).sum(1)
    lp += N * (shape * math.log(beta) - math.lgamma(shape))
    if not grad:
        return lp
    w = r / sigma_mu  # d(-1/2 r^2)/dmu
    dth = np.stack([(w * g[:, :, 1]).sum(1), (w * g[:, :, 2]).sum(1)], axis=1)
    # d/dz of the photometric term: q^2 / (1 + z) + q / sd - 1 / (1 + z)
    dz = w * g[:, :, 4] + q / sd + q ** 2 / (1.0 + zz) - 1.0 / (1.0 + zz) + (shape - 1.0) / zz - beta
    return lp, dth, dz




def carlson(which, x, y, z=None, p=None):
    """R_F(x,y,z), R_D(x,y,z), R_J(x,y,z,p) or R_C(x,y) by quadrature (complex)."""
    lib = _load()
    x = np.atleast_1d(np.asarray(x, dtype=np.complex128))
    n = x.shape[0]
    args = np.zeros((n, 4), dtype=np.complex128)
    args[:, 0] = x
    args[:, 1] = np.broadcast_to(np.asarray(y, dtype=np.complex128), (n,))
    if z is not None:
        args[:, 2] = np.broadcast_to(np.asarray(z, dtype=np.complex128), (n,))
    if p is not None:
        args[:, 3] = np.broadcast_to(np.asarray(p, dtype=np.complex128), (n,))
    a = np.ascontiguousarray(args).view(np.float64)
    out = np.empty(2 * n)
    rc = lib.oracle_carlson(CARLSON[which], n, _ptr(a), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_carlson rejected its arguments")
    return out.view(np.complex128)


def threads():
    """OpenMP threads the oracle uses by default."""
    return int(_load().oracle_threads())


def gk15_panel(rule, power, a, b):
    """Integral of t**power on [a,b] by one Kronrod (rule=1) or Gauss (rule=0) panel."""
    return _load().oracle_gk15_panel(int(rule), int(power), float(a), float(b))


def roots(params, dps=50):
    """Roots r_j of E^2(z) (eq. 3.2), by mpmath's polynomial solver at `dps` digits.

    params: (n, 4) of (H0, Om0, OL0, Or0).  Returns (n, 4) complex128 z-roots; for a
    radiationless cosmology (Or0 == 0) the cubic's three roots and a NaN slot.
    The polynomial is taken in x = 1 + z, P(x) = Or x^4 + Om x^3 + Ok x^2 + OL, and
    1 is subtracted from its roots.
    """
    import mpmath
    p = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    out = np.full((p.shape[0], 4), np.nan + 0j)
    with mpmath.workdps(dps):
        for i, (_, om, ol, orr) in enumerate(p):
            ok = mpmath.mpf(1) - mpmath.mpf(om) - mpmath.mpf(ol) - mpmath.mpf(orr)
            coeffs = [mpmath.mpf(orr), mpmath.mpf(om), ok, mpmath.mpf(0), mpmath.mpf(ol)]
            while coeffs and coeffs[0] == 0:
                coeffs.pop(0)
            rts = mpmath.polyroots(coeffs, maxsteps=400, extraprec=4 * dps)
            for j, r in enumerate(rts):
                out[i, j] = complex(r) - 1.0
    return out
