"""Pins of the CPU oracle to things other than itself.

Each test checks the oracle against closed forms, independent libraries
(mpmath tanh-sinh quadrature at 30 digits, scipy's QUADPACK wrapper, scipy's and
mpmath's Carlson routines), mathematical identities, or finite differences, so
that a dropped term, a wrong sign or a swapped operand in oracle.c fails here.
"""
import math

import numpy as np
import pytest

import oracle

C = 299792.458
TH_FACTOR = 3.0856775814913673e19 / 3.15576e16  # (1/H0) in Gyr times H0


def DH(h0):
    return C / h0


def TH(h0):
    return TH_FACTOR / h0


def rel(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


ZS = np.array([1e-5, 1e-3, 0.1, 0.5, 1.0, 2.0, 10.0, 100.0, 1000.0])


# --------------------------------------------------------------------------- rule
def test_gk15_polynomial_exactness():
    """The 15-point Kronrod rule is exact to degree 23 (3n+1 = 22, plus one from the
    rule's symmetry), the embedded 7-point Gauss rule to degree 13 (this pins every
    node and weight constant)."""
    a, b = -0.3, 1.7
    for k in range(0, 24):
        exact = (b ** (k + 1) - a ** (k + 1)) / (k + 1)
        assert abs(oracle.gk15_panel(1, k, a, b) - exact) <= 2e-15 * max(1.0, abs(exact)), k
    for k in range(0, 14):
        exact = (b ** (k + 1) - a ** (k + 1)) / (k + 1)
        assert abs(oracle.gk15_panel(0, k, a, b) - exact) <= 2e-15 * max(1.0, abs(exact)), k
    # and neither is exact one degree higher (the rules really are of that order)
    for rule, k in ((1, 24), (0, 14)):
        exact = (b ** (k + 1) - a ** (k + 1)) / (k + 1)
        assert abs(oracle.gk15_panel(rule, k, a, b) - exact) > 1e-14 * abs(exact)


# --------------------------------------------------------------------------- closed forms
def _ev(kind, params, z):
    return oracle.distance(kind, np.array([params], dtype=float), np.asarray(z, dtype=float))[0]


def test_einstein_de_sitter():
    """Om0 = 1: E = (1+z)^(3/2)."""
    h0 = 70.0
    p = (h0, 1.0, 0.0, 0.0)
    x = 1.0 + ZS
    lx = np.log1p(ZS)  # closed forms written without cancellation at small z
    assert rel(_ev("DC", p, ZS), -2 * DH(h0) * np.expm1(-0.5 * lx)) < 1e-13
    assert rel(_ev("T", p, ZS), -(2.0 / 3.0) * TH(h0) * np.expm1(-1.5 * lx)) < 1e-13
    assert rel(_ev("X", p, ZS), (2.0 / 3.0) * DH(h0) * np.expm1(1.5 * lx)) < 1e-13


def test_milne_empty_universe():
    """All densities zero, Ok0 = 1: E = 1+z; D_M = D_H sinh(ln(1+z))."""
    h0 = 65.0
    p = (h0, 0.0, 0.0, 0.0)
    x = 1.0 + ZS
    assert rel(_ev("DC", p, ZS), DH(h0) * np.log1p(ZS)) < 1e-13
    assert rel(_ev("T", p, ZS), TH(h0) * ZS / x) < 1e-13
    assert rel(_ev("X", p, ZS), DH(h0) * (ZS + ZS ** 2 / 2)) < 1e-13
    dm = DH(h0) * ZS * (2 + ZS) / (2 * x)
    assert rel(_ev("DM", p, ZS), dm) < 1e-13
    assert rel(_ev("DL", p, ZS), dm * x) < 1e-13
    assert rel(_ev("DA", p, ZS), dm / x) < 1e-13


def test_de_sitter():
    """OL0 = 1: E = 1."""
    h0 = 72.0
    p = (h0, 0.0, 1.0, 0.0)
    x = 1.0 + ZS
    assert rel(_ev("DC", p, ZS), DH(h0) * ZS) < 1e-13
    assert rel(_ev("T", p, ZS), TH(h0) * np.log1p(ZS)) < 1e-13
    assert rel(_ev("X", p, ZS), DH(h0) * np.expm1(3 * np.log1p(ZS)) / 3) < 1e-13
    assert rel(_ev("DM", p, ZS), DH(h0) * ZS) < 1e-13


def test_radiation_only():
    """Or0 = 1: E = (1+z)^2."""
    h0 = 70.0
    p = (h0, 0.0, 0.0, 1.0)
    x = 1.0 + ZS
    assert rel(_ev("DC", p, ZS), DH(h0) * ZS / x) < 1e-13
    assert rel(_ev("T", p, ZS), -TH(h0) * 0.5 * np.expm1(-2 * np.log1p(ZS))) < 1e-13
    assert rel(_ev("X", p, ZS), DH(h0) * ZS) < 1e-13


@pytest.mark.parametrize("om", [0.3, 0.05, 1.7, 3.0])
def test_matter_plus_curvature_mattig(om):
    """OL0 = Or0 = 0, Ok0 = 1 - Om0 of either sign.  D_C by substitution
    w = sqrt(Om x + Ok); D_M by Mattig's relation; X by the same substitution."""
    h0 = 68.0
    p = (h0, om, 0.0, 0.0)
    ok = 1.0 - om
    z = ZS[ZS <= 100.0]
    x = 1.0 + z
    # w = sqrt(Om x + Ok) runs from 1 to w2; w2 - 1 = Om z / (1 + w2) avoids cancellation
    w2 = np.sqrt(1 + om * z)
    dw = om * z / (1 + w2)
    if ok > 0:
        a = math.sqrt(ok)
        dc = np.log1p(2 * a * dw / ((w2 + a) * (1 - a))) / a
    else:
        a = math.sqrt(-ok)
        dc = 2.0 * np.arctan(dw * a / (a * a + w2)) / a
    assert rel(_ev("DC", p, z), DH(h0) * dc) < 1e-13
    # Mattig: D_M = 2 D_H [2 - Om(1-z) - (2-Om) w2] / (Om^2 (1+z)), rationalised
    dm = DH(h0) * 2 * z * (1 + z / (1 + w2)) / ((1 + w2) * x)
    assert rel(_ev("DM", p, z), dm) < 5e-13
    assert rel(_ev("DL", p, z), dm * x) < 5e-13
    assert rel(_ev("DA", p, z), dm / x) < 5e-13
    mu = 5 * np.log10(dm * x) + 25
    assert np.max(np.abs(_ev("MU", p, z) - mu)) < 1e-12
    # X = D_H (2/Om^2) [w^3/3 - Ok w] from w = 1 to w2
    xx = DH(h0) * (2.0 / om ** 2) * dw * ((w2 * w2 + w2 + 1) / 3 - ok)
    assert rel(_ev("X", p, z), xx) < 1e-13


def test_flat_matter_plus_radiation():
    """OL0 = 0, Or0 + Om0 = 1: D_C = (2 D_H / Om)(1 - sqrt(Or x + Om)/sqrt(x))."""
    h0 = 70.0
    om, orr = 0.7, 0.3
    p = (h0, om, 0.0, orr)
    x = 1.0 + ZS
    dc = 2 * DH(h0) * ZS / (x * (1 + np.sqrt(orr + om / x)))  # = (2 D_H/Om)(1 - sqrt(Or + Om/x))
    assert rel(_ev("DC", p, ZS), dc) < 1e-13


@pytest.mark.parametrize("ol", [0.6, 1.4])
def test_lambda_plus_curvature(ol):
    """Om0 = Or0 = 0, Ok0 = 1 - OL0: D_C = asinh / asin closed forms."""
    h0 = 70.0
    p = (h0, 0.0, ol, 0.0)
    ok = 1.0 - ol
    z = np.array([1e-4, 0.01, 0.1, 0.15]) if ok < 0 else ZS
    x = 1.0 + z
    # differences of asinh / asin folded into one call (no cancellation at small z)
    if ok > 0:
        a = math.sqrt(ok / ol)
        u, v = a * x, a
        d = a * a * z * (2 + z) / (u * math.sqrt(1 + v * v) + v * np.sqrt(1 + u * u))
        dc = np.arcsinh(d) / math.sqrt(ok)
    else:
        a = math.sqrt(-ok / ol)
        u, v = a * x, a
        d = a * a * z * (2 + z) / (u * math.sqrt(1 - v * v) + v * np.sqrt(1 - u * u))
        dc = np.arcsin(d) / math.sqrt(-ok)
    assert rel(_ev("DC", p, z), DH(h0) * dc) < 1e-13


def test_small_z_taylor():
    """D_C = D_H [z - (1+q0) z^2/2 + O(z^3)], q0 = Or0 + Om0/2 - OL0."""
    h0, om, ol, orr = 70.0, 0.3, 0.6, 1e-4
    q0 = orr + om / 2 - ol
    for z in (1e-3, 1e-4):
        v = _ev("DC", (h0, om, ol, orr), [z])[0] / DH(h0)
        approx = z - (1 + q0) * z * z / 2
        assert abs(v - approx) < 2.0 * z ** 3


def test_unphysical_path_gives_nan():
    """A cosmology without a big bang (E^2 < 0 at some finite z) gives NaN once the
    integration path reaches that redshift (sec. 3, physical-domain condition)."""
    p = (70.0, 0.05, 1.3, 0.0)
    v = _ev("DC", p, [0.1, 5.0])
    assert np.isfinite(v[0]) and np.isnan(v[1])


# --------------------------------------------------------------------------- independent quadratures
def _E_np(p, z):
    h0, om, ol, orr = p
    ok = 1 - om - ol - orr
    x = 1.0 + z
    return np.sqrt(orr * x ** 4 + om * x ** 3 + ok * x ** 2 + ol)


COSMOS = [
    (70.0, 0.3, 0.7 - 9e-5, 9e-5),
    (67.0, 0.3, 0.6, 1e-5),
    (74.0, 0.3, 0.8, 1e-4),
    (62.0, 0.25, 1.05, 5e-5),
    (70.0, 0.6, 0.1, 9e-5),
    (79.0, 0.05, 0.9, 1e-4),
    (70.0, 0.3, 0.7, 0.0),
]


def test_against_mpmath_quad_30_digits():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    for p in COSMOS[:4] + COSMOS[6:]:
        h0, om, ol, orr = (mpmath.mpf(v) for v in p)
        ok = 1 - om - ol - orr

        def E(zz):
            x = 1 + zz
            return mpmath.sqrt(orr * x ** 4 + om * x ** 3 + ok * x ** 2 + ol)

        for z in (0.5, 3.0, 1000.0):
            pts = [0] + [b for b in (1, 10, 100) if b < z] + [z]
            dc = mpmath.quad(lambda t: 1 / E(t), pts) * C / h0
            tt = mpmath.quad(lambda t: 1 / ((1 + t) * E(t)), pts) * mpmath.mpf(TH_FACTOR) / h0
            xx = mpmath.quad(lambda t: (1 + t) ** 2 / E(t), pts) * C / h0
            assert rel(_ev("DC", p, [z]), [float(dc)]) < 2e-14
            assert rel(_ev("T", p, [z]), [float(tt)]) < 2e-14
            assert rel(_ev("X", p, [z]), [float(xx)]) < 2e-14


def test_against_scipy_quad():
    """The paper's own baseline (QUADPACK via scipy), on a seeded sample."""
    from scipy.integrate import quad
    rng = np.random.default_rng(11)
    for _ in range(25):
        p = (rng.uniform(60, 80), rng.uniform(0.05, 0.6), rng.uniform(0, 1.0),
             rng.uniform(0, 1e-4))
        z = float(10 ** rng.uniform(-3, 1))
        ref = quad(lambda t: 1 / _E_np(p, t), 0, z, epsabs=0, epsrel=1e-13, limit=200)[0]
        assert rel(_ev("DC", p, [z]), [ref * DH(p[0])]) < 1e-12
        ref = quad(lambda t: 1 / ((1 + t) * _E_np(p, t)), 0, z, epsabs=0, epsrel=1e-13,
                   limit=200)[0]
        assert rel(_ev("T", p, [z]), [ref * TH(p[0])]) < 1e-12


# --------------------------------------------------------------------------- gradients
def _richardson(f, x0, h):
    d1 = (f(x0 + h) - f(x0 - h)) / (2 * h)
    d2 = (f(x0 + h / 2) - f(x0 - h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("kind", ["DC", "DM", "DL", "MU", "T", "X", "DA", "VC"])
def test_gradient_vs_richardson_differences(kind):
    """Leibniz-rule gradients vs central differences of the oracle's own values,
    for open and closed curvature."""
    for p in [(70.0, 0.3, 0.6, 1e-4), (66.0, 0.45, 0.85, 3e-5), (72.0, 0.2, 0.3, 0.0)]:
        z = 1.7
        _, g = oracle.distance(kind, np.array([p]), np.array([z]), grad=True)
        g = g[0, 0]
        for a, h in zip(range(5), (1e-2, 1e-4, 1e-4, 1e-6, 1e-4)):
            def f(v, a=a):
                q = list(p) + [z]
                q[a] = v
                return _ev(kind, tuple(q[:4]), [q[4]])[0]
            x0 = (list(p) + [z])[a]
            fd = _richardson(f, x0, h)
            scale = max(abs(fd), 1e-6 * abs(_ev(kind, p, [z])[0]) / max(abs(x0), 1e-4), 1e-12)
            if a == 3:  # Or0 enters through tiny differences; looser
                assert abs(g[a] - fd) <= 1e-5 * scale + 1e-6 * abs(g[a]), (kind, p, a, g[a], fd)
            else:
                assert abs(g[a] - fd) <= 1e-7 * scale, (kind, p, a, g[a], fd)


def test_gradient_closed_form_mattig():
    """d D_M/d Om0 along OL0 = Or0 = 0 (Ok0 = 1 - Om0 follows by closure) equals the
    derivative of Mattig's closed form; dD_M/dz likewise."""
    h0, om, z = 70.0, 0.4, 1.3
    _, g = oracle.distance("DM", np.array([[h0, om, 0.0, 0.0]]), np.array([z]), grad=True)

    def mattig(o, zz):
        return DH(h0) * 2 * (2 - o * (1 - zz) - (2 - o) * math.sqrt(1 + o * zz)) / (o ** 2 * (1 + zz))

    d_om = _richardson(lambda o: mattig(o, z), om, 1e-3)
    d_z = _richardson(lambda zz: mattig(om, zz), z, 1e-3)
    assert abs(g[0, 0, 1] - d_om) < 1e-9 * abs(d_om)
    assert abs(g[0, 0, 4] - d_z) < 1e-9 * abs(d_z)
    assert abs(g[0, 0, 0] + mattig(om, z) / h0) < 1e-12 * mattig(om, z) / h0


def test_fundamental_theorem_z_gradient():
    p = (70.0, 0.3, 0.7 - 9e-5, 9e-5)
    z = np.array([0.01, 0.5, 2.0, 30.0])
    _, g = oracle.distance("DC", np.array([p]), z, grad=True)
    assert rel(g[0, :, 4], DH(70.0) / _E_np(p, z)) < 1e-14
    _, g = oracle.distance("T", np.array([p]), z, grad=True)
    assert rel(g[0, :, 4], TH(70.0) / ((1 + z) * _E_np(p, z))) < 1e-14
    _, g = oracle.distance("X", np.array([p]), z, grad=True)
    assert rel(g[0, :, 4], DH(70.0) * (1 + z) ** 2 / _E_np(p, z)) < 1e-14


def test_fiducial_mu_gradients_against_mpmath():
    """mu-gradients at the radiationless fiducial (0.3, 0.7, H0=70), z=1, against
    mpmath's numerical differentiation of a 30-digit tanh-sinh quadrature."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30

    def mu(h0, om, ol, z):
        ok = 1 - om - ol
        E = lambda t: mpmath.sqrt(om * (1 + t) ** 3 + ok * (1 + t) ** 2 + ol)
        chi = mpmath.quad(lambda t: 1 / E(t), [0, z])
        s = mpmath.sqrt(abs(ok)) if ok != 0 else None
        if ok > 0:
            dm = mpmath.sinh(s * chi) / s
        elif ok < 0:
            dm = mpmath.sin(s * chi) / s
        else:
            dm = chi
        return 5 * mpmath.log10((1 + z) * dm * C / h0) + 25

    h0, om, ol, z = mpmath.mpf(70), mpmath.mpf("0.3"), mpmath.mpf("0.7"), mpmath.mpf(1)
    ref = [mpmath.diff(lambda v: mu(v, om, ol, z), h0),
           mpmath.diff(lambda v: mu(h0, v, ol, z), om),
           mpmath.diff(lambda v: mu(h0, om, v, z), ol),
           mpmath.diff(lambda v: mu(h0, om, ol, v), z)]
    _, g = oracle.distance("MU", np.array([[70.0, 0.3, 0.7, 0.0]]), np.array([1.0]), grad=True)
    got = [g[0, 0, 0], g[0, 0, 1], g[0, 0, 2], g[0, 0, 4]]
    for a, b in zip(got, ref):
        assert abs(a - float(b)) < 1e-11 * abs(float(b))


# --------------------------------------------------------------------------- Carlson
def _rand_c(rng, n, conj_pair=False):
    x = rng.uniform(0.1, 3, n) + 0j
    y = rng.uniform(-2, 3, n) + 1j * rng.uniform(0.05, 2, n)
    z = np.conj(y) if conj_pair else rng.uniform(-2, 3, n) + 1j * rng.uniform(-2, -0.05, n)
    return x, y, z


def test_carlson_invariants():
    rng = np.random.default_rng(3)
    for v in [0.37 + 0j, 2.5 + 0j, 1.2 + 0.7j, 0.3 - 1.1j]:
        assert abs(oracle.carlson("RF", v, v, v)[0] - v ** -0.5) < 1e-13 * abs(v ** -0.5)
        assert abs(oracle.carlson("RD", v, v, v)[0] - v ** -1.5) < 1e-13 * abs(v ** -1.5)
        assert abs(oracle.carlson("RJ", v, v, v, v)[0] - v ** -1.5) < 1e-13 * abs(v ** -1.5)
    x, y, z = _rand_c(rng, 6, conj_pair=True)
    rf = oracle.carlson("RF", x, y, z)
    assert np.max(np.abs(rf.imag)) < 1e-13 * np.max(np.abs(rf))  # conjugate pair -> real
    lam = 3.7
    assert np.max(np.abs(oracle.carlson("RF", lam * x, lam * y, lam * z) - rf * lam ** -0.5)) < 1e-13
    rd = oracle.carlson("RD", x, y, z)
    assert np.max(np.abs(oracle.carlson("RD", lam * x, lam * y, lam * z) - rd * lam ** -1.5)) < 1e-13
    # sum over cyclic permutations: R_D(x,y,z)+R_D(y,z,x)+R_D(z,x,y) = 3/sqrt(xyz)
    s = rd + oracle.carlson("RD", y, z, x) + oracle.carlson("RD", z, x, y)
    assert np.max(np.abs(s - 3 / (np.sqrt(x) * np.sqrt(y) * np.sqrt(z)))) < 1e-12
    # sum_i x_i R_D(., ., x_i) = 3 R_F
    s = z * rd + x * oracle.carlson("RD", y, z, x) + y * oracle.carlson("RD", z, x, y)
    assert np.max(np.abs(s - 3 * rf)) < 1e-12
    # R_C(x, y) = R_F(x, y, y), and closed forms for real arguments
    for a, b in [(0.3, 1.7), (2.0, 0.5)]:
        rc = oracle.carlson("RC", a, b)[0].real
        assert abs(rc - oracle.carlson("RF", a, b, b)[0].real) < 1e-14
        ref = (math.acos(math.sqrt(a / b)) / math.sqrt(b - a) if a < b
               else math.acosh(math.sqrt(a / b)) / math.sqrt(a - b))
        assert abs(rc - ref) < 1e-14 * ref


def test_carlson_complete_legendre():
    """R_F(0, 1-m, 1) = K(m) (complete first kind, textbook)."""
    from scipy.special import ellipk
    for m in (0.1, 0.5, 0.9, 0.999):
        assert abs(oracle.carlson("RF", 0.0, 1 - m, 1.0)[0].real - ellipk(m)) < 1e-13 * ellipk(m)


def test_carlson_against_scipy():
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(5)
    for pair in (True, False):
        x, y, z = _rand_c(rng, 20, conj_pair=pair)
        p = rng.uniform(0.2, 3, 20) + 1j * rng.uniform(-1, 1, 20)
        assert np.max(np.abs(oracle.carlson("RF", x, y, z) - sp.elliprf(x, y, z))
                      / np.abs(sp.elliprf(x, y, z))) < 1e-13
        assert np.max(np.abs(oracle.carlson("RD", x, y, z) - sp.elliprd(x, y, z))
                      / np.abs(sp.elliprd(x, y, z))) < 1e-13
        # scipy declines R_J outside the region where Carlson's algorithm is
        # guaranteed (the paper's fn. 9); mpmath covers it
        import mpmath
        ref = np.array([complex(mpmath.elliprj(*a)) for a in zip(x, y, z, p)])
        assert np.max(np.abs(oracle.carlson("RJ", x, y, z, p) - ref) / np.abs(ref)) < 1e-12
        assert np.max(np.abs(oracle.carlson("RC", x, y) - sp.elliprc(x, y))
                      / np.abs(sp.elliprc(x, y))) < 1e-13


# --------------------------------------------------------------------------- roots
def test_roots_vieta_reconstruction():
    """Oracle roots reproduce the coefficients of E^2 in x = 1 + z (eq. 3.2 / A.1)."""
    P = np.array(COSMOS + [(70.0, 0.3, 0.0, 1e-5), (70.0, 1.0, 1e-9, 1e-8)])
    r = oracle.roots(P)
    for (h0, om, ol, orr), rr in zip(P, r):
        ok = 1 - om - ol - orr
        if orr > 0:
            lead, rho = orr, rr + 1
            want = np.array([orr, om, ok, 0.0, ol])
        else:
            lead, rho = om, rr[:3] + 1
            want = np.array([om, ok, 0.0, ol])
        got = lead * np.poly(rho)
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def test_roots_known_factorisation():
    """Cosmology built from prescribed x-roots (a near-double pair rho, rho(1+d)):
    with Or0 = 0, P(x) = Om (x - rho)(x - rho(1+d))(x - c) and no linear term."""
    rho, d = 0.4, 1e-6
    r1, r2 = rho, rho * (1 + d)
    c = -r1 * r2 / (r1 + r2)  # makes the linear coefficient vanish
    poly = np.poly([r1, r2, c])  # monic cubic
    om = 1.0 / np.polyval(poly, 1.0)  # P(1) = 1
    ok, ol = om * poly[1], om * poly[3]
    assert abs(om * poly[2]) < 1e-15
    r = oracle.roots(np.array([[70.0, om, ol, 0.0]]))[0, :3] + 1
    got = np.sort_complex(r)
    want = np.sort_complex(np.array([c, r1, r2], dtype=complex))
    # rounding the coefficients to FP64 moves a root pair d apart by ~ eps*rho/d
    assert np.max(np.abs(got - want)) < 100 * 2.2e-16 * rho / d
    assert abs(got[0] - want[0]) < 1e-14


# --------------------------------------------------------------------------- between two redshifts
Z1 = np.array([0.0, 1e-4, 0.1, 0.5, 1.0, 3.0, 50.0])
Z2 = np.array([0.3, 2e-4, 0.1, 2.0, 0.2, 1000.0, 50.5])  # includes z1 == z2 and z1 > z2


def _bt(kind, params, z1, z2):
    return oracle.between(kind, np.array([params], dtype=float), np.asarray(z1, dtype=float),
                          np.asarray(z2, dtype=float))[0]


def _absdiff(a, b, scale):
    return np.max(np.abs(np.asarray(a) - np.asarray(b)) / scale)


def test_between_closed_forms():
    """Limits (z1, z2) of eqs. 2.3-2.5 in universes with elementary integrals,
    either order of the limits; F(z1, z2) = G(x2) - G(x1) with the antiderivative G."""
    x1, x2 = 1.0 + Z1, 1.0 + Z2
    h0 = 70.0
    # Einstein-de Sitter: E = x^(3/2)
    p = (h0, 1.0, 0.0, 0.0)
    assert _absdiff(_bt("DC", p, Z1, Z2), 2 * DH(h0) * (x1 ** -0.5 - x2 ** -0.5), DH(h0)) < 1e-14
    assert _absdiff(_bt("T", p, Z1, Z2), (2 / 3) * TH(h0) * (x1 ** -1.5 - x2 ** -1.5), TH(h0)) < 1e-14
    assert _absdiff(_bt("X", p, Z1, Z2), (2 / 3) * DH(h0) * (x2 ** 1.5 - x1 ** 1.5),
                    DH(h0) * x2 ** 1.5) < 1e-14
    # radiation only: E = x^2
    p = (h0, 0.0, 0.0, 1.0)
    assert _absdiff(_bt("DC", p, Z1, Z2), DH(h0) * (1 / x1 - 1 / x2), DH(h0)) < 1e-14
    assert _absdiff(_bt("T", p, Z1, Z2), TH(h0) * 0.5 * (x1 ** -2 - x2 ** -2), TH(h0)) < 1e-14
    assert _absdiff(_bt("X", p, Z1, Z2), DH(h0) * (x2 - x1), DH(h0) * x2) < 1e-14
    # de Sitter: E = 1
    p = (h0, 0.0, 1.0, 0.0)
    assert _absdiff(_bt("DC", p, Z1, Z2), DH(h0) * (Z2 - Z1), DH(h0) * x2) < 1e-14
    assert _absdiff(_bt("T", p, Z1, Z2), TH(h0) * np.log(x2 / x1), TH(h0)) < 1e-14
    # Milne (Ok0 = 1): E = x, D_M(z1, z2) = D_H sinh(ln(x2/x1)), D_A = D_M/x2
    p = (h0, 0.0, 0.0, 0.0)
    dm = DH(h0) * 0.5 * (x2 / x1 - x1 / x2)
    assert _absdiff(_bt("DC", p, Z1, Z2), DH(h0) * np.log(x2 / x1), DH(h0)) < 1e-14
    assert _absdiff(_bt("DM", p, Z1, Z2), dm, DH(h0) * x2) < 1e-14
    assert _absdiff(_bt("DA", p, Z1, Z2), dm / x2, DH(h0)) < 1e-14
    assert _absdiff(_bt("T", p, Z1, Z2), TH(h0) * (1 / x1 - 1 / x2), TH(h0)) < 1e-14


def test_between_to_infinity_closed_forms():
    """z2 = inf: chi(z, inf) and the age t(z, inf) (sec. 2.1) in the same universes;
    the absorption distance diverges; D_A(z, inf) = 0."""
    zz = np.array([0.0, 0.1, 1.0, 10.0, 1000.0])
    x = 1.0 + zz
    inf = np.full_like(zz, np.inf)
    h0 = 67.0
    p = (h0, 1.0, 0.0, 0.0)
    assert rel(_bt("DC", p, zz, inf), 2 * DH(h0) * x ** -0.5) < 1e-14
    assert rel(_bt("T", p, zz, inf), (2 / 3) * TH(h0) * x ** -1.5) < 1e-14
    assert np.all(np.isinf(_bt("X", p, zz, inf)))
    p = (h0, 0.0, 0.0, 1.0)
    assert rel(_bt("DC", p, zz, inf), DH(h0) / x) < 1e-14
    assert rel(_bt("T", p, zz, inf), TH(h0) * 0.5 / x ** 2) < 1e-14
    p = (h0, 0.0, 0.0, 0.0)  # Milne: chi diverges logarithmically, t(z, inf) = t_H / x
    assert rel(_bt("T", p, zz, inf), TH(h0) / x) < 1e-14
    # open matter universe (Om0 = 0.3, Ok0 = 0.7): t(0, inf) in closed form
    om = 0.3
    ok = 1 - om
    age = TH(h0) * (1 / ok - om / ok ** 1.5 * math.asinh(math.sqrt(ok / om)))
    assert rel(_bt("T", (h0, om, 0.0, 0.0), [0.0], [np.inf]), [age]) < 1e-14
    assert np.all(_bt("DA", (70.0, 0.3, 0.7, 9e-5), zz, inf) == 0.0)


@pytest.mark.parametrize("p", COSMOS)
def test_between_additivity_and_one_sided(p):
    """chi(z1, z2) + chi(z2, z3) = chi(z1, z3) (and for t, d_abs); (0, z) is the
    one-sided oracle; z2 = inf is the limit of large finite z2 (the tail of chi above
    X = 1+Z is c/H0 [1/(sqrt(Or0) X) - Om0/(4 Or0^(3/2) X^2)] to second order, from
    E = sqrt(Or0) x^2 (1 + Om0/(2 Or0 x) + ...))."""
    za = np.array([0.0, 0.01, 0.4, 1.3, 7.0])
    zb = np.array([0.02, 0.5, 0.4, 3.0, 20.0])
    zc = np.array([1.0, 0.3, 2.5, 900.0, 21.0])
    for kind, tol in (("DC", 3e-15), ("T", 3e-15), ("X", 3e-15)):
        ab, bc, ac = (_bt(kind, p, u, v) for u, v in ((za, zb), (zb, zc), (za, zc)))
        assert _absdiff(ab + bc, ac, np.abs(ab) + np.abs(bc) + np.abs(ac)) < tol, kind
        assert rel(_bt(kind, p, np.zeros(4), zc[:4]), _ev(kind, p, zc[:4])) < 1e-14
    if p[3] > 0:
        zbig = 1e9
        X = 1 + zbig
        tail = DH(p[0]) * (1 / (math.sqrt(p[3]) * X) - p[1] / (4 * p[3] ** 1.5 * X ** 2))
        inf_ = _bt("DC", p, za, np.full_like(za, np.inf))
        fin = _bt("DC", p, za, np.full_like(za, zbig))
        assert rel(inf_, fin + tail) < 1e-12


def test_between_against_mpmath_quad():
    """Generic cosmologies, finite and infinite upper limits, against mpmath's
    tanh-sinh quadrature at 30 digits."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    for p in (COSMOS[0], COSMOS[3], COSMOS[6]):
        h0, om, ol, orr = (mpmath.mpf(v) for v in p)
        ok = 1 - om - ol - orr

        def E(zz):
            x = 1 + zz
            return mpmath.sqrt(orr * x ** 4 + om * x ** 3 + ok * x ** 2 + ol)

        for z1, z2 in ((0.2, 0.25), (1.0, 40.0), (3.0, mpmath.inf)):
            dc = mpmath.quad(lambda t: 1 / E(t), [z1, z2]) * C / h0
            tt = mpmath.quad(lambda t: 1 / ((1 + t) * E(t)), [z1, z2]) * mpmath.mpf(TH_FACTOR) / h0
            zz2 = float(z2)
            assert rel(_bt("DC", p, [z1], [zz2]), [float(dc)]) < 2e-14
            assert rel(_bt("T", p, [z1], [zz2]), [float(tt)]) < 2e-14


def test_between_reversed_and_tiny_radiation():
    """chi(z2, z1) = -chi(z1, z2) over a long interval; and chi(z, inf) with a tiny
    Or0 = eps next to Or0 = 0: the integrand in s = (1+z)^(-1/2) changes only near
    s ~ sqrt(eps/Om0), by -2 sqrt(eps)/Om0 in total (to leading order), which a
    quadrature that never samples that scale would miss."""
    p = COSMOS[3]
    for kind in ("DC", "T", "X"):
        f = _bt(kind, p, [0.001, 7.6], [7.6, 0.001])
        assert abs(f[0] + f[1]) <= 1e-15 * abs(f[0]), kind
    eps = 1e-16
    zz = np.array([0.0, 1.0, 30.0])
    inf = np.full_like(zz, np.inf)
    chi0 = _bt("DC", (70.0, 0.3, 0.7, 0.0), zz, inf)
    chie = _bt("DC", (70.0, 0.3, 0.7 - eps, eps), zz, inf)
    assert rel(chie, chi0 - DH(70.0) * 2 * math.sqrt(eps) / 0.3) < 1e-13


# --------------------------------------------------------------------------- supernova model (sec. 4)
def _mu_eds(h0, z):
    x = 1.0 + np.asarray(z, dtype=float)
    dl = x * 2 * DH(h0) * (1 - 1 / np.sqrt(x))
    return 5 * np.log10(dl) + 25


def test_snia_log_joint_value():
    """Einstein-de Sitter (Om0 = 1, OL0 = 0): mu in closed form; the photometric
    likelihood and the Gamma(3, rate 3) prior against scipy.stats."""
    from scipy import stats
    theta = np.array([[1.0, 0.0]])
    z = np.array([[0.35, 1.2, 2.5]])
    zhat = np.array([0.31, 1.3, 2.45])
    z_mu = np.array([0.4, 1.2, 2.0])  # muhat = mu_EdS at these redshifts
    muhat = _mu_eds(70.0, z_mu)
    lp = oracle.snia_log_joint(theta, z, zhat, muhat)
    ref = (-0.5 * ((muhat - _mu_eds(70.0, z[0])) / 0.14) ** 2
           + stats.norm.logpdf(zhat, z[0], (1 + z[0]) * 0.04) + 0.5 * math.log(2 * math.pi)
           + stats.gamma.logpdf(z[0], a=3.0, scale=1 / 3.0)).sum()
    assert abs(lp[0] - ref) <= 1e-12 * abs(ref)


def test_snia_log_joint_gradient_fd():
    """Gradients with respect to (Om0, OL0) and every z_s against central differences
    of the value (Richardson-extrapolated)."""
    rng = np.random.default_rng(2)
    theta = np.array([[0.31, 0.68], [0.25, 0.8]])
    z = rng.gamma(3.0, 1 / 3.0, (2, 5)) + 0.05
    zhat = z[0] + 0.04 * (1 + z[0]) * rng.standard_normal(5)
    muhat = oracle.distance("MU", [[70.0, 0.3, 0.7, 0.0]], z[0])[0] + 0.14 * rng.standard_normal(5)
    lp, dth, dz = oracle.snia_log_joint(theta, z, zhat, muhat, grad=True)

    def fd(f, h):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    for a in range(2):
        def f(h, a=a):
            t = theta.copy()
            t[:, a] += h
            return oracle.snia_log_joint(t, z, zhat, muhat)
        assert rel(dth[:, a], fd(f, 1e-4)) < 1e-7, a
    for j in range(5):
        def g(h, j=j):
            zz = z.copy()
            zz[:, j] += h
            return oracle.snia_log_joint(theta, zz, zhat, muhat)
        assert rel(dz[:, j], fd(g, 1e-4)) < 1e-7, j



# --------------------------------------------------------------------------- comoving volume
def test_comoving_volume_closed_forms():
    """V_C = 4 pi int D_M^2 dD_C: flat (EdS) 4 pi D_M^3 / 3; Milne (Ok0 = 1, chi = ln(1+z))
    4 pi D_H^3 (sinh(2 chi)/2 - chi)/2; a closed matter universe (Om0 = 3, Ok0 = -2)
    4 pi D_H^3 (chi - sin(2 a chi)/(2a)) / (2|Ok0|), a = sqrt(2), chi from Mattig's
    closed form of D_M."""
    h0 = 70.0
    z = np.array([0.05, 0.5, 1.0, 3.0, 10.0])
    x = 1 + z
    dm = 2 * DH(h0) * (1 - 1 / np.sqrt(x))
    assert rel(_ev("VC", (h0, 1.0, 0.0, 0.0), z), 4 * np.pi / 3 * dm ** 3) < 1e-13
    chi = np.log(x)
    assert rel(_ev("VC", (h0, 0.0, 0.0, 0.0), z), 4 * np.pi * DH(h0) ** 3 * (np.sinh(2 * chi) / 2 - chi) / 2) < 1e-13
    om, ok = 3.0, -2.0
    a = math.sqrt(-ok)
    # Mattig: D_M = 2 D_H (om z + (om - 2)(sqrt(1 + om z) - 1)) / (om^2 (1 + z))
    dmm = 2 * DH(h0) * (om * z + (om - 2) * (np.sqrt(1 + om * z) - 1)) / (om ** 2 * x)
    chi = np.arcsin(a * dmm / DH(h0)) / a  # below the antipode for these z
    g = (chi - np.sin(2 * a * chi) / (2 * a)) / (2 * abs(ok))
    assert rel(_ev("VC", (h0, om, 0.0, 0.0), z[:3]), 4 * np.pi * DH(h0) ** 3 * g[:3]) < 1e-12


@pytest.mark.parametrize("kind", ["DC", "DM", "DA", "T"])
def test_between_gradient_vs_richardson(kind):
    """Leibniz-rule gradients between two redshifts (and to infinity) against central
    differences of the oracle's own values, open and closed curvature."""
    for p in [(70.0, 0.3, 0.6, 1e-4), (66.0, 0.45, 0.85, 3e-5), (72.0, 0.2, 0.3, 0.0)]:
        for z1, z2 in ((0.4, 1.9), (2.5, 0.7), (1.1, np.inf)):
            if kind == "DA" and np.isinf(z2):
                continue
            _, g = oracle.between(kind, np.array([p]), np.array([z1]), np.array([z2]), grad=True)
            g = g[0, 0]
            base = list(p) + [z1, z2]
            for a, h in zip(range(6), (1e-2, 1e-4, 1e-4, 1e-6, 1e-4, 1e-4)):
                if a == 5 and np.isinf(z2):
                    assert g[5] == 0.0
                    continue
                if a == 3 and np.isinf(z2) and p[3] == 0.0:
                    # d chi(z, inf)/d Or0 at Or0 = 0 is -inf (chi_eps = chi_0 - 2 sqrt(eps)/Om0 ...)
                    assert g[3] == -np.inf or (kind == "T" and np.isfinite(g[3]))
                    continue

                def f(v, a=a):
                    q = list(base)
                    q[a] = v
                    return oracle.between(kind, np.array([q[:4]]), np.array([q[4]]), np.array([q[5]]))[0, 0]
                fd = _richardson(f, base[a], h)
                v0 = f(base[a])
                scale = max(abs(fd), 1e-6 * abs(v0) / max(abs(base[a]), 1e-4), 1e-12)
                tol = 1e-5 if a == 3 else 1e-7
                assert abs(g[a] - fd) <= tol * scale + 1e-6 * abs(g[a]) * (a == 3), (kind, p, z1, z2, a, g[a], fd)
