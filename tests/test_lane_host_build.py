"""The per-lane forward formulas of the HIP path (csrc/lane.hpp: eqs. 3.7-3.9 and
B.1-B.3 through the structured Carlson duplication, with the quadrature routes),
compiled for the host through a stand-in HIP header and checked against the oracle
without a GPU, element by element:
  * FP64 path: relative error <= 1e-12;
  * FP32 path: relative error <= 1e-6 with the hardware square root / reciprocal
    modelled as correctly rounded, and also with each such result moved by a random
    +-1 ulp (the accuracy of the gfx950 instructions), on the near-degenerate and
    non-flat workloads at their full redshift ranges."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2212_01937_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
KIND = {"DC": 0, "T": 4, "X": 5}


def _build(out, noise):
    flags = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=fast", "-I", os.path.join(HERE, "host_shim")]
    if noise:
        flags.append("-DCOSMO_HOST_NOISE")
    src = os.path.join(HERE, "host_shim", "lane_host.cpp")
    try:
        subprocess.run(["g++", *flags, "-mfma", src, "-o", out], check=True)
    except subprocess.CalledProcessError:
        subprocess.run(["g++", *flags, src, "-o", out], check=True)
    return ctypes.CDLL(out)


@pytest.fixture(scope="module")
def libs(tmp_path_factory):
    d = tmp_path_factory.mktemp("lane")
    return {"exact": _build(str(d / "liblane.so"), False), "noisy": _build(str(d / "liblane_noisy.so"), True)}


def host_eval(lib, p, kind, dt, z):
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.zeros(z.size)
    lib.host_eval(np.ascontiguousarray(p, dtype=np.float64).ctypes.data_as(ctypes.c_void_p), KIND[kind], dt,
                  z.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(z.size), out.ctypes.data_as(ctypes.c_void_p))
    return out


def cases():
    p4, z4, fam = workloads.config4(n_per_family=6, n_z=400, seed=21)
    yield "config4", p4, np.broadcast_to(z4, (p4.shape[0], z4.size))
    p2, z2 = workloads.config2(n_cosmo=24, n_z=400, seed=21)
    yield "config2", p2, z2


@pytest.mark.parametrize("kind", ["DC", "T", "X"])
def test_fp64_formulas_match_oracle(libs, kind):
    for label, p, z in cases():
        for c in range(p.shape[0]):
            ref = oracle.distance(kind, p[c:c + 1], z[c])[0]
            got = host_eval(libs["exact"], p[c], kind, 1, z[c])
            e = np.abs(got / ref - 1)
            assert e.max() <= 1e-12, (label, kind, c, e.max(), z[c][np.argmax(e)])


@pytest.mark.parametrize("model", ["exact", "noisy"])
@pytest.mark.parametrize("kind", ["DC", "T", "X"])
def test_fp32_formulas_within_bound(libs, kind, model):
    for label, p, z in cases():
        z32 = z.astype(np.float32).astype(np.float64)
        for c in range(p.shape[0]):
            ref = oracle.distance(kind, p[c:c + 1], z32[c])[0]
            got = host_eval(libs[model], p[c], kind, 0, z32[c])
            e = np.abs(got / ref - 1)
            assert e.max() <= 1e-6, (label, kind, model, c, e.max(), z32[c][np.argmax(e)])


def _triples(rng, n):
    """Structured Carlson triples like the distance kernels': x > 0 with a
    conjugate pair (a +- i b, any sign of a, b != 0) or two more positive reals;
    magnitudes over four decades, so that the duplication runs from zero to many
    steps."""
    for _ in range(n):
        pair = bool(rng.random() < 0.5)
        x = 10.0 ** rng.uniform(-2, 2)
        if pair:
            r, th = 10.0 ** rng.uniform(-2, 2), rng.uniform(-0.95, 0.95) * np.pi
            yield pair, x, r * np.cos(th), r * np.sin(th)
        else:
            yield pair, x, 10.0 ** rng.uniform(-2, 2), 10.0 ** rng.uniform(-2, 2)


@pytest.mark.parametrize("model", ["exact", "noisy"])
def test_structured_rf_rd_match_oracle(libs, model):
    """rfd_s: R_F and the three R_D(., ., x_k) of one duplication sequence (the R_D
    tails from the derivative of the R_F expansion, eq. 2.10) against the oracle's
    quadrature of the defining integrals (eqs. 2.6, 2.9), FP64 and FP32 (the oracle
    at the FP32-rounded arguments), plus the identity sum_k R_D(., ., x_k) =
    3 / sqrt(x y z)."""
    rng = np.random.default_rng(7)
    worst = {0: 0.0, 1: 0.0}
    for pair, x, a, b in _triples(rng, 300):
        for dt, tol in ((1, 1e-13), (0, 2e-6 if model == "exact" else 4e-6)):
            if dt == 0:
                x, a, b = (float(np.float32(v)) for v in (x, a, b))
            y, zc = (complex(a, b), complex(a, -b)) if pair else (complex(a), complex(b))
            out = np.zeros(5)
            libs[model].host_rfd(dt, int(pair), ctypes.c_double(x), ctypes.c_double(a), ctypes.c_double(b),
                                 out.ctypes.data_as(ctypes.c_void_p))
            rf = oracle.carlson("RF", x, y, zc)[0]
            rdx = oracle.carlson("RD", y, zc, x)[0]
            rdy = oracle.carlson("RD", x, zc, y)[0]
            rdz = oracle.carlson("RD", x, y, zc)[0]
            got_rdy = complex(out[2], out[3])
            got_rdz = np.conj(got_rdy) if pair else complex(out[4])
            errs = [abs(out[0] - rf) / abs(rf), abs(out[1] - rdx) / abs(rdx), abs(got_rdy - rdy) / abs(rdy),
                    abs(got_rdz - rdz) / abs(rdz)]
            assert max(errs) <= tol, (dt, pair, x, a, b, errs)
            ident = 3.0 / np.sqrt(complex(x) * y * zc)
            s = out[1] + got_rdy + got_rdz
            assert abs(s - ident) <= 10 * tol * (abs(out[1]) + abs(got_rdy) + abs(got_rdz)), (dt, pair, x, a, b)
            worst[dt] = max(worst[dt], max(errs))
    print("max relative error", worst)


@pytest.mark.parametrize("model", ["exact", "noisy"])
def test_rc_with_x_derivative_matches_oracle(libs, model):
    """rc_rd_r: R_C(x, y) and R_D(y, y, x) = -6 dR_C/dx (eq. 2.10 with R_C = R_F(x, y, y))
    against the oracle's R_C and R_D, on pairs within the m = 0 tail's range (the FP32
    fast path: |x/y - 1| up to 0.3) and far outside it (duplication), FP64 and FP32 (the
    oracle at the FP32-rounded arguments)."""
    rng = np.random.default_rng(11)
    y = 10.0 ** rng.uniform(-3, 3, 400)
    near = y * (1.0 + rng.uniform(-0.3, 0.3, 400))
    far = y * 10.0 ** rng.uniform(-4, 4, 400)
    for x in (near, far):
        for dt, tol in ((1, 1e-13), (0, 2e-6 if model == "exact" else 4e-6)):
            xa, ya = (x, y) if dt == 1 else (x.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64))
            out = np.zeros(2 * x.size)
            libs[model].host_rc_rd(dt, xa.ctypes.data_as(ctypes.c_void_p), ya.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.c_long(x.size), out.ctypes.data_as(ctypes.c_void_p))
            rc = np.real(oracle.carlson("RC", xa, ya))
            rd = np.real(oracle.carlson("RD", ya, ya, xa))
            assert np.max(np.abs(out[0::2] - rc) / rc) <= tol, (dt, model)
            assert np.max(np.abs(out[1::2] - rd) / rd) <= tol, (dt, model)


@pytest.mark.parametrize("model", ["exact", "noisy"])
def test_refined_square_roots_of_the_time_coordinate(libs, model):
    """sqrt_nr (the FP32 root refined by one Newton step with an FP32 correction) against
    the correctly rounded FP64 root: within 1e-13 relative over 1e-6..1e6, also with the
    FP32 reciprocal square root off by an ulp ('noisy').  side_at_mixed's FP64 sides of one
    limit (sqrt(1 - sigma x), sqrt(x - rho_n), a pair's complex root and |x - rho_1|)
    against FP64 square roots of the same record's constants (pairs and three real roots;
    1e-13, 5e-13 'noisy'),
    and, on the well separated roots of the large-batch and non-flat cosmologies, against
    their definitions from the oracle's 50-digit roots."""
    lib = libs[model]
    x = 10.0 ** np.random.default_rng(13).uniform(-6, 6, 5000)
    out = np.zeros_like(x)
    lib.host_sqrt_nr(x.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(x.size), out.ctypes.data_as(ctypes.c_void_p))
    assert np.max(np.abs(out - np.sqrt(x)) / np.sqrt(x)) < 1e-13
    z = np.concatenate([np.linspace(0.0, 20.0, 400), 10.0 ** np.linspace(-5, 3, 400)]).astype(np.float32).astype(np.float64)
    xx = 1.0 + z
    p5, _ = workloads.config5(n_cosmo=4, n_z=8)
    p2, _ = workloads.config2(n_cosmo=4, n_z=8)
    p4, _, _ = workloads.config4(n_per_family=8, n_z=8)  # families C and D: three real roots
    for which, params in (("separated", np.concatenate([p5, p2])), ("record only", p4[16:32:3])):
        for prm in params:
            o = np.zeros(12 * z.size)
            lib.host_side_mixed(np.ascontiguousarray(prm).ctypes.data_as(ctypes.c_void_p),
                                z.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(z.size),
                                o.ctypes.data_as(ctypes.c_void_p))
            o = o.reshape(-1, 12)
            got, rec = o[:, :6], o[:, 6:]
            scale = np.maximum(np.abs(rec), 1e-300)
            used = np.abs(rec) > 0
            # one Newton step from a root within ~1 ulp of FP32: ~1e-14, up to ~2e-13 where
            # the FP32 estimates are themselves 1 ulp off ('noisy')
            assert np.max((np.abs(got - rec) / scale)[used]) < (1e-13 if model == "exact" else 5e-13), (which, prm)
            if which == "record only":
                continue
            sigma, rho = oracle_roots(prm)
            t = np.sqrt(1.0 - sigma * xx)
            assert np.max(np.abs(got[:, 0] - t) / t) < 1e-12
            n0 = np.sqrt(xx - rho[0].real)
            assert np.max(np.abs(got[:, 1] - n0) / n0) < 1e-12
            n1 = got[:, 2] + 1j * got[:, 3]
            ref = np.sqrt((xx - rho[1]).astype(complex))
            ref = np.where(np.sign(ref.imag) == np.sign(n1.imag), ref, np.conj(ref))
            assert np.max(np.abs(n1 - ref) / np.abs(ref)) < 1e-12
            assert np.max(np.abs(got[:, 4] - np.abs(xx - rho[1])) / np.abs(xx - rho[1])) < 1e-12


def oracle_roots(prm):
    """sigma = 1/x_l (x_l the radiation root of P(x) = Or x^4 + Om x^3 + Ok x^2 + OL, the
    real root of largest modulus; 0 without radiation) and the roots rho_n of the cubic
    factor (a real root, then a pair with positive imaginary part first), from the
    oracle's 50-digit roots."""
    x = oracle.roots(prm[None, :])[0] + 1.0
    x = x[np.isfinite(x)]
    order = np.argsort(-np.abs(x))
    if prm[3] > 0:
        sigma, rest = 1.0 / x[order[0]].real, list(x[order[1:]])
    else:
        sigma, rest = 0.0, list(x)
    cplx = [v for v in rest if abs(v.imag) > 1e-12 * max(1.0, abs(v))]
    assert len(cplx) == 2, "a root pair is expected here"
    r0 = [v for v in rest if abs(v.imag) <= 1e-12 * max(1.0, abs(v))][0]
    r1 = max(cplx, key=lambda v: v.imag)
    return sigma, [complex(r0.real, 0.0), r1, r1.conjugate()]


KIND_BTW = {"DC": 0, "DM": 1, "T": 4, "DA": 6}


def host_between(lib, p, kind, dt, z1, z2):
    z1 = np.ascontiguousarray(z1, dtype=np.float64)
    z2 = np.ascontiguousarray(z2, dtype=np.float64)
    out = np.zeros(z1.size)
    lib.host_between(np.ascontiguousarray(p, dtype=np.float64).ctypes.data_as(ctypes.c_void_p), KIND_BTW[kind], dt,
                     z1.ctypes.data_as(ctypes.c_void_p), z2.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(z1.size),
                     out.ctypes.data_as(ctypes.c_void_p))
    return out


def between_pairs(rng, n):
    """Seeded limit pairs: log-uniform z1 on [1e-4, 10], z2 = z1 + a log-uniform step on
    [1e-6, 10] (close planes to long baselines), some reversed, some z2 = inf."""
    z1 = 10.0 ** rng.uniform(-4, 1, n)
    z2 = z1 + 10.0 ** rng.uniform(-6, 1, n)
    flip = rng.random(n) < 0.2
    z1[flip], z2[flip] = z2[flip], z1[flip].copy()
    z2[rng.random(n) < 0.1] = np.inf
    return z1, z2


def _between_cases():
    p4, _, _ = workloads.config4(n_per_family=4, n_z=8, seed=23)
    p2, _ = workloads.config2(n_cosmo=16, n_z=8, seed=23)
    return np.concatenate([p4, p2])


@pytest.mark.parametrize("model", ["exact", "noisy"])
@pytest.mark.parametrize("kind", ["DC", "DM", "DA", "T"])
def test_between_formulas_match_oracle(libs, kind, model):
    """between.hpp (eqs. 3.7-3.8 with both limits per lane; z2 = inf by the limit form)
    against the oracle's quadrature from z1 to z2: FP64 <= 1e-12 relative, FP32 <= 1e-6
    relative (D_M and D_A relative to the conditioning scale |D_M| + |C chi| D_H as in
    the one-sided tests), at the FP32-rounded limits for FP32."""
    rng = np.random.default_rng(5)
    params = _between_cases()
    for c in range(params.shape[0]):
        z1, z2 = between_pairs(rng, 60)
        if kind in ("DM", "DA"):
            z2[np.isinf(z2)] = 1e4  # the transverse distances at infinity are covered by DC
        for dt, tol in ((1, 1e-12), (0, 1e-6)):
            if dt == 1 and model == "noisy":
                continue
            a = z1.astype(np.float32).astype(np.float64) if dt == 0 else z1
            b = z2.astype(np.float32).astype(np.float64) if dt == 0 else z2
            ref = oracle.between(kind, params[c:c + 1], a, b)[0]
            got = host_between(libs[model], params[c], kind, dt, a, b)
            fin = np.isfinite(ref)
            if kind in ("DM", "DA"):
                chi = oracle.between("DC", params[c:c + 1], a, b)[0]
                ok = 1 - params[c, 1:].sum()
                h = 299792.458 / params[c, 0]
                sk = np.sqrt(abs(ok)) if ok != 0 else 0.0
                cc = np.cosh(sk * chi / h) if ok > 0 else (np.cos(sk * chi / h) if ok < 0 else 1.0)
                scale = np.abs(ref) + np.abs(cc * chi) / (1 + (b if kind == "DA" else 0))
            else:
                scale = np.abs(ref)
            e = np.abs(got - ref)[fin] / np.maximum(scale[fin], 1e-300)
            assert e.size and e.max() <= tol, (kind, model, dt, c, e.max(), a[fin][np.argmax(e)], b[fin][np.argmax(e)])
            assert np.all(got[a == b] == 0.0)


def host_time_between_grad(lib, p, dt, z1, z2):
    z1 = np.ascontiguousarray(z1, dtype=np.float64)
    z2 = np.ascontiguousarray(z2, dtype=np.float64)
    out = np.zeros((z1.size, 3))
    lib.host_time_between_grad(np.ascontiguousarray(p, dtype=np.float64).ctypes.data_as(ctypes.c_void_p), dt,
                               z1.ctypes.data_as(ctypes.c_void_p), z2.ctypes.data_as(ctypes.c_void_p),
                               ctypes.c_long(z1.size), out.ctypes.data_as(ctypes.c_void_p))
    return out


def test_time_between_gradient_matches_oracle(libs):
    """gl_time_between (the Leibniz-rule derivatives of t(z1, z2) in s = (1+z)^(-1/2),
    to z2 = inf) against the oracle's Leibniz derivatives from its own quadrature in
    u = ln(1+z): FP64 <= 1e-10, FP32 <= 1e-4 of |d t/d theta| + 1e-3 |t| (the floor
    where a derivative crosses zero), on the non-flat and near-degenerate sets."""
    rng = np.random.default_rng(9)
    params = _between_cases()
    for c in range(params.shape[0]):
        z1, z2 = between_pairs(rng, 40)
        th = 977.7922216807892 / params[c, 0]
        for dt, tol in ((1, 1e-10), (0, 1e-4)):
            a = z1.astype(np.float32).astype(np.float64) if dt == 0 else z1
            b = z2.astype(np.float32).astype(np.float64) if dt == 0 else z2
            val, g = oracle.between("T", params[c:c + 1], a, b, grad=True)
            ref = g[0, :, 1:4] / th
            got = host_time_between_grad(libs["exact"], params[c], dt, a, b)
            fin = np.isfinite(ref).all(1)
            scale = np.abs(ref) + 1e-3 * np.abs(val[0] / th)[:, None]
            e = np.abs(got - ref)[fin] / scale[fin]
            assert e.size and e.max() <= tol, (dt, c, params[c], float(e.max()))


def host_x_route(lib, p, dt, z):
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.zeros(z.size, dtype=np.int32)
    lib.host_x_route(np.ascontiguousarray(p, dtype=np.float64).ctypes.data_as(ctypes.c_void_p), dt,
                     z.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(z.size), out.ctypes.data_as(ctypes.c_void_p))
    return out


def test_x_takes_the_carlson_route_on_every_workload(libs):
    """The absorption distance (eq. 3.9 in its regular arrangement, eq. B.3) needs no
    quadrature on any workload: route 0 (Carlson in the lane precision) or, for FP32
    lanes whose terms cancel by more than 8, route 1 (the same formulas in FP64); never
    route 2 (Gauss-Legendre).  Workloads 1, 2, 4 (all families) and 5 at their full
    redshift ranges."""
    p1, z1 = workloads.config1()
    p2, z2 = workloads.config2(n_cosmo=64, n_z=256, seed=31)
    p4, z4, _ = workloads.config4(n_per_family=16, n_z=256, seed=31)
    p5, z5 = workloads.config5(n_cosmo=32, n_z=256, seed=31)
    sets = [(p1, np.broadcast_to(z1, (1, z1.size))), (p2, z2), (p4, np.broadcast_to(z4, (p4.shape[0], z4.size))),
            (p5, np.broadcast_to(z5, (p5.shape[0], z5.size)))]
    counts = np.zeros((2, 3), dtype=np.int64)
    for p, z in sets:
        for c in range(p.shape[0]):
            for dt in (0, 1):
                r = host_x_route(libs["exact"], p[c], dt, z[c])
                assert (r >= 0).all() and (r <= 2).all()
                counts[dt] += np.bincount(r, minlength=3)
    print("FP32 routes (Carlson, FP64, quadrature)", counts[0], "FP64 routes", counts[1])
    assert counts[0, 2] == 0 and counts[1, 2] == 0
    assert counts[1, 1] == 0  # the FP64 path has no FP64 re-evaluation route


@pytest.mark.parametrize("model", ["exact", "noisy"])
def test_rfjx_derivative_matches_mpmath(libs, model):
    """rfjx_s: R_F, R_J(x, y, z, p) and dR_J/dx (forward-mode through the duplication)
    against mpmath's R_F, R_J and its numerical derivative of R_J at 30 digits, on
    structured triples with p both close to x (relative 1e-9 .. 1, the regular form of
    eq. 3.9) and unrelated to it: FP64 <= 2e-14, FP32 <= 4e-6 (arguments rounded)."""
    import mpmath as mp
    mp.mp.dps = 30
    rng = np.random.default_rng(17)
    for n, (pair, x, a, b) in enumerate(_triples(rng, 120)):
        p = x * (1 + rng.choice([-1, 1]) * 10 ** rng.uniform(-9, 0)) if n % 2 else 10 ** rng.uniform(-2, 2)
        for dt, tol in ((1, 2e-14), (0, 4e-6)):
            if dt == 0:
                x, a, b, p = (float(np.float32(v)) for v in (x, a, b, p))
            y, zc = (mp.mpc(a, b), mp.mpc(a, -b)) if pair else (mp.mpf(a), mp.mpf(b))
            ref = [mp.re(mp.elliprf(x, y, zc)), mp.re(mp.elliprj(x, y, zc, p)),
                   mp.re(mp.diff(lambda t: mp.elliprj(t, y, zc, p), x))]
            out = np.zeros(3)
            libs[model].host_rfjx(dt, int(pair), ctypes.c_double(x), ctypes.c_double(a), ctypes.c_double(b),
                                  ctypes.c_double(p), out.ctypes.data_as(ctypes.c_void_p))
            errs = [abs(out[k] / float(ref[k]) - 1) for k in range(3)]
            assert max(errs) <= tol, (dt, pair, x, a, b, p, errs)


def host_between_grad(lib, p, kind, dt, z1, z2):
    z1 = np.ascontiguousarray(z1, dtype=np.float64)
    z2 = np.ascontiguousarray(z2, dtype=np.float64)
    out = np.zeros((z1.size, 6))
    lib.host_between_grad(np.ascontiguousarray(p, dtype=np.float64).ctypes.data_as(ctypes.c_void_p), KIND_BTW[kind],
                          dt, z1.ctypes.data_as(ctypes.c_void_p), z2.ctypes.data_as(ctypes.c_void_p),
                          ctypes.c_long(z1.size), out.ctypes.data_as(ctypes.c_void_p))
    return out


def test_time_between_root_chain_gradient_matches_oracle(libs):
    """t(z1, z2) differentiated through eq. 3.8 with both limits (t_grad_between: Carlson
    derivatives, eqs. 2.10-2.11, and the root Jacobian of app. A), finished with the
    root-Jacobian contraction, against the oracle's Leibniz derivatives in (Om0, OL0, Or0)
    and its fundamental-theorem limit derivatives: FP64 <= 1e-11, FP32 <= 1e-4 (Or0: 5e-4,
    the root-chain cancellation of that component), each relative to the largest
    magnitude of that derivative over the lanes of the cosmology; lens-source pairs, close
    limits and the age t(z, inf) on the headline and non-flat cosmologies."""
    rng = np.random.default_rng(19)
    p5, _ = workloads.config5(n_cosmo=6, n_z=4, seed=19)
    p2, _ = workloads.config2(n_cosmo=6, n_z=4, seed=19)
    for p in np.concatenate([p5, p2]):
        z1 = rng.uniform(0.05, 1.5, 60)
        z2 = z1 + rng.uniform(0.01, 2.0, 60)
        z2[:10] = z1[:10] + 10.0 ** rng.uniform(-6, -2, 10)
        z1[40:] = rng.uniform(0.0, 20.0, 20)
        z2[40:] = np.inf
        for dt, tol in ((1, (1e-11, 1e-11, 1e-11)), (0, (1e-4, 1e-4, 5e-4))):
            a = z1.astype(np.float32).astype(np.float64) if dt == 0 else z1
            b = z2.astype(np.float32).astype(np.float64) if dt == 0 else z2
            val, g = oracle.between("T", p[None], a, b, grad=True)
            got = host_between_grad(libs["exact"], p, "T", dt, a, b)
            assert np.max(np.abs(got[:, 0] / val[0] - 1)) <= (1e-12 if dt == 1 else 1e-6)
            for th in range(3):
                ref = g[0, :, 1 + th]
                e = np.abs(got[:, 1 + th] - ref) / np.abs(ref).max()
                assert e.max() <= tol[th], (dt, th, p, float(e.max()))
            fin = np.isfinite(b)
            for q, col in ((4, 4), (5, 5)):
                ref = g[0, fin, col]
                e = np.abs(got[fin, q] - ref) / np.abs(ref).max()
                assert e.max() <= (1e-12 if dt == 1 else 1e-6), (dt, q, float(e.max()))


def test_sincos_reduction_matches_library(libs):
    """sincos_red (sin and cos of the curvature transform, sec. 2.1.1 for Ok0 < 0):
    Cody-Waite reduction by pi/2 and Taylor polynomials, against numpy's sin and cos
    in FP64 on arguments spanning every quadrant up to several windings, both signs,
    and the multiples of pi/2 where one of the two crosses zero: FP64 within 2e-16
    absolute (the functions are bounded by one), FP32 within 2.5e-7 of the FP64 value of
    the float argument; NaN beyond |x| = 2^16."""
    rng = np.random.default_rng(23)
    x = np.concatenate([rng.uniform(-40.0, 40.0, 4000), np.arange(-24, 25) * (np.pi / 2),
                        10.0 ** rng.uniform(-8, 0, 200), [0.0, 1e-30, 65535.0]])
    for dt, tol in ((1, 2e-16), (0, 2.5e-7)):
        xa = x.astype(np.float32).astype(np.float64) if dt == 0 else x
        s = np.zeros(x.size)
        c = np.zeros(x.size)
        libs["exact"].host_sincos(dt, xa.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(x.size),
                                  s.ctypes.data_as(ctypes.c_void_p), c.ctypes.data_as(ctypes.c_void_p))
        assert np.max(np.abs(s - np.sin(xa))) <= tol, dt
        assert np.max(np.abs(c - np.cos(xa))) <= tol, dt
        # relative accuracy near zero (sin x ~ x): the reduction leaves r = x there
        small = np.abs(xa) < 1e-3
        eps = np.finfo(np.float32 if dt == 0 else np.float64).eps
        assert np.all(np.abs(s[small] - np.sin(xa[small])) <= 2 * eps * np.abs(xa[small]))
    big = np.array([7e4, -1e6, np.inf])
    s = np.zeros(3)
    c = np.zeros(3)
    libs["exact"].host_sincos(1, big.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(3),
                              s.ctypes.data_as(ctypes.c_void_p), c.ctypes.data_as(ctypes.c_void_p))
    assert np.all(np.isnan(s)) and np.all(np.isnan(c))


def test_fp64_log10_and_exp_match_library(libs):
    """The FP64 lanes' log10 (mu = 5 log10(D_L/Mpc) + 25, fn. 22) and exp (sinh of the
    curvature transform for Ok0 > 0, sec. 2.1.1), written as polynomials (atanh series of
    the reduced mantissa; Taylor series after reduction by ln 2): against numpy within
    4 ulp relative (exp: on the curvature transform's range; log10: on distances from
    1e-3 to 1e6 Mpc and beyond, subnormal included), the special values as the library."""
    rng = np.random.default_rng(29)
    x = np.concatenate([10.0 ** rng.uniform(-3, 6, 5000), 10.0 ** rng.uniform(-300, 300, 500),
                        [1.0, 2.0, 0.5, np.sqrt(0.5), np.sqrt(2.0), 10.0, 1e-310]])
    lg = np.zeros(x.size)
    ex = np.zeros(x.size)
    libs["exact"].host_log10_exp(x.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(x.size),
                                 lg.ctypes.data_as(ctypes.c_void_p), ex.ctypes.data_as(ctypes.c_void_p))
    ref = np.log10(x)
    err = np.abs(lg - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() <= 4 * np.finfo(float).eps, float(err.max())
    xe = np.concatenate([rng.uniform(-30.0, 30.0, 5000), [0.0, 1.0, -1.0, 700.0]])
    lg = np.zeros(xe.size)
    ex = np.zeros(xe.size)
    libs["exact"].host_log10_exp(xe.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(xe.size),
                                 lg.ctypes.data_as(ctypes.c_void_p), ex.ctypes.data_as(ctypes.c_void_p))
    e = np.abs(ex / np.exp(xe) - 1)
    assert e.max() <= 4 * np.finfo(float).eps, float(e.max())
    sp = np.array([0.0, -1.0, np.inf, np.nan])
    lg = np.zeros(4)
    ex = np.zeros(4)
    libs["exact"].host_log10_exp(sp.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(4),
                                 lg.ctypes.data_as(ctypes.c_void_p), ex.ctypes.data_as(ctypes.c_void_p))
    assert lg[0] == -np.inf and np.isnan(lg[1]) and lg[2] == np.inf and np.isnan(lg[3])
