"""GPU parity of the forward path against the CPU oracle (element by element).

FP64 path: max relative error <= 1e-12 (D_C, D_M, D_L, D_A, T, X); mu absolute
<= 2.2e-12 mag (a relative error 1e-12 of D_L moves mu by 5/ln 10 x 1e-12).  FP32 path
(FP64 roots): max relative error <= 1e-6, mu <= 1e-4 mag absolute (the stated bounds
of the method's two precisions).  Beyond the antipode of a closed universe D_M and mu
are measured against the size a relative error of chi moves them by (cond_scale).
"""
import numpy as np
import pytest
import torch

import oracle
from margins import note
from paper_2212_01937_amd import cosmo, workloads

pytestmark = pytest.mark.gpu

KINDS = ["DC", "DM", "DL", "MU", "T", "X", "DA", "VC"]
TOL = {torch.float64: 1e-12, torch.float32: 1e-6}
MU_TOL = {torch.float64: 2.2e-12, torch.float32: 1e-4}


def cond_scale(kind, params, z, ref):
    """Error scale of an observable that applies the curvature transform sinn to
    chi = D_C/D_H: a relative error eps in chi moves it by eps |d out/d chi| chi, which
    beyond the antipode of a closed universe (sin near zero) exceeds eps |out|.
    Returns |out| + |d out/d chi| chi (mu, in magnitudes: max(1, |C chi / S|), the
    factor by which a relative error of chi exceeds the relative error of D_L it causes,
    which is 1 for a flat universe; the comoving volume: max(|V|, chi dV/dchi))."""
    params = np.asarray(params, dtype=np.float64).reshape(-1, 4)
    n = params.shape[0]
    ref2 = np.asarray(ref, dtype=np.float64).reshape(n, -1)
    zz = np.broadcast_to(np.asarray(z, dtype=np.float64).reshape(-1) if np.size(z) == ref2.shape[1]
                         else np.asarray(z, dtype=np.float64).reshape(n, -1), ref2.shape)
    dc = oracle.distance("DC", params, np.ascontiguousarray(zz), shared_z=False)
    dh = 299792.458 / params[:, :1]
    ok = (1 - params[:, 1] - params[:, 2] - params[:, 3])[:, None]
    chi = dc / dh
    x = np.sqrt(np.abs(ok)) * chi
    c = np.where(ok < 0, np.cos(x), np.cosh(x))
    sk = np.where(ok == 0, 1.0, np.sqrt(np.abs(ok)))
    s = np.where(ok == 0, chi, np.where(ok < 0, np.sin(x), np.sinh(x)) / sk)
    if kind == "MU":
        with np.errstate(divide="ignore", invalid="ignore"):
            out = np.maximum(1.0, np.abs(c * chi / s))
    elif kind == "VC":
        # V_C = 4 pi D_H^3 G(chi): a relative error eps in chi moves it by eps chi dV/dchi
        # = eps 4 pi D_H^3 chi S^2 (about 3 |V| for small curvature)
        out = np.maximum(np.abs(ref2), 4 * np.pi * dh ** 3 * chi * s ** 2)
    else:
        factor = {"DM": 1.0, "DL": 1 + zz, "DA": 1 / (1 + zz)}[kind]
        out = np.abs(ref2) + np.abs(dh * c * chi * factor)
    return out.reshape(np.shape(ref))


def errs(kind, got, ref, scale=None):
    got = np.asarray(got, dtype=np.float64)
    if kind == "MU":
        e = np.abs(got - ref)
        return e if scale is None else e / scale
    return np.abs(got - ref) / (np.abs(ref) if scale is None else scale)


def check(kind, dt, got, ref, label="", params=None, z=None):
    got = np.asarray(got)
    ref = np.asarray(ref)
    scale = None
    if params is not None and kind in ("DM", "DL", "DA", "MU", "VC"):
        scale = cond_scale(kind, params, z, ref).ravel()
    got = got.ravel()
    ref = ref.ravel()
    # mu is undefined (NaN on both sides) where D_L <= 0, beyond the antipode of a
    # closed universe; everything else must be finite
    undef = np.isnan(ref) if kind == "MU" else np.zeros(ref.shape, bool)
    differ = np.isnan(got) != undef
    if kind == "MU" and differ.any() and params is not None:
        # a sign flip of D_M within rounding of the antipode is allowed
        p2 = np.asarray(params, dtype=np.float64).reshape(-1, 4)
        zz = np.broadcast_to(np.asarray(z, dtype=np.float64).reshape(-1) if np.size(z) * p2.shape[0] == ref.size
                             else np.asarray(z, dtype=np.float64).reshape(p2.shape[0], -1),
                             (p2.shape[0], ref.size // p2.shape[0]))
        dm = oracle.distance("DM", p2, np.ascontiguousarray(zz), shared_z=False).ravel()
        dh = np.broadcast_to(299792.458 / p2[:, :1], zz.shape).ravel()
        differ &= ~(np.abs(dm) <= 100 * TOL[dt] * dh)
    assert not differ.any(), (label, kind, dt, "NaN pattern differs from the oracle")
    undef |= np.isnan(got)
    assert np.all(np.isfinite(got[~undef])), (label, kind, dt, "non-finite output")
    got, ref = got[~undef], ref[~undef]
    if scale is not None:
        scale = scale[~undef]
    if got.size == 0:
        return
    e = errs(kind, got, ref, scale)
    tol = MU_TOL[dt] if kind == "MU" else TOL[dt]
    i = int(np.argmax(e))
    note(f"fwd {label} {kind} {dt}", e[i], tol)
    assert e[i] <= tol, f"{label} {kind} {dt}: max err {e[i]:.3e} at flat index {i}"


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_config1_golden(dev, dt):
    g = np.loadtxt(__file__.rsplit("/", 1)[0] + "/golden/config1_oracle.txt")
    params, z = workloads.config1()
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(z, dtype=dt, device=dev)
    zref = zt.double().cpu().numpy()  # the oracle sees the same (rounded) redshifts
    for kind, col in (("DC", 1), ("DL", 2), ("MU", 3)):
        out = cosmo.cosmo_distance(kind, p, zt)[0].cpu().numpy()
        ref = g[:, col] if dt == torch.float64 else oracle.distance(kind, params, zref)[0]
        check(kind, dt, out, ref, "config1")


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_config1_all_kinds(dev, dt):
    params, z = workloads.config1()
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(z, dtype=dt, device=dev)
    zref = zt.double().cpu().numpy()
    for kind in KINDS:
        out = cosmo.cosmo_distance(kind, p, zt)[0].cpu().numpy()
        check(kind, dt, out, oracle.distance(kind, params, zref)[0], "config1")


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_config2_subset_per_cosmology_z(dev, dt):
    """37 cosmologies x 300 per-cosmology redshifts: several tiles and a ragged tail."""
    params, z = workloads.config2(n_cosmo=37, n_z=300, seed=7)
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(z, dtype=dt, device=dev)
    zref = zt.double().cpu().numpy()
    for kind in KINDS:
        out, info = cosmo.cosmo_distance(kind, p, zt, info=True)
        ref = oracle.distance(kind, params, zref, shared_z=False)
        check(kind, dt, out.cpu().numpy(), ref, "config2-subset", params, zref)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_config4_families(dev, dt):
    """Near-degenerate cosmologies (near-flat, near-cubic, near-double root, near-EdS),
    z log-uniform on [1e-5, 1e3]."""
    params, z, fam = workloads.config4(n_per_family=8, n_z=700, seed=11)
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(z, dtype=dt, device=dev)
    zref = zt.double().cpu().numpy()
    for kind in KINDS:
        out = cosmo.cosmo_distance(kind, p, zt).cpu().numpy()
        ref = oracle.distance(kind, params, zref)
        for f in "ABCD":
            check(kind, dt, out[fam == f], ref[fam == f], f"config4-{f}", params[fam == f], zref)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_config2_full_size_sampled(dev, dt):
    params, z = workloads.config2()
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(z, dtype=dt, device=dev)
    ci, zi = workloads.subsample(params.shape[0], z.shape[1], 600)
    zs = zt.double().cpu().numpy()[ci, zi]
    for kind in ("DC", "DM", "T", "X"):
        out = cosmo.cosmo_distance(kind, p, zt)[ci, zi].cpu().numpy()
        ref = np.array([oracle.distance(kind, params[c:c + 1], np.array([zz]))[0, 0] for c, zz in zip(ci, zs)])
        check(kind, dt, out, ref, "config2-full-sampled",
              *(([params[ci], zs[:, None]]) if kind == "DM" else []))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_config5_full_size_sampled(dev, dt):
    params, z = workloads.config5()
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(z, dtype=dt, device=dev)
    mu = cosmo.cosmo_distance("MU", p, zt)
    assert mu.shape == (256, 10 ** 6)
    assert torch.isfinite(mu).all()
    ci, zi = workloads.subsample(256, 10 ** 6, 600)
    zs = zt.double().cpu().numpy()[zi]
    got = mu[ci, zi].double().cpu().numpy()
    ref = np.array([oracle.distance("MU", params[c:c + 1], np.array([zz]))[0, 0] for c, zz in zip(ci, zs)])
    check("MU", dt, got, ref, "config5-full-sampled")


def test_closed_forms_on_gpu(dev):
    """Einstein-de Sitter (cubic branch, triple root at x = 0) and the radiationless
    open matter universe (Mattig) through the full GPU path, FP64."""
    z = np.array([1e-5, 1e-3, 0.1, 0.5, 1.0, 2.0, 10.0, 100.0, 1000.0])
    zt = torch.tensor(z, dtype=torch.float64, device=dev)
    dh = 299792.458 / 70.0
    x = 1 + z
    p = torch.tensor([[70.0, 1.0, 0.0, 0.0]], dtype=torch.float64, device=dev)
    dc = cosmo.cosmo_distance("DC", p, zt)[0].cpu().numpy()
    assert np.max(np.abs(dc / (-2 * dh * np.expm1(-0.5 * np.log1p(z))) - 1)) < 1e-13
    xx = cosmo.cosmo_distance("X", p, zt)[0].cpu().numpy()
    assert np.max(np.abs(xx / ((2.0 / 3.0) * dh * np.expm1(1.5 * np.log1p(z))) - 1)) < 1e-12
    om = 0.3
    p = torch.tensor([[70.0, om, 0.0, 0.0]], dtype=torch.float64, device=dev)
    w2 = np.sqrt(1 + om * z)
    dm = dh * 2 * z * (1 + z / (1 + w2)) / ((1 + w2) * x)
    got = cosmo.cosmo_distance("DM", p, zt)[0].cpu().numpy()
    assert np.max(np.abs(got / dm - 1)) < 1e-12


def test_domain_flags_and_nan(dev):
    """No Big Bang (red region of Fig. 1), degree < 3, and a radiation-only universe
    outside the method: NaN outputs and the documented info bits."""
    params = np.array([[70.0, 0.05, 1.3, 0.0],      # two positive real roots: RED
                       [70.0, 0.0, 1.0, 0.0],       # de Sitter: degree 0
                       [70.0, 0.0, 0.0, 0.0],       # Milne: degree 2
                       [70.0, 0.3, 0.7, 0.0],       # fine
                       [-5.0, 0.3, 0.7, 0.0]])      # H0 <= 0
    p = torch.tensor(params, device=dev)
    zt = torch.tensor([0.5, 1.0], dtype=torch.float64, device=dev)
    out, info = cosmo.cosmo_distance("DC", p, zt, info=True)
    out = out.cpu().numpy()
    info = info.cpu().numpy()
    assert info[0] & cosmo.INFO["RED"] and np.all(np.isnan(out[0]))
    assert info[1] & cosmo.INFO["DOMAIN"] and np.all(np.isnan(out[1]))
    assert info[2] & cosmo.INFO["DOMAIN"] and np.all(np.isnan(out[2]))
    assert info[3] & cosmo.INFO["CUBIC"] and np.all(np.isfinite(out[3]))
    assert info[4] & cosmo.INFO["DOMAIN"] and np.all(np.isnan(out[4]))


def test_empty_and_tiny_inputs(dev):
    p = torch.tensor([[70.0, 0.3, 0.7, 9e-5]], dtype=torch.float64, device=dev)
    out = cosmo.cosmo_distance("DC", p, torch.empty(0, dtype=torch.float64, device=dev))
    assert out.shape == (1, 0)
    out = cosmo.cosmo_distance("DC", torch.empty((0, 4), dtype=torch.float64, device=dev),
                               torch.tensor([0.5], dtype=torch.float64, device=dev))
    assert out.shape == (0, 1)
    out = cosmo.cosmo_distance("DC", p, torch.tensor([0.0, 1e-12], dtype=torch.float64, device=dev)).cpu().numpy()
    assert out[0, 0] == 0.0 and abs(out[0, 1] / (299792.458 / 70 * 1e-12) - 1) < 1e-10


def test_determinism(dev):
    params, z = workloads.config2(n_cosmo=64, n_z=512, seed=3)
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(z, dtype=torch.float32, device=dev)
    a = cosmo.cosmo_distance("T", p, zt)
    b = cosmo.cosmo_distance("T", p, zt)
    assert torch.equal(a, b)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_config4_full_size_sampled(dev, dt):
    """1024 near-degenerate cosmologies x 4096 shared z on [1e-5, 1e3], sampled per family."""
    params, z, fam = workloads.config4()
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(z, dtype=dt, device=dev)
    zr = zt.double().cpu().numpy()
    ci, zi = workloads.subsample(params.shape[0], z.shape[0], 400, seed=404)
    for kind in ("DC", "DM", "T", "X", "MU"):
        out = cosmo.cosmo_distance(kind, p, zt)[ci, zi].double().cpu().numpy()
        ref = np.array([oracle.distance(kind, params[c:c + 1], np.array([zr[i]]))[0, 0] for c, i in zip(ci, zi)])
        for f in "ABCD":
            m = fam[ci] == f
            check(kind, dt, out[m][:, None], ref[m][:, None], f"config4-full-{f}", params[ci][m], zr[zi][m][:, None])


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_value_from_the_adjoint_pass(dev, dt):
    """cosmo_distance_vjp with an `out` buffer: the observable written by the adjoint
    kernel meets the forward bounds against the oracle, and the gradients equal those
    of the gradient-only call bit for bit (same lanes, same summation order)."""
    params, z = workloads.config2(n_cosmo=37, n_z=300, seed=7)
    params = np.concatenate([params, [[70.0, 0.05, 1.3, 0.0]]])  # a RED cosmology: NaN row
    p = torch.tensor(params, device=dev)
    zt = torch.tensor(np.concatenate([z, z[:1]]), dtype=dt, device=dev)
    zref = zt.double().cpu().numpy()
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    w = torch.randn(zt.shape, dtype=dt, device=dev, generator=gen)
    for kind in KINDS:
        val, gp, gz, info = cosmo.cosmo_distance_vjp(kind, p, zt, w, want_value=True, info=True)
        gp0, gz0 = cosmo.cosmo_distance_vjp(kind, p, zt, w)
        assert torch.equal(gp[:-1], gp0[:-1]) and torch.equal(gz[:-1], gz0[:-1]), kind
        v = val.cpu().numpy()
        assert np.all(np.isnan(v[-1])), kind
        ref = oracle.distance(kind, params[:-1], zref[:-1], shared_z=False)
        check(kind, dt, v[:-1], ref, "vjp-value", params[:-1], zref[:-1])
        if kind == "X":
            _, finfo = cosmo.cosmo_distance("X", p, zt, info=True)
            assert torch.equal(info, finfo)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_x_carlson_route_on_every_workload(dev, dt):
    """The absorption distance takes the Carlson route (eq. 3.9 in its regular
    arrangement, eq. B.3 without radiation) on workloads 1, 2, 4 and 5 at full size:
    the X_QUADRATURE bit is clear for every cosmology.  The matter-poor open cosmologies
    of workload 2 (Om0 < 0.06, OL0 < 0.15: a real root of Q near -15, terms cancelling by
    ~300 at z = 1e-3) are checked against the oracle on every one of their redshifts."""
    sets = []
    p1, z1 = workloads.config1()
    sets.append((p1, z1))
    p2, z2 = workloads.config2()
    sets.append((p2, z2))
    p4, z4, _ = workloads.config4()
    sets.append((p4, z4))
    p5, z5 = workloads.config5(n_z=2 ** 18)
    sets.append((p5, z5))
    for params, z in sets:
        p = torch.tensor(params, device=dev)
        zt = torch.tensor(z, dtype=dt, device=dev)
        _, info = cosmo.cosmo_distance("X", p, zt, info=True)
        flagged = int(((info & cosmo.INFO["X_QUADRATURE"]) != 0).sum())
        assert flagged == 0, (params.shape, z.shape, flagged)
    poor = np.where((p2[:, 1] < 0.06) & (p2[:, 2] < 0.15))[0]
    assert poor.size >= 4
    p = torch.tensor(p2[poor], device=dev)
    zt = torch.tensor(z2[poor], dtype=dt, device=dev)
    zref = zt.double().cpu().numpy()
    out = cosmo.cosmo_distance("X", p, zt).cpu().numpy()
    ref = oracle.distance("X", p2[poor], zref, shared_z=False)
    check("X", dt, out, ref, "config2-matter-poor")
