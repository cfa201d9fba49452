"""GPU unit parity of the Carlson entry points and the root finder."""
import numpy as np
import pytest
import torch

import oracle
from paper_2212_01937_amd import cosmo, workloads

pytestmark = pytest.mark.gpu


def _args(rng, n, pair):
    x = rng.uniform(0.05, 3, n) + 0j
    y = rng.uniform(-2, 3, n) + 1j * rng.uniform(0.05, 2, n)
    z = np.conj(y) if pair else rng.uniform(0.1, 3, n) + 1j * rng.uniform(-1, 1, n)
    p = rng.uniform(0.2, 3, n) + 1j * rng.uniform(-0.5, 0.5, n)
    return x, y, z, p


@pytest.mark.parametrize("cdt,tol", [(torch.complex128, 1e-13), (torch.complex64, 2e-6)])
def test_carlson_vs_oracle(dev, cdt, tol):
    rng = np.random.default_rng(1)
    for pair in (True, False):
        x, y, z, p = _args(rng, 120, pair)
        T = lambda a: torch.tensor(a, dtype=cdt, device=dev)
        for name, fn, args in (("RF", cosmo.carlson_rf, (x, y, z)), ("RD", cosmo.carlson_rd, (x, y, z)),
                               ("RJ", cosmo.carlson_rj, (x, y, z, p)), ("RC", cosmo.carlson_rc, (x, y))):
            got = fn(*[T(a) for a in args]).cpu().numpy().astype(np.complex128)
            if cdt == torch.complex64:  # the oracle sees the rounded arguments
                args = [np.asarray(a, dtype=np.complex64).astype(np.complex128) for a in args]
            ref = oracle.carlson(name, *args)
            err = np.max(np.abs(got - ref) / np.abs(ref))
            assert err < tol, (name, pair, cdt, err)


def test_carlson_invariants_and_principal_value(dev):
    v = torch.tensor([0.37, 2.5, 1.2 + 0.7j], dtype=torch.complex128, device=dev)
    assert torch.allclose(cosmo.carlson_rf(v, v, v), v ** -0.5, rtol=1e-14)
    assert torch.allclose(cosmo.carlson_rd(v, v, v), v ** -1.5, rtol=1e-14)
    assert torch.allclose(cosmo.carlson_rj(v, v, v, v), v ** -1.5, rtol=1e-14)
    # R_C(x, y) for y < 0: Cauchy principal value (closed form, DLMF 19.2.20/19.2.19)
    x = torch.tensor([0.5, 2.0], dtype=torch.complex128, device=dev)
    y = torch.tensor([-1.0, -0.25], dtype=torch.complex128, device=dev)
    got = cosmo.carlson_rc(x, y).real.cpu().numpy()
    xr, yr = np.array([0.5, 2.0]), np.array([-1.0, -0.25])
    ref = np.sqrt(xr / (xr - yr)) * np.arccosh(np.sqrt((xr - yr) / (-yr))) / np.sqrt(xr)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-13


def test_roots_vs_oracle_and_backward_error(dev):
    p2, _ = workloads.config2(n_cosmo=96, n_z=2, seed=5)
    p4, _, fam = workloads.config4(n_per_family=16, n_z=2, seed=5)
    params = np.concatenate([p2, p4, [[70.0, 0.3, 0.7, 0.0], [70.0, 1.0, 0.0, 0.0]]])
    r, info = cosmo.cosmo_roots(torch.tensor(params, device=dev))
    r = r.cpu().numpy()
    info = info.cpu().numpy()
    ref = oracle.roots(params)
    for i, (pp, rr, rf) in enumerate(zip(params, r, ref)):
        _, om, ol, orr = pp
        ok = 1 - om - ol - orr
        if orr > 0:
            got = rr + 1.0
            want = np.array([orr, om, ok, 0.0, ol])
            recon = orr * np.poly(got)
            # backward error of the factorisation: coefficients reproduced to ~eps
            scale = np.max(np.abs(want))
            assert np.max(np.abs(recon.real - want)) < 1e-12 * scale, i
        else:
            got = rr[:3] + 1.0
            want = np.array([om, ok, 0.0, ol])
            recon = om * np.poly(got)
            assert np.max(np.abs(recon.real - want)) < 1e-13 * np.max(np.abs(want)), i
        # and the roots themselves match the oracle's up to the conditioning of each root
        gr = np.sort_complex(np.round(rr[np.isfinite(rr)], 12))
        fr = np.sort_complex(np.round(rf[np.isfinite(rf)], 12))
        assert len(gr) == len(fr)
        sep = info[i] & cosmo.INFO["NEAR_MULTIROOT"]
        tol = 1e-6 if sep else 1e-9
        assert np.max(np.abs(gr - fr) / np.maximum(1, np.abs(fr))) < tol, (i, gr, fr)
    assert np.all(info[:96] & cosmo.INFO["QUARTIC"])
    assert info[-1] & cosmo.INFO["CUBIC"]
