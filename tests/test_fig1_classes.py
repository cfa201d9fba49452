"""The root classes of Fig. 1 (sec. 3: the physical-domain condition), as the set-up
of the HIP path reports them in the info word, checked without a GPU on a host build
of csrc/setup.hpp against the oracle's 50-digit roots of E^2 over a grid of (Om0, OL0)
at several Or0:
  RED         a real root x = 1 + z >= 1 of E^2 on the integration path (no Big Bang);
  YELLOW      a complex pair of the cubic factor with Re(r) > 0, i.e. Re(x) > 1;
  THREE_REAL  the cubic factor (E^2 without the radiation root) has three real roots;
  DOMAIN      with Or0 > 0, no negative real root to serve as the radiation root;
and ROOT_NOCONV (a root iteration that hit its cap) is set on no cosmology of any of
the workloads.  Grid points within 1e-9 of a class boundary (a root's imaginary part
or its distance from x = 1) are skipped: there the class is decided by rounding."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2212_01937_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
INFO = {"THREE_REAL": 0x4, "YELLOW": 0x8, "RED": 0x10, "DOMAIN": 0x20, "ROOT_NOCONV": 0x40}


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("fig1") / "libsetup_host.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=fast", "-I",
                    os.path.join(HERE, "host_shim"), os.path.join(HERE, "host_shim", "setup_host.cpp"), "-o", out],
                   check=True)
    return ctypes.CDLL(out)


def info_of(lib, params):
    p = np.ascontiguousarray(params, dtype=np.float64)
    n = p.shape[0]
    out = np.zeros((n, 12))
    info = np.zeros(n, np.int32)
    lib.host_setup(p.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(n), out.ctypes.data_as(ctypes.c_void_p),
                   info.ctypes.data_as(ctypes.c_void_p))
    return info


def oracle_class(row, r):
    """Expected bits from the oracle's z-roots r (NaN slot when cubic); None where a
    class boundary is within rounding."""
    orr = row[3]
    x = r[np.isfinite(r)] + 1.0
    eps = 1e-9
    if orr > 0:
        neg = [v for v in x if abs(v.imag) <= eps * max(1.0, abs(v)) and v.real < 0]
        if not neg:
            return INFO["DOMAIN"]
        rad = min(neg, key=lambda v: v.real)  # largest modulus among the negative reals
        k = int(np.argmin(np.abs(x - rad)))
        cub = np.delete(x, k)
    else:
        cub = x
    im = np.abs(cub.imag)
    if np.any((im > 0) & (im <= eps * np.maximum(1.0, np.abs(cub)))):
        return None  # a pair about to become two real roots
    real = cub[im == 0].real if np.any(im == 0) else cub[im <= eps].real
    cplx = cub[im > eps]
    if np.any(np.abs(cub.real - 1.0) <= eps):
        return None
    bits = 0
    if len(cplx) == 0:
        bits |= INFO["THREE_REAL"]
    if np.any(real >= 1.0):
        bits |= INFO["RED"]
    if len(cplx) and np.any(cplx.real > 1.0):
        bits |= INFO["YELLOW"]
    return bits


@pytest.mark.parametrize("orr", [0.0, 1e-8, 1e-5, 1e-4])
def test_classes_on_a_grid(lib, orr):
    om, ol = np.meshgrid(np.linspace(0.02, 1.6, 23), np.linspace(-0.4, 2.6, 23))
    params = np.stack([np.full(om.size, 70.0), om.ravel(), ol.ravel(), np.full(om.size, orr)], 1)
    info = info_of(lib, params)
    roots = oracle.roots(params)
    mask = INFO["THREE_REAL"] | INFO["YELLOW"] | INFO["RED"] | INFO["DOMAIN"]
    seen = {}
    checked = 0
    for row, r, got in zip(params, roots, info):
        want = oracle_class(row, r)
        if want is None:
            continue
        checked += 1
        if want & INFO["DOMAIN"]:
            assert got & INFO["DOMAIN"], (row, r, got)
            continue
        assert not (got & INFO["ROOT_NOCONV"]), row
        assert (got & mask) == want, (row, r, hex(got), hex(want))
        seen[want] = seen.get(want, 0) + 1
    assert checked > 0.9 * params.shape[0]
    # the grid reaches the green, yellow and red regions and both structures of the cubic
    assert any(not (b & (INFO["RED"] | INFO["YELLOW"])) for b in seen)
    assert any(b & INFO["YELLOW"] for b in seen) and any(b & INFO["RED"] for b in seen)
    assert any(b & INFO["THREE_REAL"] for b in seen)


def test_no_root_iteration_hits_its_cap(lib):
    sets = [workloads.config1()[0], workloads.config2(n_z=2)[0], workloads.config3(n_sn=4)[3],
            workloads.config4(n_z=2)[0], workloads.config5(n_z=2)[0]]
    for p in sets:
        info = info_of(lib, p)
        assert not np.any(info & INFO["ROOT_NOCONV"])
        assert not np.any(info & (INFO["RED"] | INFO["DOMAIN"]))
