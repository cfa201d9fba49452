"""The device arithmetic (set-up: roots, root Jacobian, lane constants; per-lane
formulas of D_C, T and X in both precisions; the observables between two redshifts and
the Leibniz derivatives of the time coordinate) compiled for the host with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, no GPU code involved) and run
over cosmologies of every workload family: no sanitizer report (undefined behaviour
aborts the run), and the results equal those of the plain build bit for bit."""
import os
import subprocess

import numpy as np
import pytest

from paper_2212_01937_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host_shim", "sanitize_main.cpp")
BASE = ["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-I", os.path.join(HERE, "host_shim")]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def exes(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    plain, san = str(d / "plain"), str(d / "san")
    subprocess.run(BASE + [SRC, "-o", plain], check=True)
    subprocess.run(BASE + SAN + [SRC, "-o", san], check=True)
    return plain, san, d


def _input(path, params, z):
    with open(path, "wb") as f:
        np.array([params.shape[0], z.size], dtype=np.int64).tofile(f)
        np.ascontiguousarray(params, dtype=np.float64).tofile(f)
        np.ascontiguousarray(z, dtype=np.float64).tofile(f)


@pytest.mark.parametrize("name", ["config1", "config2", "config4", "config5", "edge"])
def test_sanitized_run_is_clean_and_equal(exes, name):
    plain, san, d = exes
    if name == "config1":
        p, z = workloads.config1()
        z = z[::20]
    elif name == "config2":
        p, z = workloads.config2(n_cosmo=12, n_z=40, seed=2)
        z = z[0]
    elif name == "config4":
        p, z, _ = workloads.config4(n_per_family=3, n_z=40, seed=2)
    elif name == "config5":
        p, z = workloads.config5(n_cosmo=6, n_z=40)
    else:
        # outside the method or at its edges: no Big Bang, degree < 3, H0 <= 0, NaN,
        # Einstein-de Sitter (triple root), a double root of the cubic (OL = 0)
        p = np.array([[70.0, 0.05, 1.3, 0.0], [70.0, 0.0, 1.0, 0.0], [70.0, 0.0, 0.0, 0.0], [-1.0, 0.3, 0.7, 0.0],
                      [70.0, np.nan, 0.7, 0.0], [70.0, 1.0, 0.0, 0.0], [70.0, 0.3, 0.0, 0.0],
                      [70.0, 0.3, 0.7, 1e-20]])
        z = np.array([0.0, 1e-7, 1e-3, 0.5, 3.0, 1e3])
    inp = str(d / f"{name}.in")
    _input(inp, p, z)
    outs = []
    for exe, tag in ((plain, "plain"), (san, "san")):
        o = str(d / f"{name}.{tag}.out")
        r = subprocess.run([exe, inp, o], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, (tag, r.returncode, r.stderr[-3000:])
        assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
        outs.append(np.fromfile(o, dtype=np.float64))
    a, b = outs
    assert a.size == b.size and a.size > 0
    assert np.array_equal(a, b, equal_nan=True)
