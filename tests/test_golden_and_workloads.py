"""The golden fixture stays what the oracle writes, and the seeded generators are
deterministic and produce physical cosmologies of the stated shapes."""
import os

import numpy as np

import oracle
from paper_2212_01937_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def test_golden_config1_reproduced_by_oracle():
    g = np.loadtxt(os.path.join(HERE, "golden", "config1_oracle.txt"))
    params, z = workloads.config1()
    assert np.array_equal(g[:, 0], z)
    assert np.allclose(oracle.distance("DC", params, z)[0], g[:, 1], rtol=1e-15, atol=0)
    assert np.allclose(oracle.distance("DL", params, z)[0], g[:, 2], rtol=1e-15, atol=0)
    assert np.allclose(oracle.distance("MU", params, z)[0], g[:, 3], rtol=0, atol=1e-13)


def test_generators_deterministic_and_physical():
    p1, z1 = workloads.config2(n_cosmo=64, n_z=32)
    p2, z2 = workloads.config2(n_cosmo=64, n_z=32)
    assert np.array_equal(p1, p2) and np.array_equal(z1, z2)
    assert z1.shape == (64, 32) and np.all(np.diff(z1, axis=1) >= 0)
    assert np.all(workloads.physical(p1))
    p, z, fam = workloads.config4(n_per_family=16, n_z=64)
    assert p.shape == (64, 4) and z.shape == (64,)
    assert np.all(workloads.physical(p))
    assert sorted(set(fam)) == ["A", "B", "C", "D"]
    # family C really has a root pair within 1e-6 (relative) of each other
    r = oracle.roots(p[fam == "C"][:4]) + 1.0
    for rr in r:
        small = rr[np.argsort(np.abs(rr))][:3]
        d = min(abs(small[i] - small[j]) / abs(small[i]) for i in range(3) for j in range(i + 1, 3))
        assert d < 2e-6
    fid, zs, noise, th = workloads.config3(n_sn=1000, n_samples=8)
    assert zs.min() >= 0.01 and zs.max() <= 1.5 and th.shape == (8, 4) and np.all(th[:, 3] == 0)
    p5, z5 = workloads.config5(n_cosmo=8, n_z=100)
    assert np.all(p5[:, 3] == 9e-5) and np.all(np.diff(z5) >= 0)
