"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

Shared by the tests, the smoke check and the benchmark: both the HIP path and
the CPU oracle are fed from here.  Every generator is numpy PCG64 with the seed
193700 + k for workload k, so the same call returns the same arrays everywhere.

Parameter rows are (H0 [km/s/Mpc], Om0, OL0, Or0); Ok0 = 1 - Om0 - OL0 - Or0 is
implied (sec. 2.1 closure).  Redshifts are float64 here; callers cast.

Workloads (sizes are n_cosmo x n_z):
  1  flat LCDM+radiation, 1 x 1000, z on an even grid in [0.01, 2]
  2  non-flat batch, 4096 x 1024 per-cosmology log-uniform z in [1e-3, 10]
  3  mock SN Ia likelihood, 64 parameter samples x 1e6 SNe with p(z) ~ z^2 on [0.01, 1.5]
  4  near-degenerate stress set, 1024 x 4096 shared log-uniform z in [1e-5, 1e3]
  5  large batch, 256 x 1e6 shared z ~ U(0.01, 2.3)
Limit pairs for the observables between two redshifts (the cosmologies of 5):
  lensing_pairs  lens z1 ~ U(0.05, 1.5), source z2 = z1 + U(0.01, 2), shared
  age_redshifts  z ~ U(0, 20) for t(z, inf)
Supernova model of sec. 4 (mock catalogue):
  snia_mock      true z ~ Gamma(3, rate 3), standard-normal noise draws for zhat, muhat
"""
import numpy as np

SEED0 = 193700


def _rng(k, seed=None):
    return np.random.default_rng(np.random.PCG64(SEED0 + k if seed is None else seed))


def physical(params, zmax=None):
    """Domain screen used to reject draws: E^2(z) > 0 on the whole path [0, zmax]
    (zmax=None: up to the Big Bang).  A dense sampling check, not a root solve:
    E^2 is tabulated on a log grid and, beyond it, the leading positive term
    (radiation, else matter) guarantees positivity."""
    p = np.atleast_2d(np.asarray(params, dtype=np.float64))
    top = 1e6 if zmax is None else zmax
    z = np.concatenate([[0.0], np.geomspace(1e-6, top, 4000)])
    x = 1.0 + z[None, :]
    om, ol, orr = p[:, 1:2], p[:, 2:3], p[:, 3:4]
    ok = 1.0 - om - ol - orr
    e2 = orr * x ** 4 + om * x ** 3 + ok * x ** 2 + ol
    ok_path = np.all(e2 > 0, axis=1)
    if zmax is None:
        lead_ok = (p[:, 3] > 0) | ((p[:, 3] == 0) & (p[:, 1] > 0))
        ok_path &= lead_ok
    return ok_path


def config1():
    """One flat cosmology (H0=70, Om0=0.3, Or0=9e-5, OL0 = 1 - Om0 - Or0), 1000
    redshifts evenly spaced on [0.01, 2]."""
    params = np.array([[70.0, 0.3, 1.0 - 0.3 - 9e-5, 9e-5]])
    z = np.linspace(0.01, 2.0, 1000)
    return params, z


def config2(n_cosmo=4096, n_z=1024, seed=None):
    """Non-flat batch: Om0~U(0.05,0.6), OL0~U(0,1.2), Or0~U(0,1e-4), H0~U(60,80),
    drawn in that order per cosmology; draws without a Big Bang or with E^2 <= 0 on
    [0, 10] are redrawn.  Per-cosmology z: n_z log-uniform on [1e-3, 10], sorted.
    Returns params (n_cosmo, 4) and z (n_cosmo, n_z)."""
    rng = _rng(2, seed)
    rows = []
    while len(rows) < n_cosmo:
        om = rng.uniform(0.05, 0.6)
        ol = rng.uniform(0.0, 1.2)
        orr = rng.uniform(0.0, 1e-4)
        h0 = rng.uniform(60.0, 80.0)
        row = (h0, om, ol, orr)
        if physical(row)[0]:
            rows.append(row)
    params = np.array(rows)
    z = np.sort(10.0 ** rng.uniform(-3.0, 1.0, size=(n_cosmo, n_z)), axis=1)
    return params, z


def config3(n_sn=10 ** 6, n_samples=64, seed=None):
    """Mock SN Ia set: z_s with p(z) ~ z^2 on [0.01, 1.5] (inverse CDF), Gaussian
    magnitude noise N(0, 0.1^2) (to be added to the fiducial mu by the caller), and
    parameter samples (Om0, OL0, H0) ~ N((0.3, 0.7, 70), diag(0.05^2, 0.05^2, 2^2))
    with Or0 = 0, redrawn when unphysical.  Fiducial: (70, 0.3, 0.7, 0).
    Returns fiducial (1, 4), z (n_sn,), noise (n_sn,), params (n_samples, 4)."""
    rng = _rng(3, seed)
    u = rng.uniform(size=n_sn)
    lo, hi = 0.01, 1.5
    z = (lo ** 3 + u * (hi ** 3 - lo ** 3)) ** (1.0 / 3.0)
    noise = rng.normal(0.0, 0.1, size=n_sn)
    rows = []
    while len(rows) < n_samples:
        om, ol, h0 = rng.normal((0.3, 0.7, 70.0), (0.05, 0.05, 2.0))
        row = (h0, om, ol, 0.0)
        if om > 0 and physical(row)[0]:
            rows.append(row)
    fid = np.array([[70.0, 0.3, 0.7, 0.0]])
    return fid, z, noise, np.array(rows)


def config4(n_per_family=256, n_z=4096, seed=None):
    """Near-degenerate stress set in four families of n_per_family:
      A near-flat:  Om0~U(0.1,0.6), |Ok0| log-U[1e-9,1e-3] of random sign,
                    Or0~U(0,1e-8), OL0 closes the sum.
      B near-cubic: Om0~U(0.1,0.6), OL0~U(0.3,0.9), Or0 = 0 (a quarter of the
                    family) or log-U[1e-20,1e-8].
      C near-double root: E^2 in x=1+z built from prescribed roots: a pair
                    (rho, rho(1+d)), rho~U(0.05,0.9), d log-U[1e-9,1e-6], with
                    P(x) = Or0 (x^2 - s x + p)(x^2 + a x + b), no linear term
                    (p a = s b) and P(1) = 1; Or0~U(1e-12,1e-8).
      D near-EdS cluster: |Ok0| log-U[1e-9,1e-3] of random sign, OL0 =
                    2.5e-13 |Ok0| U(0,1), Or0~U(0,1e-8), Om0 closes the sum.
    H0~U(60,80).  Shared z: n_z log-uniform on [1e-5, 1e3], sorted.
    Returns params (4*n_per_family, 4), z (n_z,), family labels (array of 'A'..'D')."""
    rng = _rng(4, seed)
    n = n_per_family
    out, fam = [], []

    def h0():
        return rng.uniform(60.0, 80.0)

    def sign():
        return 1.0 if rng.uniform() < 0.5 else -1.0

    while len([f for f in fam if f == "A"]) < n:
        om = rng.uniform(0.1, 0.6)
        ok = sign() * 10.0 ** rng.uniform(-9, -3)
        orr = rng.uniform(0, 1e-8)
        row = (h0(), om, 1.0 - om - ok - orr, orr)
        if physical(row)[0]:
            out.append(row)
            fam.append("A")
    k = 0
    while len([f for f in fam if f == "B"]) < n:
        om = rng.uniform(0.1, 0.6)
        ol = rng.uniform(0.3, 0.9)
        orr = 0.0 if k % 4 == 0 else 10.0 ** rng.uniform(-20, -8)
        k += 1
        row = (h0(), om, ol, orr)
        if physical(row)[0]:
            out.append(row)
            fam.append("B")
    while len([f for f in fam if f == "C"]) < n:
        rho = rng.uniform(0.05, 0.9)
        d = 10.0 ** rng.uniform(-9, -6)
        orr = rng.uniform(1e-12, 1e-8)
        s = rho * (2.0 + d)
        p = rho * rho * (1.0 + d)
        # P(1) = Or (1 - s + p)(1 + a + b) = 1 with b = p a / s
        a = (1.0 / (orr * (1.0 - s + p)) - 1.0) / (1.0 + p / s)
        b = p * a / s
        om = orr * (a - s)
        ol = orr * p * b
        row = (h0(), om, ol, orr)
        if physical(row)[0]:
            out.append(row)
            fam.append("C")
    while len([f for f in fam if f == "D"]) < n:
        ok = sign() * 10.0 ** rng.uniform(-9, -3)
        ol = 2.5e-13 * abs(ok) * rng.uniform()
        orr = rng.uniform(0, 1e-8)
        row = (h0(), 1.0 - ok - ol - orr, ol, orr)
        if physical(row)[0]:
            out.append(row)
            fam.append("D")
    z = np.sort(10.0 ** rng.uniform(-5.0, 3.0, size=n_z))
    return np.array(out), z, np.array(fam)


def config5(n_cosmo=256, n_z=10 ** 6, seed=None):
    """Large batch: Om0~U(0.1,0.5), OL0~U(0.4,1.0), Or0 = 9e-5, H0~U(65,75);
    shared z: n_z ~ U(0.01, 2.3), sorted.  The cotangent weights of the headline
    fwd+grad step are drawn by the caller (on the device) from `cotangent_seed`."""
    rng = _rng(5, seed)
    rows = []
    while len(rows) < n_cosmo:
        om = rng.uniform(0.1, 0.5)
        ol = rng.uniform(0.4, 1.0)
        h0 = rng.uniform(65.0, 75.0)
        row = (h0, om, ol, 9e-5)
        if physical(row)[0]:
            rows.append(row)
    z = np.sort(rng.uniform(0.01, 2.3, size=n_z))
    return np.array(rows), z


def lensing_pairs(n=10 ** 6, seed=None):
    """Lens and source redshifts (z1, z2), z1 ~ U(0.05, 1.5), z2 = z1 + U(0.01, 2),
    float64, shared by all cosmologies (strong-lensing time-delay and D_A(z_l, z_s)
    geometry)."""
    rng = _rng(6, seed)
    z1 = rng.uniform(0.05, 1.5, n)
    z2 = z1 + rng.uniform(0.01, 2.0, n)
    return z1, z2


def age_redshifts(n=10 ** 6, seed=None):
    """Redshifts z ~ U(0, 20) (float64) for the age t(z, inf)."""
    return _rng(7, seed).uniform(0.0, 20.0, n)


def snia_mock(n=1000, seed=None):
    """Mock supernova catalogue draws for the model of sec. 4: true redshifts
    z ~ Gamma(shape 3, rate 3) and two standard-normal noise vectors; the caller forms
    zhat = z + (1 + z) sigma_z eps_z and muhat = mu(z; theta_true) + sigma_mu eps_mu.
    True cosmology (Om0, OL0) = (0.3, 0.7), Or0 = 0, H0 = 70.
    Returns z (n,), eps_z (n,), eps_mu (n,), theta_true (2,)."""
    rng = _rng(8, seed)
    z = rng.gamma(3.0, 1.0 / 3.0, n)
    return z, rng.standard_normal(n), rng.standard_normal(n), np.array([0.3, 0.7])


def cotangent_seed():
    return SEED0 + 50


def subsample(n_total_c, n_total_z, n, seed=SEED0 + 99):
    """Seeded (cosmology, z) index pairs for sampled checks at full size."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return rng.integers(0, n_total_c, n), rng.integers(0, n_total_z, n)
