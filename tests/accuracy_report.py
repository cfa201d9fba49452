"""Accuracy report (run by hand on a GPU machine; not collected by pytest): the
maximum and median errors of every output against the oracle on each workload,
for the FP64 and the FP32 path.

    python tests/accuracy_report.py [--out report.md] [--skip-widened | --only-widened]

Relative errors for D_C, T, X; D_M relative to its conditioning scale (it crosses
zero beyond the antipode of a closed universe); mu in magnitudes, per the same
conditioning.  Workloads 1, 2 and 4 in full; the large workloads 3 and 5 on 1e6
seeded (cosmology, z) pairs of the full-size launch.  For the FP32 path the oracle is evaluated at the redshifts
rounded to FP32 (the errors are those of the path, not of the input rounding).
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

import oracle  # noqa: E402
from paper_2212_01937_amd import cosmo, workloads  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_forward import cond_scale  # noqa: E402

KINDS = ["DC", "DM", "T", "X", "MU"]


def errors(kind, got, ref, finite_ref, params=None, z=None):
    """Relative error (D_C, T, X), for D_M relative to the conditioning scale |D_M| +
    |dD_M/dchi| chi (D_M crosses zero beyond the antipode of a closed universe, where a
    relative error of chi moves it by that much), and for mu in mag, divided by
    max(1, |C chi / S|): the absolute error in magnitudes wherever a relative error of
    chi moves D_L by no more than itself (flat and closed universes before the antipode),
    and beyond that the error relative to the amplification of chi's error."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if kind in ("DM", "MU"):
        with np.errstate(invalid="ignore"):
            e = np.abs(got - ref) / cond_scale(kind, params, z, ref)
    else:
        e = np.abs(got - ref) / np.abs(ref)
    return e[finite_ref]


def full(label, params, z, shared, dev, rows):
    p = torch.tensor(params, device=dev)
    for dt, name in ((torch.float64, "FP64"), (torch.float32, "FP32")):
        zt = torch.tensor(z, dtype=dt, device=dev)
        zr = zt.double().cpu().numpy()
        cells = []
        for kind in KINDS:
            out = cosmo.cosmo_distance(kind, p, zt).double().cpu().numpy()
            ref = oracle.distance(kind, params, zr, shared_z=shared)
            fin = np.isfinite(ref)
            e = errors(kind, out, ref, fin, params, zr)
            cells.append((e.max(), np.median(e)))
        rows.append((label, name, int(np.prod(out.shape)), cells))
        print(label, name, cells, flush=True)


def sampled(label, params, z, dev, rows, n=10 ** 6, seed=31):
    p = torch.tensor(params, device=dev)
    ci, zi = workloads.subsample(params.shape[0], z.shape[0], n, seed=seed)
    order = np.argsort(ci, kind="stable")
    ci, zi = ci[order], zi[order]
    for dt, name in ((torch.float64, "FP64"), (torch.float32, "FP32")):
        zt = torch.tensor(z, dtype=dt, device=dev)
        zr = zt.double().cpu().numpy()
        cells = []
        for kind in KINDS:
            out = cosmo.cosmo_distance(kind, p, zt)
            got = out[torch.tensor(ci, device=dev), torch.tensor(zi, device=dev)].double().cpu().numpy()
            del out
            ref = np.empty(n)
            for c in np.unique(ci):
                m = ci == c
                ref[m] = oracle.distance(kind, params[c:c + 1], zr[zi[m]])[0]
            fin = np.isfinite(ref)
            e = errors(kind, got, ref, fin, params[ci], zr[zi][:, None])
            cells.append((e.max(), np.median(e)))
        rows.append((label + f" ({n} sampled pairs)", name, n, cells))
        print(label, name, cells, flush=True)


def sample_sorted(n_c, n_z, n, seed):
    ci, zi = workloads.subsample(n_c, n_z, n, seed=seed)
    order = np.argsort(ci, kind="stable")
    return ci[order], zi[order]


def widened(dev, rows, n=10 ** 6):
    """Observables between two redshifts (the lens-source pairs and the age t(z, inf)
    on the large batch's cosmologies) and the comoving volume (the large batch), on
    seeded sampled outputs of the full-size launch."""
    params, zv = workloads.config5()
    z1, z2 = workloads.lensing_pairs()
    zage = workloads.age_redshifts()
    p = torch.tensor(params, device=dev)
    cases = (("chi(z_l, z_s)", "DC", z1, z2), ("D_A(z_l, z_s)", "DA", z1, z2),
             ("t(z, inf)", "T", zage, np.full_like(zage, np.inf)))
    for label, kind, a, b in cases:
        ci, zi = sample_sorted(params.shape[0], a.size, n, 41)
        for dt, name in ((torch.float64, "FP64"), (torch.float32, "FP32")):
            ta, tb = torch.tensor(a, dtype=dt, device=dev), torch.tensor(b, dtype=dt, device=dev)
            out = cosmo.cosmo_distance_between(kind, p, ta, tb)
            got = out[torch.tensor(ci, device=dev), torch.tensor(zi, device=dev)].double().cpu().numpy()
            del out
            ar, br = ta.double().cpu().numpy()[zi], tb.double().cpu().numpy()[zi]
            ref = np.empty(n)
            for c in np.unique(ci):
                m = ci == c
                ref[m] = oracle.between(kind, params[c:c + 1], ar[m], br[m])[0]
            scale = np.abs(ref)
            if kind == "DA":
                chi = np.empty(n)
                for c in np.unique(ci):
                    m = ci == c
                    chi[m] = oracle.between("DC", params[c:c + 1], ar[m], br[m])[0]
                dh = 299792.458 / params[ci, 0]
                ok = 1 - params[ci, 1:].sum(1)
                x = np.sqrt(np.abs(ok)) * chi / dh
                cc = np.where(ok < 0, np.cos(x), np.where(ok > 0, np.cosh(x), 1.0))
                scale = scale + np.abs(cc * chi / (1 + br))
            e = np.abs(got - ref) / scale
            rows.append((f"{label}, 256 x 1e6 shared pairs ({n} sampled)", name, n, (e.max(), np.median(e))))
            print(label, name, e.max(), np.median(e), flush=True)
    nv = n // 10
    ci, zi = sample_sorted(params.shape[0], zv.size, nv, 43)
    for dt, name in ((torch.float64, "FP64"), (torch.float32, "FP32")):
        zt = torch.tensor(zv, dtype=dt, device=dev)
        out = cosmo.cosmo_distance("VC", p, zt)
        got = out[torch.tensor(ci, device=dev), torch.tensor(zi, device=dev)].double().cpu().numpy()
        del out
        zr = zt.double().cpu().numpy()[zi]
        ref = np.empty(nv)
        scale = np.empty(nv)
        for c in np.unique(ci):
            m = ci == c
            ref[m] = oracle.distance("VC", params[c:c + 1], zr[m])[0]
            scale[m] = cond_scale("VC", params[c:c + 1], zr[m], ref[m])
        e = np.abs(got - ref) / scale
        rows.append((f"V_C(z), 256 x 1e6 ({nv} sampled)", name, nv, (e.max(), np.median(e))))
        print("VC", name, e.max(), np.median(e), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--skip-widened", action="store_true", help="skip the between-redshift and volume rows")
    ap.add_argument("--only-widened", action="store_true", help="only the between-redshift and volume rows")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    rows = []
    t0 = time.time()
    if not args.only_widened:
        p1, z1 = workloads.config1()
        full("1: flat LCDM+radiation, 1 x 1000", p1, z1, True, dev, rows)
        p2, z2 = workloads.config2()
        full("2: non-flat, 4096 x 1024", p2, z2, False, dev, rows)
        p4, z4, _ = workloads.config4()
        full("4: near-degenerate, 1024 x 4096", p4, z4, True, dev, rows)
        _, z3, _, th3 = workloads.config3()
        sampled("3: SN likelihood cosmologies, 64 x 1e6", th3, z3, dev, rows)
        p5, z5 = workloads.config5()
        sampled("5: large batch, 256 x 1e6", p5, z5, dev, rows)
    wide = []
    if not args.skip_widened:
        widened(dev, wide)
    lines = ["| workload | path | evals | " + " | ".join(f"{k} max / median" for k in KINDS) + " |",
             "|---|---|---|" + "---|" * len(KINDS)]
    for label, name, n, cells in rows:
        lines.append(f"| {label} | {name} | {n} | " + " | ".join(f"{a:.1e} / {b:.1e}" for a, b in cells) + " |")
    if wide:
        lines += ["", "| widened row | path | evals | max / median |", "|---|---|---|---|"]
        for label, name, n, (a, b) in wide:
            lines.append(f"| {label} | {name} | {n} | {a:.1e} / {b:.1e} |")
    text = "\n".join(lines) + (f"\n\n(relative errors; D_M relative to |D_M| + |dD_M/dchi| chi, D_A(z_l, z_s) to "
                                f"|D_A| + |C chi/(1 + z_s)|, V_C to max(|V_C|, chi dV_C/dchi); MU in mag, divided "
                                f"by max(1, |C chi / S|); {time.time() - t0:.0f} s)\n")
    print(text)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)


if __name__ == "__main__":
    main()
