"""Writes gl_tables.hpp: the Gauss-Legendre nodes and weights of the quadrature routes
(20 nodes in FP64, 8 nodes in FP32, on [-1, 1]) as literal constant arrays, so that the
library needs no run-time initialisation.

    python paper_2212_01937_amd/csrc/gen_gl_tables.py [--check]

Nodes are the zeros of the Legendre polynomial P_n, found by Newton's method at 50
significant digits (mpmath); weights 2 / ((1 - x^2) P_n'(x)^2).  Each value is rounded
once to the table's type.  --check compares the file on disk with what would be written.
"""
import os
import sys

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "gl_tables.hpp")
N64, N32 = 20, 8


def legendre_rule(n):
    mp.mp.dps = 50
    xs, ws = [], []
    for i in range(n):
        t = mp.cos(mp.pi * (i + mp.mpf(3) / 4) / (n + mp.mpf(1) / 2))
        for _ in range(100):
            p0, p1 = mp.mpf(1), t
            for k in range(2, n + 1):
                p0, p1 = p1, ((2 * k - 1) * t * p1 - (k - 1) * p0) / k
            dp = n * (t * p1 - p0) / (t * t - 1)
            dt = p1 / dp
            t -= dt
            if abs(dt) < mp.mpf(10) ** -45:
                break
        p0, p1 = mp.mpf(1), t
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * t * p1 - (k - 1) * p0) / k
        dp = n * (t * p1 - p0) / (t * t - 1)
        xs.append(t)
        ws.append(2 / ((1 - t * t) * dp * dp))
    return xs, ws


def _fmt64(v):
    return repr(float(v))


def _fmt32(v):
    # the float nearest to v (rounding through a double first could round twice)
    f = np.float32(float(v))
    cands = [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
    f = min(cands, key=lambda c: abs(mp.mpf(float(c)) - v))
    s = np.format_float_scientific(f, unique=True)
    return s + "f"


def render():
    x64, w64 = legendre_rule(N64)
    x32, w32 = legendre_rule(N32)
    lines = [
        "// gl_tables.hpp -- written by gen_gl_tables.py; do not edit.",
        "// Gauss-Legendre nodes x_i and weights w_i on [-1, 1] (zeros of the Legendre",
        "// polynomial by Newton's method at 50 digits, each value rounded once).",
        "#pragma once",
        "",
        "namespace cosmo {",
        "",
        f"constexpr int kGlN64 = {N64}; // nodes per panel, FP64",
        f"constexpr int kGlN32 = {N32};  // nodes per panel, FP32",
        "",
    ]
    for name, vals, fmt in (("c_gl64_x", x64, _fmt64), ("c_gl64_w", w64, _fmt64),
                            ("c_gl32_x", x32, _fmt32), ("c_gl32_w", w32, _fmt32)):
        ty = "double" if "64" in name else "float"
        n = "kGlN64" if "64" in name else "kGlN32"
        body = ",\n    ".join(", ".join(fmt(v) for v in vals[i:i + 4]) for i in range(0, len(vals), 4))
        lines.append(f"__constant__ const {ty} {name}[{n}] = {{\n    {body}}};")
    lines += ["", "} // namespace cosmo", ""]
    return "\n".join(lines)


if __name__ == "__main__":
    text = render()
    if "--check" in sys.argv:
        ok = os.path.exists(OUT) and open(OUT).read() == text
        print("gl_tables.hpp is current" if ok else "gl_tables.hpp differs from the generator's output")
        sys.exit(0 if ok else 1)
    with open(OUT, "w") as f:
        f.write(text)
    print(OUT)
