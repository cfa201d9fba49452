"""The Gauss-Legendre tables compiled into the library (csrc/gl_tables.hpp): the file is
what its generator writes, and each rule integrates every polynomial of degree below
2n exactly (which fixes all of its nodes and weights), in the table's precision."""
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_01937_amd", "csrc")


def _table(name):
    text = open(os.path.join(CSRC, "gl_tables.hpp")).read()
    m = re.search(name + r"\[[^\]]*\] = \{([^}]*)\}", text)
    return np.array([float(v.rstrip("f")) for v in m.group(1).replace("\n", " ").split(",")])


def test_tables_are_the_generators_output():
    r = subprocess.run([sys.executable, os.path.join(CSRC, "gen_gl_tables.py"), "--check"], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_rules_integrate_polynomials_exactly():
    for n, sfx, tol in ((20, "64", 4e-16), (8, "32", 3e-7)):
        x, w = _table("c_gl" + sfx + "_x"), _table("c_gl" + sfx + "_w")
        assert x.size == n and w.size == n
        for k in range(2 * n):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            got = np.sum(w * x ** k)
            assert abs(got - exact) <= tol * 2 * max(1.0, k), (n, k, got, exact)
        # the degree-2n monomial is not integrated exactly: the n-point rule's error for
        # x^(2n) is 2^(2n+1) (n!)^4 / ((2n+1) ((2n)!)^2)
        from math import factorial
        e = 2.0 ** (2 * n + 1) * factorial(n) ** 4 / ((2 * n + 1) * factorial(2 * n) ** 2)
        got = 2.0 / (2 * n + 1) - np.sum(w * x ** (2 * n))
        assert abs(got / e - 1) < 3e-3, (n, got, e)
