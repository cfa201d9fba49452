"""C-ABI checks that need no GPU: the library loads, exports every function that
include/cosmo.h declares, and rejects bad arguments synchronously with the
documented status codes (no HIP call is made on these paths)."""
import ctypes
import os
import re

import pytest

from paper_2212_01937_amd import build, cosmo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if build.stale():
        build.build()
    return cosmo.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cosmo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "cosmo_distance" in names and "cosmo_distance_vjp" in names and "carlson_rj" in names
    assert set(names) == set(cosmo.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.cosmo_version().startswith(b"cosmo-carlson")


def test_argument_errors_are_synchronous(lib):
    E_ARG, E_KIND, E_DTYPE = -1, -2, -3
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced on these paths
    null = None
    # unknown kind / dtype
    assert lib.cosmo_distance(99, 1, dummy, 1, dummy, 1, 0, dummy, null, null, 0, null) == E_KIND
    assert lib.cosmo_distance(0, 7, dummy, 1, dummy, 1, 0, dummy, null, null, 0, null) == E_DTYPE
    assert lib.cosmo_distance_vjp(-1, 1, dummy, 1, dummy, 1, 0, dummy, null, null, null, null, null, 0, null) == E_KIND
    # NULL pointers and negative sizes
    assert lib.cosmo_distance(0, 1, null, 1, dummy, 1, 0, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance(0, 1, dummy, -1, dummy, 1, 0, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance(0, 1, dummy, 1, dummy, 1, -5, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance(0, 1, dummy, 1, null, 1, 0, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_vjp(0, 1, dummy, 1, dummy, 1, 0, null, dummy, null, null, null, null, 0, null) == E_ARG
    assert lib.cosmo_roots(null, 3, dummy, null, null) == E_ARG
    assert lib.cosmo_roots(dummy, -1, dummy, null, null) == E_ARG
    assert lib.carlson_rf(0, 4, dummy, dummy, null, dummy, null) == E_ARG
    assert lib.carlson_rj(1, 4, dummy, dummy, dummy, null, dummy, null) == E_ARG
    assert lib.carlson_rc(5, 4, dummy, dummy, dummy, null) == E_DTYPE
    # rows of 2^29 redshifts or more (32-bit byte offsets within a row in the kernels)
    big = 1 << 29
    assert lib.cosmo_distance(0, 1, dummy, 1, dummy, big, 0, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_vjp(3, 0, dummy, 1, dummy, big, 0, dummy, null, dummy, null, null, null, 0,
                                  null) == E_ARG
    assert lib.cosmo_distance_jac(3, 0, dummy, 1, dummy, big, 0, null, dummy, null, null, 0, null) == E_ARG
    # empty problems are valid no-ops
    assert lib.cosmo_roots(null, 0, null, null, null) == 0
    assert lib.carlson_rd(0, 0, null, null, null, null, null) == 0
    assert lib.cosmo_distance(0, 1, null, 0, null, 0, 0, null, null, null, 0, null) == 0


def test_workspace_size_monotone(lib):
    sz = [cosmo.workspace_size(nc, nz) for nc, nz in ((1, 1), (16, 1000), (256, 10 ** 6))]
    assert sz[0] > 0 and sz[0] <= sz[1] <= sz[2]
    b = ctypes.c_size_t(0)
    assert lib.cosmo_workspace_size(-1, 3, ctypes.byref(b)) == -1


def test_loglike_and_jacobian_argument_errors(lib):
    E_ARG, E_KIND = -1, -2
    dummy = ctypes.c_void_p(0x1000)
    null = None
    assert lib.cosmo_gaussian_loglike(42, 1, dummy, 1, dummy, 1, 0, dummy, dummy, null, null, null, null, null,
                                      null, 0, null) == E_KIND
    # missing observations / inverse variances
    assert lib.cosmo_gaussian_loglike(3, 1, dummy, 1, dummy, 1, 0, null, dummy, null, null, null, null, null,
                                      null, 0, null) == E_ARG
    assert lib.cosmo_gaussian_loglike(3, 1, dummy, 1, dummy, 1, 0, dummy, null, null, null, null, null, null,
                                      null, 0, null) == E_ARG
    # missing Jacobian buffer
    assert lib.cosmo_distance_jac(0, 1, dummy, 1, dummy, 1, 0, null, null, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_jac(0, 1, dummy, -1, dummy, 1, 0, null, dummy, null, null, 0, null) == E_ARG


def test_between_argument_errors(lib):
    E_ARG, E_KIND, E_DTYPE = -1, -2, -3
    dummy = ctypes.c_void_p(0x1000)
    null = None
    # kinds outside (DC, DM, DA, T): D_L, mu, X
    for k in (2, 3, 5, 17):
        assert lib.cosmo_distance_between(k, 1, dummy, 1, dummy, dummy, 1, 0, dummy, null, null, 0, null) == E_KIND
    assert lib.cosmo_distance_between(0, 4, dummy, 1, dummy, dummy, 1, 0, dummy, null, null, 0, null) == E_DTYPE
    # a missing limit or output, negative sizes
    assert lib.cosmo_distance_between(0, 1, dummy, 1, null, dummy, 1, 0, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_between(0, 1, dummy, 1, dummy, null, 1, 0, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_between(4, 1, dummy, 1, dummy, dummy, 1, 0, null, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_between(0, 1, dummy, 1, dummy, dummy, -3, 0, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_between(0, 1, dummy, 1, dummy, dummy, 1, -1, dummy, null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_between(6, 1, null, 0, null, null, 0, 0, null, null, null, 0, null) == 0


def test_binding_declares_every_argument(lib):
    """Every entry point of the binding has ctypes argument types, one per parameter
    of its declaration in include/cosmo.h (without them, 64-bit sizes and strides
    passed on the stack would be truncated to 32 bits with undefined upper halves)."""
    src = open(os.path.join(ROOT, "include", "cosmo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(([^)]*)\)\s*;", src, flags=re.M):
        name, params = m.group(1), m.group(2).strip()
        n_params = 0 if params in ("", "void") else params.count(",") + 1
        fn = getattr(lib, name)
        if n_params == 0:
            continue
        assert fn.argtypes is not None and len(fn.argtypes) == n_params, (name, n_params, fn.argtypes)


def test_between_vjp_argument_errors(lib):
    E_ARG, E_KIND = -1, -2
    dummy = ctypes.c_void_p(0x1000)
    null = None
    for k in (2, 3, 5, 7):  # DL, MU, X, VC
        assert lib.cosmo_distance_between_vjp(k, 1, dummy, 1, dummy, dummy, 1, 0, dummy, null, dummy, null, null,
                                              null, null, 0, null) == E_KIND
    # a missing cotangent or limit
    assert lib.cosmo_distance_between_vjp(0, 1, dummy, 1, dummy, dummy, 1, 0, null, null, dummy, null, null,
                                          null, null, 0, null) == E_ARG
    assert lib.cosmo_distance_between_vjp(0, 1, dummy, 1, null, dummy, 1, 0, dummy, null, dummy, null, null,
                                          null, null, 0, null) == E_ARG


def test_supernova_entry_points_argument_errors(lib):
    E_ARG, E_DTYPE = -1, -3
    d = ctypes.c_void_p(0x1000)
    assert lib.snia_draw(7, 1, 1, d, d, d, d, d, d, None) == E_DTYPE
    assert lib.snia_draw(0, -1, 1, d, d, d, d, d, d, None) == E_ARG
    assert lib.snia_draw(0, 2, 3, d, None, d, d, d, d, None) == E_ARG
    assert lib.snia_draw(0, 0, 3, None, None, None, None, None, None, None) == 0  # nothing to draw
    for sz, sh, rt in ((0.0, 3.0, 3.0), (0.04, 0.0, 3.0), (0.04, 3.0, -3.0), (float("inf"), 3.0, 3.0)):
        assert lib.snia_latent_vjp(0, 2, 3, d, d, d, d, d, d, None, sz, sh, rt, d, d, d, d, None, 0, None) == E_ARG
    assert lib.snia_latent_vjp(0, 2, 3, d, d, d, d, d, d, None, 0.04, 3.0, 3.0, None, d, d, d, None, 0, None) == E_ARG
    assert lib.snia_latent_vjp(0, 2, 3, d, d, d, d, d, d, None, 0.04, 3.0, 3.0, d, None, d, d, None, 0, None) == E_ARG
    nb = ctypes.c_size_t()
    assert lib.snia_workspace_size(4, 1000, ctypes.byref(nb)) == 0 and nb.value >= 8 * 4 * 9
    assert lib.snia_workspace_size(-1, 1000, ctypes.byref(nb)) == E_ARG
    assert lib.snia_workspace_size(4, 1000, None) == E_ARG


def test_noalloc_refuses_problems_beyond_its_array(lib):
    """cosmo_distance_vjp_noalloc checks the problem against its fixed device array on
    the host, before any HIP call (so these run without a GPU)."""
    E_ARG, E_KIND, E_SCRATCH = -1, -2, -6
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced on these paths
    null = None
    f = lib.cosmo_distance_vjp_noalloc
    assert f(42, 0, dummy, 1, dummy, 1, 0, dummy, null, dummy, dummy, null, null) == E_KIND
    assert f(3, 0, dummy, 1, dummy, 1, 0, null, null, dummy, dummy, null, null) == E_ARG
    assert f(3, 0, dummy, -1, dummy, 1, 0, dummy, null, dummy, dummy, null, null) == E_ARG
    # record table alone beyond the array (1e5 cosmologies, ~88 MB of records)
    assert f(3, 1, dummy, 100000, dummy, 1, 0, dummy, null, null, null, null, null) == E_SCRATCH
    # 256 cosmologies x 1e6 shared redshifts, FP64: the parameter partials fit (44 MB),
    # the 16 tile planes of the shared-z gradient (128 MB) do not
    assert f(3, 1, dummy, 256, dummy, 10 ** 6, 0, dummy, null, dummy, dummy, null, null) == E_SCRATCH
    # 4096 cosmologies x 65536 shared redshifts, FP32: 256 tile planes (67 MB)
    assert f(3, 0, dummy, 4096, dummy, 65536, 0, dummy, null, null, dummy, null, null) == E_SCRATCH
    assert cosmo.NOALLOC_SCRATCH_BYTES == 64 << 20
    src = open(os.path.join(ROOT, "include", "cosmo.h")).read()
    assert "#define COSMO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)" in src
