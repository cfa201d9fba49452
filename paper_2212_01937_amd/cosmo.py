"""ctypes binding of libcosmo.so -- the C ABI of include/cosmo.h -- on torch tensors.

Argument marshalling only: every step of the computation runs in the HIP
kernels of csrc/.  Entry points keep the C names (cosmo_roots, carlson_rf,
carlson_rd, carlson_rj, carlson_rc, cosmo_distance, cosmo_distance_vjp, cosmo_distance_jac);
`distance` wraps the forward/adjoint pair in a torch.autograd.Function.

Device tensors are passed as raw pointers together with the current torch
stream, so calls are stream-ordered with surrounding torch work.  There is no
CPU implementation behind these functions: if the shared library is missing or
no GPU is visible they raise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcosmo.so")

KINDS = {"DC": 0, "DM": 1, "DL": 2, "MU": 3, "T": 4, "X": 5, "DA": 6, "VC": 7}
DTYPES = {torch.float32: 0, torch.float64: 1}
STATUS = {0: "COSMO_OK", -1: "COSMO_E_ARG", -2: "COSMO_E_KIND", -3: "COSMO_E_DTYPE",
          -4: "COSMO_E_HIP", -5: "COSMO_E_WORKSPACE", -6: "COSMO_E_SCRATCH"}
NOALLOC_SCRATCH_BYTES = 64 << 20  # COSMO_NOALLOC_SCRATCH_BYTES
INFO = {"CUBIC": 0x1, "QUARTIC": 0x2, "THREE_REAL": 0x4, "YELLOW": 0x8, "RED": 0x10,
        "DOMAIN": 0x20, "ROOT_NOCONV": 0x40, "NEAR_MULTIROOT": 0x80, "X_QUADRATURE": 0x100,
        "NEAR_MULTIROOT_F32": 0x200}

# every function declared in include/cosmo.h
EXPORTS = ("cosmo_workspace_size", "cosmo_roots", "carlson_rf", "carlson_rd", "carlson_rj",
           "carlson_rc", "cosmo_distance", "cosmo_distance_between", "cosmo_distance_between_vjp",
           "cosmo_distance_vjp", "cosmo_distance_vjp_noalloc", "cosmo_distance_jac", "cosmo_route_counts",
           "cosmo_gaussian_loglike", "snia_draw", "snia_latent_vjp", "snia_workspace_size", "cosmo_version")

_lib = None


class CosmoError(RuntimeError):
    pass


def load():
    """Load libcosmo.so (built by paper_2212_01937_amd.build).  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CosmoError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_01937_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32p = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
    lib.cosmo_workspace_size.argtypes = [i64, i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.cosmo_roots.argtypes = [vp, i64, vp, i32p, vp]
    for n in ("carlson_rf", "carlson_rd"):
        getattr(lib, n).argtypes = [ctypes.c_int, i64, vp, vp, vp, vp, vp]
    lib.carlson_rj.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp, vp, vp]
    lib.carlson_rc.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp]
    lib.cosmo_distance.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, vp, i64, i64, vp, i32p, vp,
                                   ctypes.c_size_t, vp]
    lib.cosmo_distance_between.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, vp, vp, i64, i64, vp, i32p, vp,
                                           ctypes.c_size_t, vp]
    lib.cosmo_distance_between_vjp.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, vp, vp, i64, i64, vp, vp, vp,
                                               vp, vp, i32p, vp, ctypes.c_size_t, vp]
    lib.cosmo_distance_vjp.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, vp, i64, i64, vp, vp, vp, vp,
                                       i32p, vp, ctypes.c_size_t, vp]
    lib.cosmo_distance_vjp_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, vp, i64, i64, vp, vp, vp, vp,
                                               i32p, vp]
    lib.cosmo_route_counts.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, vp, i64, i64, vp, vp, ctypes.c_size_t, vp]
    lib.cosmo_distance_jac.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, vp, i64, i64, vp, vp, i32p, vp,
                                       ctypes.c_size_t, vp]
    lib.cosmo_gaussian_loglike.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, vp, i64, i64, vp, vp, vp, vp, vp,
                                           vp, i32p, vp, ctypes.c_size_t, vp]
    f64 = ctypes.c_double
    lib.snia_draw.argtypes = [ctypes.c_int, i64, i64, vp, vp, vp, vp, vp, vp, vp]
    lib.snia_latent_vjp.argtypes = [ctypes.c_int, i64, i64, vp, vp, vp, vp, vp, vp, vp, f64, f64, f64, vp, vp, vp,
                                    vp, vp, ctypes.c_size_t, vp]
    lib.snia_workspace_size.argtypes = [i64, i64, ctypes.POINTER(ctypes.c_size_t)]
    for n in EXPORTS[:-1]:
        getattr(lib, n).restype = ctypes.c_int
    lib.cosmo_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc, what):
    if rc != 0:
        raise CosmoError(f"{what} failed: {STATUS.get(rc, rc)}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _need_gpu(t, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise CosmoError(f"{name} must be a CUDA (HIP) tensor; this library has no CPU path")


def _params(params):
    _need_gpu(params, "params")
    if params.dtype != torch.float64:
        raise CosmoError("params must be float64 (H0, Om0, OL0, Or0) rows")
    p = params.reshape(-1, 4)
    return p if p.is_contiguous() else p.contiguous()


def _z_layout(z, n_cosmo):
    """Returns (z_contig, n_z, stride, shared).  A 2-D z is passed to the library as
    dense rows (stride n_z): the per-element inputs the library reads with z's stride
    (observed values, inverse variances) are packed that way, and a stride of 0 would
    mean a shared row to the library.  Views that are not dense rows (column slices,
    expanded rows) are copied."""
    _need_gpu(z, "z")
    if z.dtype not in DTYPES:
        raise CosmoError("z must be float32 or float64")
    if z.dim() == 1:
        zc = z if z.is_contiguous() else z.contiguous()
        return zc, zc.shape[0], 0, True
    if z.dim() == 2 and z.shape[0] == n_cosmo:
        n_z = z.shape[1]
        dense = z.stride(1) == 1 and (z.stride(0) == n_z or n_cosmo <= 1)
        zc = z if dense else z.contiguous()
        return zc, n_z, n_z, False
    raise CosmoError("z must be [n_z] (shared) or [n_cosmo, n_z]")


def workspace_size(n_cosmo, n_z):
    lib = load()
    b = ctypes.c_size_t(0)
    _check(lib.cosmo_workspace_size(int(n_cosmo), int(n_z), ctypes.byref(b)), "cosmo_workspace_size")
    return int(b.value)


def _workspace(n_cosmo, n_z, dev):
    return torch.empty(max(workspace_size(n_cosmo, n_z), 1), dtype=torch.uint8, device=dev)


def cosmo_roots(params, with_info=True):
    """Roots of E^2(z) per cosmology: complex128 [n, 4] (slot 3: radiation root, NaN if
    Or0 == 0) and int32 info flags."""
    lib = load()
    p = _params(params)
    n = p.shape[0]
    out = torch.empty((n, 4, 2), dtype=torch.float64, device=p.device)
    info = torch.empty(n, dtype=torch.int32, device=p.device)
    with torch.cuda.device(p.device):
        _check(lib.cosmo_roots(_ptr(p), n, _ptr(out), _ptr(info), _stream(p.device)), "cosmo_roots")
    r = torch.view_as_complex(out)
    return (r, info) if with_info else r


def _carlson(name, args):
    lib = load()
    dev = args[0].device
    cdt = args[0].dtype
    if cdt not in (torch.complex64, torch.complex128):
        raise CosmoError("Carlson arguments must be complex64 or complex128 tensors")
    n = args[0].numel()
    conv = []
    for a in args:
        _need_gpu(a, name)
        if a.dtype != cdt or a.numel() != n:
            raise CosmoError(f"{name}: arguments must share dtype and size")
        conv.append(torch.view_as_real(a.reshape(-1).contiguous()))
    out = torch.empty(n, dtype=cdt, device=dev)
    ro = torch.view_as_real(out)
    dt = 0 if cdt == torch.complex64 else 1
    with torch.cuda.device(dev):
        rc = getattr(lib, name)(dt, n, *[_ptr(a) for a in conv], _ptr(ro), _stream(dev))
    _check(rc, name)
    return out.reshape(args[0].shape)


def carlson_rf(x, y, z):
    return _carlson("carlson_rf", (x, y, z))


def carlson_rd(x, y, z):
    return _carlson("carlson_rd", (x, y, z))


def carlson_rj(x, y, z, p):
    return _carlson("carlson_rj", (x, y, z, p))


def carlson_rc(x, y):
    return _carlson("carlson_rc", (x, y))


def cosmo_distance(kind, params, z, info=False, workspace=None):
    """Observable `kind` ('DC','DM','DL','MU','T','X','DA') of shape [n_cosmo, n_z],
    in z's dtype.  With info=True also returns the int32 per-cosmology flags."""
    lib = load()
    p = _params(params)
    n_c = p.shape[0]
    zc, n_z, stride, _ = _z_layout(z, n_c)
    if zc.device != p.device:
        raise CosmoError("params and z must be on the same device")
    out = torch.empty((n_c, n_z), dtype=zc.dtype, device=p.device)
    inf = torch.empty(n_c, dtype=torch.int32, device=p.device) if info else None
    ws = workspace if workspace is not None else _workspace(n_c, n_z, p.device)
    with torch.cuda.device(p.device):
        rc = lib.cosmo_distance(KINDS[kind], DTYPES[zc.dtype], _ptr(p), n_c, _ptr(zc), n_z, stride,
                                _ptr(out), _ptr(inf), _ptr(ws), ws.numel(), _stream(p.device))
    _check(rc, "cosmo_distance")
    return (out, inf) if info else out


ROUTES = ("carlson", "carlson_fp64_rf", "quadrature", "adjoint_quadrature")


def cosmo_route_counts(kind, params, z, workspace=None):
    """Per-cosmology lane counts of the routes of `kind` (int64 [n_cosmo, 4], columns as
    ROUTES): value by the Carlson reduction in the dtype's precision; FP32 X lanes with
    the R_F term refined in FP64; value by quadrature; adjoint by Leibniz quadrature."""
    lib = load()
    p = _params(params)
    n_c = p.shape[0]
    zc, n_z, stride, _ = _z_layout(z, n_c)
    counts = torch.empty((n_c, 4), dtype=torch.int64, device=p.device)
    ws = workspace if workspace is not None else _workspace(n_c, n_z, p.device)
    with torch.cuda.device(p.device):
        rc = lib.cosmo_route_counts(KINDS[kind], DTYPES[zc.dtype], _ptr(p), n_c, _ptr(zc), n_z, stride,
                                    _ptr(counts), _ptr(ws), ws.numel(), _stream(p.device))
    _check(rc, "cosmo_route_counts")
    return counts


def cosmo_distance_between(kind, params, z1, z2, info=False, workspace=None):
    """Observable `kind` ('DC', 'DM', 'DA', 'T') between redshifts z1 and z2 (either
    order; z2 may be +inf: chi(z1, inf), D_M(z1, inf), D_A = 0, the age t(z1, inf)),
    shape [n_cosmo, n_z] in the dtype of z1.  z1 and z2: same shape and dtype, [n_z]
    shared by all cosmologies or [n_cosmo, n_z]."""
    lib = load()
    p = _params(params)
    n_c = p.shape[0]
    a, n_z, stride, _ = _z_layout(z1, n_c)
    _need_gpu(z2, "z2")
    if z2.shape != z1.shape or z2.dtype != z1.dtype:
        raise CosmoError("z1 and z2 must have the same shape and dtype")
    b = z2.contiguous()
    a = a.contiguous()
    stride = 0 if a.dim() == 1 else n_z
    if a.device != p.device or b.device != p.device:
        raise CosmoError("params, z1 and z2 must be on the same device")
    out = torch.empty((n_c, n_z), dtype=a.dtype, device=p.device)
    inf = torch.empty(n_c, dtype=torch.int32, device=p.device) if info else None
    ws = workspace if workspace is not None else _workspace(n_c, n_z, p.device)
    with torch.cuda.device(p.device):
        rc = lib.cosmo_distance_between(KINDS[kind], DTYPES[a.dtype], _ptr(p), n_c, _ptr(a), _ptr(b), n_z, stride,
                                        _ptr(out), _ptr(inf), _ptr(ws), ws.numel(), _stream(p.device))
    _check(rc, "cosmo_distance_between")
    return (out, inf) if info else out


def cosmo_distance_between_vjp(kind, params, z1, z2, cot, want_params=True, want_z=True, info=False,
                               workspace=None, want_value=False):
    """Adjoint of cosmo_distance_between for 'DC', 'DM', 'DA', 'T': (grad_params [n_cosmo, 4]
    float64 or None, grad_z1, grad_z2 like the limits (summed over cosmologies when
    shared) or None); with want_value=True the observable first."""
    lib = load()
    p = _params(params)
    n_c = p.shape[0]
    a, n_z, _, shared = _z_layout(z1, n_c)
    _need_gpu(z2, "z2")
    if z2.shape != z1.shape or z2.dtype != z1.dtype:
        raise CosmoError("z1 and z2 must have the same shape and dtype")
    a = a.contiguous()
    b = z2.contiguous()
    stride = 0 if shared else n_z
    _need_gpu(cot, "cot")
    c = cot.to(a.dtype).reshape(n_c, n_z).contiguous()
    gp = torch.empty((n_c, 4), dtype=torch.float64, device=p.device) if want_params else None
    g1 = g2 = None
    if want_z:
        g1 = torch.empty(n_z if shared else (n_c, n_z), dtype=a.dtype, device=p.device)
        g2 = torch.empty_like(g1)
    val = torch.empty((n_c, n_z), dtype=a.dtype, device=p.device) if want_value else None
    inf = torch.empty(n_c, dtype=torch.int32, device=p.device) if info else None
    ws = workspace if workspace is not None else _workspace(n_c, n_z, p.device)
    with torch.cuda.device(p.device):
        rc = lib.cosmo_distance_between_vjp(KINDS[kind], DTYPES[a.dtype], _ptr(p), n_c, _ptr(a), _ptr(b), n_z,
                                            stride, _ptr(c), _ptr(val), _ptr(gp), _ptr(g1), _ptr(g2), _ptr(inf),
                                            _ptr(ws), ws.numel(), _stream(p.device))
    _check(rc, "cosmo_distance_between_vjp")
    res = ((val,) if want_value else ()) + (gp, g1, g2)
    return res + (inf,) if info else res


def _vjp_call(name, kind, params, z, cot, want_params, want_z, info, workspace, want_value):
    lib = load()
    p = _params(params)
    n_c = p.shape[0]
    zc, n_z, stride, shared = _z_layout(z, n_c)
    _need_gpu(cot, "cot")
    c = cot.to(zc.dtype).reshape(n_c, n_z).contiguous()
    gp = torch.empty((n_c, 4), dtype=torch.float64, device=p.device) if want_params else None
    gz = None
    if want_z:
        gz = torch.empty(n_z if shared else (n_c, n_z), dtype=zc.dtype, device=p.device)
    val = torch.empty((n_c, n_z), dtype=zc.dtype, device=p.device) if want_value else None
    inf = torch.empty(n_c, dtype=torch.int32, device=p.device) if info else None
    args = (KINDS[kind], DTYPES[zc.dtype], _ptr(p), n_c, _ptr(zc), n_z, stride, _ptr(c), _ptr(val), _ptr(gp),
            _ptr(gz), _ptr(inf))
    with torch.cuda.device(p.device):
        if name == "cosmo_distance_vjp":
            ws = workspace if workspace is not None else _workspace(n_c, n_z, p.device)
            rc = lib.cosmo_distance_vjp(*args, _ptr(ws), ws.numel(), _stream(p.device))
        else:
            rc = lib.cosmo_distance_vjp_noalloc(*args, _stream(p.device))
    _check(rc, name)
    res = ((val,) if want_value else ()) + (gp, gz)
    return res + (inf,) if info else res


def cosmo_distance_vjp(kind, params, z, cot, want_params=True, want_z=True, info=False, workspace=None,
                       want_value=False):
    """Adjoint: (grad_params [n_cosmo, 4] float64 or None, grad_z like z or None).
    With want_value=True the observable is computed in the same pass and returned
    first: (value [n_cosmo, n_z], grad_params, grad_z)."""
    return _vjp_call("cosmo_distance_vjp", kind, params, z, cot, want_params, want_z, info, workspace, want_value)


def cosmo_distance_vjp_noalloc(kind, params, z, cot, want_params=True, want_z=True, info=False,
                               want_value=False):
    """cosmo_distance_vjp with the library's fixed per-GPU device array in place of a
    workspace (the C entry point allocates nothing; the outputs returned here are
    torch tensors allocated by this wrapper).  Problems beyond NOALLOC_SCRATCH_BYTES
    raise CosmoError (COSMO_E_SCRATCH); calls overlapping in time on one GPU race."""
    return _vjp_call("cosmo_distance_vjp_noalloc", kind, params, z, cot, want_params, want_z, info, None,
                     want_value)


def cosmo_distance_jac(kind, params, z, want_value=True, info=False, workspace=None):
    """Materialised Jacobian: (value [n_cosmo, n_z] or None, jac [5, n_cosmo, n_z]) with
    jac[q] = d value / d(H0, Om0, OL0, Or0, z)[q], in z's dtype."""
    lib = load()
    p = _params(params)
    n_c = p.shape[0]
    zc, n_z, stride, _ = _z_layout(z, n_c)
    if zc.device != p.device:
        raise CosmoError("params and z must be on the same device")
    val = torch.empty((n_c, n_z), dtype=zc.dtype, device=p.device) if want_value else None
    jac = torch.empty((5, n_c, n_z), dtype=zc.dtype, device=p.device)
    inf = torch.empty(n_c, dtype=torch.int32, device=p.device) if info else None
    ws = workspace if workspace is not None else _workspace(n_c, n_z, p.device)
    with torch.cuda.device(p.device):
        rc = lib.cosmo_distance_jac(KINDS[kind], DTYPES[zc.dtype], _ptr(p), n_c, _ptr(zc), n_z, stride,
                                    _ptr(val), _ptr(jac), _ptr(inf), _ptr(ws), ws.numel(), _stream(p.device))
    _check(rc, "cosmo_distance_jac")
    return (val, jac, inf) if info else (val, jac)


def cosmo_gaussian_loglike(kind, params, z, obs, sigma=None, ivar=None, weights=None, want_params=True,
                           want_z=True, info=False, workspace=None):
    """Fused Gaussian log-likelihood: loglike[c] = -1/2 sum_i (obs_i - out_ci)^2 / sigma_i^2
    with its gradient (d/d(H0, Om0, OL0, Or0) per cosmology [n_cosmo, 4] float64, and
    d/dz like cosmo_distance_vjp's grad_z), from one pass.  obs and sigma (or ivar =
    1/sigma^2; a scalar broadcasts) are laid out as z; weights [n_cosmo] scale each
    cosmology's term in the gradient.  Returns (loglike, grad_params, grad_z)."""
    lib = load()
    p = _params(params)
    n_c = p.shape[0]
    zc, n_z, stride, shared = _z_layout(z, n_c)
    if (sigma is None) == (ivar is None):
        raise CosmoError("give exactly one of sigma and ivar")
    iv = ivar if ivar is not None else 1.0 / torch.as_tensor(sigma, dtype=torch.float64, device=p.device) ** 2
    shape = zc.shape
    ob = torch.as_tensor(obs, device=p.device).to(zc.dtype).expand(shape).contiguous()
    iv = torch.as_tensor(iv, device=p.device).to(zc.dtype).expand(shape).contiguous()
    wc = None
    if weights is not None:
        wc = torch.as_tensor(weights, dtype=torch.float64, device=p.device).reshape(n_c).contiguous()
    ll = torch.empty(n_c, dtype=torch.float64, device=p.device)
    gp = torch.empty((n_c, 4), dtype=torch.float64, device=p.device) if want_params else None
    gz = None
    if want_z:
        gz = torch.empty(n_z if shared else (n_c, n_z), dtype=zc.dtype, device=p.device)
    inf = torch.empty(n_c, dtype=torch.int32, device=p.device) if info else None
    ws = workspace if workspace is not None else _workspace(n_c, n_z, p.device)
    with torch.cuda.device(p.device):
        rc = lib.cosmo_gaussian_loglike(KINDS[kind], DTYPES[zc.dtype], _ptr(p), n_c, _ptr(zc), n_z, stride,
                                        _ptr(ob), _ptr(iv), _ptr(wc), _ptr(ll), _ptr(gp), _ptr(gz), _ptr(inf),
                                        _ptr(ws), ws.numel(), _stream(p.device))
    _check(rc, "cosmo_gaussian_loglike")
    return (ll, gp, gz, inf) if info else (ll, gp, gz)


class _GaussianLogLike(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kind, params, z, obs, ivar):
        need_p, need_z = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        ll, gp, gz = cosmo_gaussian_loglike(kind, params.detach(), z.detach(), obs, ivar=ivar,
                                            want_params=need_p, want_z=need_z)
        ctx.kind = kind
        ctx.save_for_backward(params, z, obs, ivar)
        ctx.grads = (gp, gz)
        return ll

    @staticmethod
    def backward(ctx, g):
        params, z, obs, ivar = ctx.saved_tensors
        gp, gz = ctx.grads
        # The forward pass computed the gradients for unit weights.  Parameter gradients are
        # per cosmology, so any upstream weights rescale them row by row; the z-gradient of
        # a shared z row is a sum over cosmologies, which takes the weights inside the sum:
        # recomputed with them unless there is a single cosmology.  (No host
        # synchronisation: which case applies follows from shapes, not values.)
        if gp is not None:
            gp = gp * g[:, None]
        if gz is not None:
            if gz.dim() == 2:
                gz = gz * g[:, None].to(gz.dtype)
            elif g.shape[0] == 1:
                gz = gz * g[0].to(gz.dtype)
            else:
                _, _, gz = cosmo_gaussian_loglike(ctx.kind, params.detach(), z.detach(), obs, ivar=ivar, weights=g,
                                                  want_params=False, want_z=True)
        if gz is not None:
            gz = gz.reshape(z.shape)
        return None, gp.reshape(params.shape) if gp is not None else None, gz, None, None


def gaussian_loglike(kind, params, z, obs, sigma):
    """Differentiable fused Gaussian log-likelihood per cosmology (see cosmo_gaussian_loglike)."""
    zc = z.detach()
    iv = (1.0 / torch.as_tensor(sigma, device=zc.device, dtype=torch.float64) ** 2).to(zc.dtype)
    return _GaussianLogLike.apply(kind, params, z, torch.as_tensor(obs, device=zc.device).to(zc.dtype),
                                  iv.expand(zc.shape[-1:] if zc.dim() == 1 else zc.shape).contiguous())


def _f64(t, shape, name):
    _need_gpu(t, name)
    if t.dtype != torch.float64 or tuple(t.shape) != tuple(shape):
        raise CosmoError(f"{name} must be float64 of shape {tuple(shape)}")
    return t.contiguous()


def snia_draw(a, b, log_s, dtheta, eps, dtype=torch.float32):
    """Latent redshifts of the supernova model's guide (see include/cosmo.h: snia_draw):
    z[s][n] = exp(a[n] + dtheta[s] . b[n] + exp(log_s[n]) eps[s][n]) in `dtype`."""
    lib = load()
    n_sn = a.shape[0]
    S = dtheta.shape[0]
    args = [_f64(a, (n_sn,), "a"), _f64(b, (n_sn, 2), "b"), _f64(log_s, (n_sn,), "log_s"),
            _f64(dtheta, (S, 2), "dtheta"), _f64(eps, (S, n_sn), "eps")]
    z = torch.empty((S, n_sn), dtype=dtype, device=a.device)
    with torch.cuda.device(a.device):
        rc = lib.snia_draw(DTYPES[dtype], S, n_sn, *(_ptr(t) for t in args), _ptr(z), _stream(a.device))
    _check(rc, "snia_draw")
    return z


def snia_latent_vjp(a, b, log_s, dtheta, eps, zhat, grad_z, sigma_z, gamma_shape, gamma_rate, dtype=torch.float32,
                    workspace=None):
    """Per-supernova terms of the model's log joint summed over draws and supernovae,
    and the adjoint of those terms plus an outside term whose z-gradient is grad_z (see
    include/cosmo.h: snia_latent_vjp).  Returns (F, grad_dtheta [S, 2], grad_a,
    grad_b [N, 2], grad_log_s), all float64."""
    lib = load()
    n_sn = a.shape[0]
    S = dtheta.shape[0]
    args = [_f64(a, (n_sn,), "a"), _f64(b, (n_sn, 2), "b"), _f64(log_s, (n_sn,), "log_s"),
            _f64(dtheta, (S, 2), "dtheta"), _f64(eps, (S, n_sn), "eps"), _f64(zhat, (n_sn,), "zhat")]
    gz = None
    if grad_z is not None:
        _need_gpu(grad_z, "grad_z")
        if grad_z.dtype != dtype or tuple(grad_z.shape) != (S, n_sn):
            raise CosmoError(f"grad_z must be {dtype} of shape {(S, n_sn)}")
        gz = grad_z.contiguous()
    dev = a.device
    vd = torch.empty(1 + 2 * S, dtype=torch.float64, device=dev)
    ga = torch.empty(n_sn, dtype=torch.float64, device=dev)
    gb = torch.empty((n_sn, 2), dtype=torch.float64, device=dev)
    gl = torch.empty(n_sn, dtype=torch.float64, device=dev)
    if workspace is None:
        nb = ctypes.c_size_t()
        _check(lib.snia_workspace_size(S, n_sn, ctypes.byref(nb)), "snia_workspace_size")
        workspace = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        rc = lib.snia_latent_vjp(DTYPES[dtype], S, n_sn, *(_ptr(t) for t in args), _ptr(gz), float(sigma_z),
                                 float(gamma_shape), float(gamma_rate), _ptr(vd), _ptr(ga), _ptr(gb), _ptr(gl),
                                 _ptr(workspace), workspace.numel(), _stream(dev))
    _check(rc, "snia_latent_vjp")
    return vd[0], vd[1:].reshape(S, 2), ga, gb, gl


class _Distance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kind, params, z):
        ctx.kind = kind
        ctx.save_for_backward(params, z)
        return cosmo_distance(kind, params.detach(), z.detach())

    @staticmethod
    def backward(ctx, grad_out):
        params, z = ctx.saved_tensors
        gp, gz = cosmo_distance_vjp(ctx.kind, params.detach(), z.detach(), grad_out,
                                    want_params=ctx.needs_input_grad[1], want_z=ctx.needs_input_grad[2])
        if gz is not None:
            gz = gz.reshape(z.shape)
        return None, gp.reshape(params.shape) if gp is not None else None, gz


def distance(kind, params, z):
    """Differentiable observable: autograd through cosmo_distance / cosmo_distance_vjp."""
    return _Distance.apply(kind, params, z)


class _Between(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kind, params, z1, z2):
        ctx.kind = kind
        ctx.save_for_backward(params, z1, z2)
        return cosmo_distance_between(kind, params.detach(), z1.detach(), z2.detach())

    @staticmethod
    def backward(ctx, grad_out):
        params, z1, z2 = ctx.saved_tensors
        want_z = ctx.needs_input_grad[2] or ctx.needs_input_grad[3]
        gp, g1, g2 = cosmo_distance_between_vjp(ctx.kind, params.detach(), z1.detach(), z2.detach(), grad_out,
                                                want_params=ctx.needs_input_grad[1], want_z=want_z)
        g1 = g1.reshape(z1.shape) if (g1 is not None and ctx.needs_input_grad[2]) else None
        g2 = g2.reshape(z2.shape) if (g2 is not None and ctx.needs_input_grad[3]) else None
        return None, gp.reshape(params.shape) if gp is not None else None, g1, g2


def distance_between(kind, params, z1, z2):
    """Differentiable observable between two redshifts ('DC', 'DM', 'DA', 'T'): autograd
    through cosmo_distance_between / cosmo_distance_between_vjp."""
    return _Between.apply(kind, params, z1, z2)


def version():
    return load().cosmo_version().decode()
