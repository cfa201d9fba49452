"""MI355X-native batched, differentiable LambdaCDM+radiation distances.

Karchev, "Analytic auto-differentiable LambdaCDM cosmography" (arXiv:2212.01937):
the distance integrals (eqs. 2.3-2.5) are reduced to Carlson symmetric elliptic
integrals (sec. 3.1, eqs. 3.7-3.9; app. B.1, eqs. B.1-B.3) and evaluated by
hand-written HIP kernels for gfx950 behind a C ABI (include/cosmo.h).

Submodules:
  cosmo      ctypes binding of libcosmo.so (same entry-point names as the C ABI)
             and the torch.autograd.Function built on it
  workloads  seeded synthetic inputs (no method arithmetic)
  build      compiles libcosmo.so with hipcc for gfx950
"""
__all__ = ["cosmo", "workloads", "build"]
