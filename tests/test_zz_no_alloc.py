"""The entry point that allocates nothing (cosmo_distance_vjp_noalloc) against the
workspace entry point it varies (cosmo_distance_vjp): same kernels, same reduction
order, so every output must agree bit for bit.  Two calls in a row, the second on
a smaller problem, so the second reads only what it wrote into the shared device
array; both the shared-z layout with several cosmology tiles (tile partials of the
z-gradient in the array) and per-cosmology rows are covered."""
import numpy as np
import pytest
import torch

from paper_2212_01937_amd import cosmo, workloads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(n_cosmo, n_z, shared, dt, seed):
    params, _ = workloads.config2(n_cosmo=n_cosmo, n_z=8)
    rng = np.random.default_rng(seed)
    if shared:
        z = np.sort(10 ** rng.uniform(-3, 1, n_z))
    else:
        z = np.sort(10 ** rng.uniform(-3, 1, (n_cosmo, n_z)), axis=1)
    w = rng.standard_normal((n_cosmo, n_z))
    return (torch.tensor(params, device=DEV), torch.tensor(z, dtype=dt, device=DEV),
            torch.tensor(w, dtype=dt, device=DEV))


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", ["MU", "T"])
def test_noalloc_equals_workspace_entry_point(dt, kind):
    # 40 x 9000 shared: 8 redshifts per lane, 40 one-cosmology tiles (tile partials of
    # grad_z in the array); then 7 x 1500 per-cosmology rows; then 3 x 100 shared
    for n_c, n_z, shared, seed in ((40, 9000, True, 1), (7, 1500, False, 2), (3, 100, True, 3)):
        p, z, w = _case(n_c, n_z, shared, dt, seed)
        print(f"noalloc {kind} {dt} {n_c}x{n_z} shared={shared}", flush=True)
        na = cosmo.cosmo_distance_vjp_noalloc(kind, p, z, w, want_value=True, info=True)
        ref = cosmo.cosmo_distance_vjp(kind, p, z, w, want_value=True, info=True)
        torch.cuda.synchronize()
        for a, b, name in zip(na, ref, ("value", "grad_params", "grad_z", "info")):
            assert a.shape == b.shape and a.dtype == b.dtype, name
            if a.is_floating_point():
                assert torch.equal(torch.isnan(a), torch.isnan(b)), (name, n_c, n_z)
                a, b = torch.nan_to_num(a, nan=0.0), torch.nan_to_num(b, nan=0.0)
            assert torch.equal(a, b), (name, n_c, n_z)
        assert torch.isfinite(na[1]).all() and torch.isfinite(na[2]).all()


def test_noalloc_partial_outputs_and_refusal():
    """Gradient outputs requested one at a time (the layout packs only what is
    needed), and a problem beyond the array is refused without launching."""
    p, z, w = _case(20, 3000, True, torch.float32, 5)
    gp_only = cosmo.cosmo_distance_vjp_noalloc("DL", p, z, w, want_z=False)
    gz_only = cosmo.cosmo_distance_vjp_noalloc("DL", p, z, w, want_params=False)
    ref = cosmo.cosmo_distance_vjp("DL", p, z, w)
    torch.cuda.synchronize()
    assert gp_only[1] is None and gz_only[0] is None
    assert torch.equal(gp_only[0], ref[0]) and torch.equal(gz_only[1], ref[1])
    big_p = torch.tensor([[70.0, 0.3, 0.7, 0.0]], dtype=torch.float64, device=DEV).repeat(100000, 1)
    zz = torch.ones(1, dtype=torch.float64, device=DEV)
    with pytest.raises(cosmo.CosmoError, match="COSMO_E_SCRATCH"):
        cosmo.cosmo_distance_vjp_noalloc("DC", big_p, zz, torch.ones(100000, 1, dtype=torch.float64, device=DEV))
