"""The entry points under HIP graph capture (torch.cuda.graph): a captured call with a
caller-supplied workspace records only kernel launches (no allocation, no memset),
and every replay -- with eager work of the program and synchronisations between the
replays, and after the captured inputs are overwritten in place -- matches the eager
call on the same inputs bit for bit (the kernels and their reduction orders are the
same).  The eager results themselves are checked against the oracle elsewhere."""
import numpy as np
import pytest
import torch

from paper_2212_01937_amd import cosmo, workloads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _eager_noise(p):
    """Work of the program between replays: another call on other inputs, torch ops."""
    z = torch.linspace(0.05, 3.0, 777, dtype=torch.float64, device=DEV)
    out = cosmo.cosmo_distance("DC", p, z)
    return (out * 2.0).sum().item()


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_vjp_graph_replays_match_eager(dt):
    params, z = workloads.config2(n_cosmo=24, n_z=3000)
    p = torch.tensor(params, device=DEV)
    zt = torch.tensor(z, dtype=dt, device=DEV)
    w = torch.tensor(np.random.default_rng(3).standard_normal(z.shape), dtype=dt, device=DEV)
    ws = torch.empty(cosmo.workspace_size(*z.shape), dtype=torch.uint8, device=DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture (torch's own allocations)
        cosmo.cosmo_distance_vjp("MU", p, zt, w, want_value=True, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        val, gp, gz = cosmo.cosmo_distance_vjp("MU", p, zt, w, want_value=True, workspace=ws)
    rng = np.random.default_rng(4)
    for rep in range(4):
        if rep == 2:  # new inputs written into the captured buffers
            zt.copy_(torch.tensor(np.sort(10 ** rng.uniform(-3, 1, z.shape), axis=1), dtype=dt, device=DEV))
            w.copy_(torch.tensor(rng.standard_normal(z.shape), dtype=dt, device=DEV))
        _eager_noise(p)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        rv, rgp, rgz = cosmo.cosmo_distance_vjp("MU", p, zt.clone(), w.clone(), want_value=True)
        torch.cuda.synchronize()
        assert torch.equal(val, rv) and torch.equal(gp, rgp) and torch.equal(gz, rgz), (dt, rep)


def test_forward_and_likelihood_graph_replays_match_eager():
    """The launch-bound small case (one cosmology x 1000 redshifts) forward and the fused
    likelihood (shared z, gradient summed over cosmologies across tiles)."""
    p1, z1 = workloads.config1()
    p = torch.tensor(p1, device=DEV)
    zt = torch.tensor(z1, dtype=torch.float32, device=DEV)
    ws = torch.empty(cosmo.workspace_size(1, z1.size), dtype=torch.uint8, device=DEV)
    params5, z5 = workloads.config5(n_cosmo=40, n_z=20000)
    p5 = torch.tensor(params5, device=DEV)
    z5t = torch.tensor(z5, dtype=torch.float32, device=DEV)
    obs = cosmo.cosmo_distance("MU", p5[:1], z5t)[0] + 0.1
    # inverse variances as a device tensor made before the capture (a Python scalar
    # would be copied from the host inside it), formed as the binding forms sigma's
    ivar = (1.0 / torch.as_tensor(0.1, dtype=torch.float64, device=DEV) ** 2).to(torch.float32)
    ivar = ivar.expand(z5t.shape).contiguous()
    ws5 = torch.empty(cosmo.workspace_size(40, z5.size), dtype=torch.uint8, device=DEV)
    cosmo.cosmo_distance("MU", p, zt, workspace=ws)
    cosmo.cosmo_gaussian_loglike("MU", p5, z5t, obs, ivar=ivar, workspace=ws5)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mu = cosmo.cosmo_distance("MU", p, zt, workspace=ws)
        ll, gp, gz = cosmo.cosmo_gaussian_loglike("MU", p5, z5t, obs, ivar=ivar, workspace=ws5)
    for rep in range(3):
        _eager_noise(p)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(mu, cosmo.cosmo_distance("MU", p, zt)), rep
        rl, rgp, rgz = cosmo.cosmo_gaussian_loglike("MU", p5, z5t, obs, sigma=0.1)
        assert torch.equal(ll, rl) and torch.equal(gp, rgp) and torch.equal(gz, rgz), rep


_FIRST_CALL_SCRIPT = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
from paper_2212_01937_amd import cosmo, workloads

dev = torch.device("cuda:0")
params, z = workloads.config2(n_cosmo=24, n_z=3000)
p = torch.tensor(params, device=dev)
zt = torch.tensor(z, dtype=torch.float32, device=dev)
w = torch.tensor(np.random.default_rng(3).standard_normal(z.shape), dtype=torch.float32, device=dev)
ws = torch.empty(cosmo.workspace_size(*z.shape), dtype=torch.uint8, device=dev)
cosmo.load()  # dlopen only: no call into the library before the capture
torch.cuda.synchronize()
g = torch.cuda.CUDAGraph()
with torch.cuda.graph(g):
    val, gp, gz = cosmo.cosmo_distance_vjp("MU", p, zt, w, want_value=True, workspace=ws)
for rep in range(3):
    g.replay()
    torch.cuda.synchronize()
    rv, rgp, rgz = cosmo.cosmo_distance_vjp("MU", p, zt, w, want_value=True)
    torch.cuda.synchronize()
    assert torch.equal(val, rv) and torch.equal(gp, rgp) and torch.equal(gz, rgz), rep
print("first call captured and replayed", flush=True)
"""


def test_first_library_call_of_a_process_is_capturable():
    """The library needs no initialisation: in a fresh process the very first call into
    it can be captured in a HIP graph, and every replay equals the eager call."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _FIRST_CALL_SCRIPT, root], capture_output=True, text=True,
                       timeout=110)
    assert r.returncode == 0 and "first call captured" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
