"""Supernova Ia cosmology model of sec. 4 with variational inference, the distance
path as its inner loop.

Model (sec. 4, fig. 4b), for N supernovae with observed redshifts zhat_s and distance
moduli muhat_s:
    Om0, OL0               free (flat prior over the region where the method applies)
    z_s                    ~ Gamma(shape 3, rate beta = 3)                (the redshift prior)
    zhat_s | z_s           ~ N(z_s, (1 + z_s)^2 sigma_z^2),  sigma_z = 0.04 (photometric toy model)
    muhat_s | z_s, theta   ~ N(mu(z_s; theta), sigma_mu^2),  sigma_mu = 0.14
with radiationless LambdaCDM (Or0 = 0) and H0 fixed (it is degenerate with the
absolute magnitude).  mu(z; theta) and its gradients with respect to theta and every
z_s come from one fused pass of the HIP library (cosmo_gaussian_loglike).

Guide: a partial multivariate normal (sec. 4) -- a bivariate normal for (Om0, OL0) and,
per supernova, a normal for zeta_s = log z_s whose mean depends linearly on the
global parameters (correlations between each latent redshift and the cosmology are
kept, those between different supernovae are not):
    theta ~ N(m, L L^T),   zeta_s | theta ~ N(a_s + b_s . (theta - m), s_s^2),   z_s = exp(zeta_s).
The ELBO is estimated with S reparametrised samples per step and maximised with Adam.
"""
import math

import torch

from . import cosmo

SIGMA_MU = 0.14
SIGMA_Z = 0.04
BETA = 3.0
GAMMA_SHAPE = 3.0
H0 = 70.0


def params_of(theta):
    """(S, 2) of (Om0, OL0) -> (S, 4) rows (H0, Om0, OL0, Or0 = 0), float64."""
    s = theta.shape[0]
    h = torch.full((s, 1), H0, dtype=torch.float64, device=theta.device)
    zero = torch.zeros((s, 1), dtype=torch.float64, device=theta.device)
    return torch.cat([h, theta.to(torch.float64), zero], dim=1)


def log_joint(theta, z, zhat, muhat):
    """log p(theta, z, zhat, muhat) per sample, up to a constant: theta (S, 2) float64,
    z (S, N) latent redshifts in the compute dtype (float32 or float64), zhat and
    muhat (N,).  Differentiable in theta and z.  Returns (S,) float64."""
    S, N = z.shape
    obs = muhat.to(z.dtype).expand(S, N).contiguous()
    ll_mu = cosmo.gaussian_loglike("MU", params_of(theta), z, obs, SIGMA_MU)
    zd = z.to(torch.float64)
    zh = zhat.to(torch.float64)
    sd = (1.0 + zd) * SIGMA_Z
    ll_z = (-0.5 * ((zh - zd) / sd) ** 2 - torch.log(sd)).sum(1)
    lp_z = ((GAMMA_SHAPE - 1.0) * torch.log(zd) - BETA * zd).sum(1) + N * (
        GAMMA_SHAPE * math.log(BETA) - math.lgamma(GAMMA_SHAPE))
    return ll_mu + ll_z + lp_z


class PMVNGuide(torch.nn.Module):
    """Partial multivariate normal proposal over (Om0, OL0, {log z_s})."""

    def __init__(self, zhat, theta0=(0.3, 0.7), dtype=torch.float32):
        super().__init__()
        dev = zhat.device
        n = zhat.shape[0]
        self.dtype = dtype
        self.m = torch.nn.Parameter(torch.tensor(theta0, dtype=torch.float64, device=dev))
        self.l_raw = torch.nn.Parameter(torch.tensor([math.log(0.05), 0.0, math.log(0.05)], dtype=torch.float64,
                                                     device=dev))  # log diag 0, off-diag, log diag 1
        zc = zhat.to(torch.float64).clamp_min(0.02)
        self.a = torch.nn.Parameter(torch.log(zc))
        self.b = torch.nn.Parameter(torch.zeros((n, 2), dtype=torch.float64, device=dev))
        self.log_s = torch.nn.Parameter(torch.log((1.0 + zc) * SIGMA_Z / zc))

    def chol(self):
        l00, l10, l11 = torch.exp(self.l_raw[0]), self.l_raw[1], torch.exp(self.l_raw[2])
        zero = torch.zeros((), dtype=torch.float64, device=l00.device)
        return torch.stack([torch.stack([l00, zero]), torch.stack([l10, l11])])

    def normals(self, n_samples, gen):
        """The standard normals behind one set of draws: eg (S, 2) for the globals and
        el (S, N) for the latent redshifts (drawn in that order)."""
        dev = self.m.device
        eg = torch.randn((n_samples, 2), dtype=torch.float64, device=dev, generator=gen)
        el = torch.randn((n_samples, self.a.shape[0]), dtype=torch.float64, device=dev, generator=gen)
        return eg, el

    def draw(self, n_samples, gen):
        """Reparametrised draws: theta (S, 2), zeta (S, N) and the standard normals
        behind them, eg (S, 2) and el (S, N)."""
        eg, el = self.normals(n_samples, gen)
        dtheta = eg @ self.chol().T
        theta = self.m + dtheta
        s = torch.exp(self.log_s)
        # the per-supernova regression on the globals as two broadcast multiply-adds (a
        # (N, 2) x (2, S) product would go to a GEMM shaped badly for N ~ 1e6)
        zeta = self.a + dtheta[:, 0:1] * self.b[:, 0] + dtheta[:, 1:2] * self.b[:, 1] + s * el
        return theta, zeta, eg, el

    def sample(self, n_samples, gen):
        """Reparametrised draws: theta (S, 2), zeta (S, N) and log q(theta, zeta) (S,)."""
        theta, zeta, eg, el = self.draw(n_samples, gen)
        n = self.a.shape[0]
        logq = (-0.5 * (eg ** 2).sum(1) - torch.log(torch.diagonal(self.chol())).sum()
                - 0.5 * (el ** 2).sum(1) - self.log_s.sum()
                - 0.5 * (n + 2) * math.log(2 * math.pi))
        return theta, zeta, logq


class _SupernovaTerms(torch.autograd.Function):
    """sum_s loglike_mu(theta_s, z_s) + sum_{s,n} (photometric likelihood + redshift
    prior + Jacobian + eps^2/2) as a function of the guide's per-supernova parameters
    (a, b, log_s) and each draw's (dtheta, theta): the latent redshifts by snia_draw,
    the distance likelihood and its z- and theta-gradients by cosmo_gaussian_loglike,
    the remaining terms and the adjoint to the guide by snia_latent_vjp.  Value and
    gradients come from the one forward pass; the backward scales them."""

    @staticmethod
    def forward(ctx, a, b, log_s, dtheta, theta, eps, zhat, obs, ivar, dtype):
        a, b, log_s, dtheta, theta = (t.detach() for t in (a, b, log_s, dtheta, theta))
        z = cosmo.snia_draw(a, b, log_s, dtheta, eps, dtype)
        ll, gp, gz = cosmo.cosmo_gaussian_loglike("MU", params_of(theta), z, obs, ivar=ivar)
        F, gd, ga, gb, gl = cosmo.snia_latent_vjp(a, b, log_s, dtheta, eps, zhat, gz, SIGMA_Z, GAMMA_SHAPE, BETA,
                                                  dtype)
        ctx.save_for_backward(ga, gb, gl, gd, gp[:, 1:3])
        return ll.sum() + F

    @staticmethod
    def backward(ctx, go):
        ga, gb, gl, gd, gth = ctx.saved_tensors
        return go * ga, go * gb, go * gl, go * gd, go * gth, None, None, None, None, None


def _planes(guide, muhat, S, dtype):
    """Observed magnitudes and inverse variances laid out as the latent redshifts
    (S, N) in the distance precision, kept between steps."""
    key = (S, dtype, muhat.data_ptr())
    cache = getattr(guide, "_planes", None)
    if cache is None or cache[0] != key:
        N = muhat.shape[0]
        obs = muhat.to(dtype).expand(S, N).contiguous()
        ivar = torch.full((S, N), 1.0 / SIGMA_MU ** 2, dtype=dtype, device=muhat.device)
        guide._planes = cache = (key, obs, ivar)
    return cache[1], cache[2]


def elbo(guide, zhat, muhat, n_samples, gen):
    """Monte-Carlo ELBO estimate (mean over n_samples draws): E_q[log p(theta, z(zeta))
    + sum zeta (the Jacobian of z = exp(zeta)) - log q(theta, zeta)] + const.

    The per-supernova work (latent redshifts, distance likelihood, photometric
    likelihood, redshift prior, Jacobian, the guide's density in eps, and all their
    gradients) runs in the library's kernels (_SupernovaTerms); what stays here is the
    algebra of the two global parameters.  Equal to the mean over draws of log_joint +
    sum zeta - sample()'s log q - N log(2 pi)/2 on the same draws."""
    S = n_samples
    N = zhat.shape[0]
    eg, el = guide.normals(S, gen)
    L = guide.chol()
    dtheta = eg @ L.T
    theta = guide.m + dtheta
    obs, ivar = _planes(guide, muhat, S, guide.dtype)
    terms = _SupernovaTerms.apply(guide.a, guide.b, guide.log_s, dtheta, theta, el,
                                  zhat.to(torch.float64).contiguous(), obs, ivar, guide.dtype)
    const = S * N * (GAMMA_SHAPE * math.log(BETA) - math.lgamma(GAMMA_SHAPE)) - 0.5 * S * N * math.log(2 * math.pi)
    logq_rest = (-0.5 * (eg ** 2).sum() - S * torch.log(torch.diagonal(L)).sum()
                 - S * guide.log_s.sum() - 0.5 * S * (N + 2) * math.log(2 * math.pi))
    return (terms + const - logq_rest) / S


def fit(zhat, muhat, steps=2000, n_samples=4, lr=0.02, dtype=torch.float32, seed=0, theta0=(0.3, 0.7)):
    """Maximise the ELBO with Adam; returns the guide and the ELBO trace."""
    guide = PMVNGuide(zhat, theta0=theta0, dtype=dtype)
    opt = torch.optim.Adam(guide.parameters(), lr=lr, fused=True)  # one fused update kernel per step
    gen = torch.Generator(device=zhat.device)
    gen.manual_seed(seed)
    # the ELBO trace stays on the device during the fit (no host synchronisation per
    # step) and is copied to the host once at the end
    trace = torch.empty(steps, dtype=torch.float64, device=zhat.device)
    for i in range(steps):
        opt.zero_grad(set_to_none=True)
        loss = -elbo(guide, zhat, muhat, n_samples, gen)
        loss.backward()
        opt.step()
        trace[i] = -loss.detach()
    return guide, trace.cpu().tolist()
