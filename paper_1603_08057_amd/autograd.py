"""torch.autograd.Function around the HIP log-likelihood and its score.

forward(theta) returns l(theta) (eq. loglikelihood) from a fresh factorization
of Sigma(theta); backward returns grad_out * g(theta) with g from rsf_grad
(eq. gradient, traces by peeling).  The factor is rebuilt for each theta and
dropped after backward (recomputation rather than storage).
"""
import torch

from ._lib import Factor


class _LogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, points, z, kernel, eps, leaf, eps_peel, seed, opts):
        th = [float(v) for v in theta.detach().cpu().tolist()]
        F = Factor(points, th, kernel=kernel, eps=eps, leaf=leaf, **opts)
        ell = F.loglik(z)
        ctx.F = F
        ctx.z = z
        ctx.eps_peel = eps_peel
        ctx.seed = seed
        return torch.tensor(ell, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        g, _ = ctx.F.grad(ctx.z, ctx.eps_peel, ctx.seed)
        ctx.F.close()
        ctx.F = None
        gt = torch.tensor(g, dtype=torch.float64, device=grad_out.device) * grad_out
        return gt, None, None, None, None, None, None, None, None


def loglik_fn(theta, points, z, kernel=1, eps=1e-6, leaf=64, eps_peel=None, seed=0, **opts):
    """l(theta) as a differentiable function of theta = (rho, sigma2, nugget)."""
    return _LogLik.apply(theta, points, z, kernel, eps, leaf, eps_peel, seed, opts)
