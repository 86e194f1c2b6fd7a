"""torch.autograd.Function around the HIP log-likelihood and its score.

forward(theta) returns l(theta) (eq. loglikelihood) from a fresh factorization
of Sigma(theta); backward returns grad_out * g(theta) with g from rsf_grad
(eq. gradient, traces by peeling).  The factorization made in forward is kept
for backward, or, when memory is short (or on request), released after
forward and made again in backward from the same inputs: recomputation rather
than storage.  The factorization is deterministic, so both give the same
score.
"""
import torch

from ._lib import Factor


def _keep(F, keep_factor):
    """Whether to hold F from forward to backward.  "auto": only while the free
    device memory is at least twice the factor's bytes (the score's peeling
    needs working memory of that order beside the factor)."""
    if keep_factor != "auto":
        return bool(keep_factor)
    free, _ = torch.cuda.mem_get_info()
    return free >= 2 * F.tree_info()["factor_bytes"]


class _LogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, points, z, kernel, eps, leaf, eps_peel, seed, keep_factor, opts):
        th = [float(v) for v in theta.detach().cpu().tolist()]
        F = Factor(points, th, kernel=kernel, eps=eps, leaf=leaf, **opts)
        ell = F.loglik(z)
        if _keep(F, keep_factor):
            ctx.F = F
        else:
            F.close()
            ctx.F = None
            ctx.rebuild = (points, th, kernel, eps, leaf, opts)
        ctx.z = z
        ctx.eps_peel = eps_peel
        ctx.seed = seed
        return torch.tensor(ell, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        F = ctx.F
        if F is None:
            points, th, kernel, eps, leaf, opts = ctx.rebuild
            F = Factor(points, th, kernel=kernel, eps=eps, leaf=leaf, **opts)
        g, _ = F.grad(ctx.z, ctx.eps_peel, ctx.seed)
        F.close()
        ctx.F = None
        gt = torch.tensor(g, dtype=torch.float64, device=grad_out.device) * grad_out
        return gt, None, None, None, None, None, None, None, None, None


def loglik_fn(theta, points, z, kernel=1, eps=1e-6, leaf=64, eps_peel=None, seed=0, keep_factor="auto", **opts):
    """l(theta) as a differentiable function of theta = (rho, sigma2, nugget).

    keep_factor: True holds the factorization from forward to backward; False
    releases it after forward and factors again in backward; "auto" keeps it
    only while the free device memory is at least twice its size."""
    return _LogLik.apply(theta, points, z, kernel, eps, leaf, eps_peel, seed, keep_factor, opts)
