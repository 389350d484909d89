"""torch.autograd wrapper: the optimal UOT value as a differentiable function
of the marginals (mu, nu).

Forward runs the HIP domain-decomposition solver and returns the dual value
D(alpha_bar, beta_hat) of its certificate (equal to the optimal value at
convergence, Theorem existence-global-solution); backward returns the
envelope-theorem gradients computed on the device by dd_uot_backward.  The
tensors only carry data in and out; every step runs in libdd_uot.so.
"""
from __future__ import annotations

import torch

from . import binding as B


class UOTValue(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, nu, cfg, half_iters):
        m = mu.detach().to("cpu", torch.float64).numpy()
        v = nu.detach().to("cpu", torch.float64).numpy()
        stream = torch.cuda.current_stream().cuda_stream if mu.is_cuda else None
        h = B.dd_uot_init(cfg, m, v, stream=stream)
        try:
            B.dd_uot_iterate(h, half_iters, stats=False)
            s = B.dd_uot_score(h, 0)
            dmu, dnu = B.dd_uot_backward(h, 0, cfg.n1, cfg.n2)
        finally:
            B.dd_uot_destroy(h)
        ctx.save_for_backward(torch.from_numpy(dmu).to(mu.device, mu.dtype),
                              torch.from_numpy(dnu).to(nu.device, nu.dtype))
        ctx.score = s
        return mu.new_tensor(s["dual"])

    @staticmethod
    def backward(ctx, gout):
        dmu, dnu = ctx.saved_tensors
        return gout * dmu, gout * dnu, None, None


def uot_value(mu: torch.Tensor, nu: torch.Tensor, cfg, half_iters: int) -> torch.Tensor:
    """Differentiable optimal value of the unbalanced problem between mu and nu
    (n1 x n2 tensors of point masses) after `half_iters` DD half-iterations."""
    if mu.shape != (cfg.n1, cfg.n2) or nu.shape != (cfg.n1, cfg.n2):
        raise ValueError("marginals must have the grid shape of the config")
    return UOTValue.apply(mu, nu, cfg, int(half_iters))


__all__ = ["UOTValue", "uot_value"]
