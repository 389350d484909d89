"""torch.autograd wrapper: the optimal UOT value as a differentiable function
of the marginals (mu, nu) and, optionally, of the control values theta of a
smooth displacement of the Y points (y' = y + u_theta(y), cubic B-spline
tensor field, see inputs.displaced_points).

Forward runs the HIP domain-decomposition solver and returns the dual value
D(alpha_bar, beta_hat) of its certificate (equal to the optimal value at
convergence, Theorem existence-global-solution); backward returns the
envelope-theorem gradients computed on the device by dd_uot_backward and
dd_uot_backward_ypos (d/dy' = sum_x pi(x, y') 2 (y' - x), the plan recomputed
on the fly), and d/dtheta = B^T (d/dy') B through the linear B-spline map.
The tensors only carry data in and out (their device memory is handed to the
library directly); every step of the solve runs in libdd_uot.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from .inputs import displaced_points, displacement_basis


class UOTValue(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, nu, theta, cfg, half_iters):
        # the marginals go to the library as they are (device or host
        # memory, FP64), on the tensors' stream; the gradients come back
        # into tensors on the same device
        m = mu.detach().to(torch.float64).contiguous().view(-1)
        v = nu.detach().to(torch.float64).contiguous().view(-1)
        stream = torch.cuda.current_stream(mu.device).cuda_stream if mu.is_cuda else None
        n1, n2 = cfg.n1, cfg.n2
        if theta is None:
            h = B.dd_uot_init(cfg, m, v, stream=stream)
        else:
            th = theta.detach().to("cpu", torch.float64).numpy()
            y = displaced_points(n1, n2, cfg.h, th)
            h = B.dd_uot_init_moved(cfg, m, v, y, stream=stream)
        try:
            B.dd_uot_iterate(h, half_iters, stats=False)
            s = B.dd_uot_score(h, 0)
            dmu = torch.empty(n1 * n2, dtype=torch.float64, device=mu.device)
            dnu = torch.empty(n1 * n2, dtype=torch.float64, device=nu.device)
            B.dd_uot_backward(h, 0, n1, n2, out=(dmu, dnu))
            dth = None
            if theta is not None:
                dy = B.dd_uot_backward_ypos(h, 0, n1, n2)
                G = theta.shape[1]
                B1 = displacement_basis(n1, G)
                B2 = displacement_basis(n2, G)
                dth = np.stack([B1.T @ dy[..., c] @ B2 for c in range(2)])
        finally:
            B.dd_uot_destroy(h)
        ctx.save_for_backward(dmu.view(n1, n2).to(mu.dtype), dnu.view(n1, n2).to(nu.dtype))
        ctx.dth = None if dth is None else torch.from_numpy(dth).to(theta.device, theta.dtype)
        ctx.score = s
        return mu.new_tensor(s["dual"])

    @staticmethod
    def backward(ctx, gout):
        dmu, dnu = ctx.saved_tensors
        dth = None if ctx.dth is None else gout * ctx.dth
        return gout * dmu, gout * dnu, dth, None, None


def uot_value(mu: torch.Tensor, nu: torch.Tensor, cfg, half_iters: int,
              theta: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable optimal value of the unbalanced problem between mu and nu
    (n1 x n2 tensors of point masses) after `half_iters` DD half-iterations;
    theta (2, G, G): control values of the Y displacement (None: the grid)."""
    if mu.shape != (cfg.n1, cfg.n2) or nu.shape != (cfg.n1, cfg.n2):
        raise ValueError("marginals must have the grid shape of the config")
    if theta is not None and (theta.dim() != 3 or theta.shape[0] != 2 or
                              theta.shape[1] != theta.shape[2]):
        raise ValueError("theta must have shape (2, G, G)")
    return UOTValue.apply(mu, nu, theta, cfg, int(half_iters))


__all__ = ["UOTValue", "uot_value"]
