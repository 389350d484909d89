"""Gradients of the optimal UOT value (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

The optimal value W(mu, nu) = E(pi^dagger) = D(alpha^dagger, beta^dagger)
(Theorem existence-global-solution: unique primal optimum, dual optimality).
By the envelope theorem the derivative with respect to a point mass is the
partial derivative of the dual functional D of Definition
unbalanced-entropic-transport at the optimal pair:

  dW/dmu(x) = eps |nu| - eps P_X pi(x)/mu(x) - lam (exp(-alpha(x)/lam) - 1)
  dW/dnu(y) = eps |mu| - eps P_Y pi(y)/nu(y) - lam (exp(-beta(y)/lam) - 1)

and for a moved support point y' (cost c(x,y') = |x - y'|^2), differentiating
the primal at the optimal plan gives dW/dy' = sum_x pi(x,y') 2 (y' - x).
Pinned by central finite differences of the converged dense Sinkhorn value.
"""
from __future__ import annotations

import numpy as np

from . import uot


def grads_from_pair(alpha, beta, pi, mu, nu, eps, lam):
    """(dW/dmu, dW/dnu) from an optimal pair and its plan."""
    mu = np.ravel(mu)
    nu = np.ravel(nu)
    px, py = pi.sum(1), pi.sum(0)
    dmu = eps * nu.sum() - eps * px / mu - lam * (np.exp(-np.ravel(alpha) / lam) - 1.0)
    dnu = eps * mu.sum() - eps * py / nu - lam * (np.exp(-np.ravel(beta) / lam) - 1.0)
    return dmu, dnu


def grad_ypos(pi, xs, ys):
    """dW/dy' = sum_x pi(x, y') 2 (y' - x), shape (ny, 2)."""
    py = pi.sum(0)
    m = pi.T @ xs
    return 2.0 * (ys * py[:, None] - m)


def solve_value(mu, nu, xs, ys, eps, lam, tol=None):
    """Converged dense Sinkhorn: returns (W, alpha, beta, pi)."""
    c = uot.sq_cost(xs, ys)
    sol = uot.sinkhorn(mu, nu, c, eps, lam, tol=tol)
    pi = uot.plan(sol["alpha"], sol["beta"], mu, nu, c, eps)
    return uot.primal(pi, mu, nu, c, eps, lam), sol["alpha"], sol["beta"], pi
