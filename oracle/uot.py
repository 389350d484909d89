"""Global entropic unbalanced OT with D1 = D2 = lambda*KL (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Everything here is the plain definition from the paper:
  * KL with the "+1" term, eq. (KL) in Sec. 2.1;
  * primal E(pi | nu_-) of Definition (unbalanced-entropic-transport), Sec. 2.2;
  * dual D(alpha, beta | nu_-) of the same definition, with the conjugate of
    lambda*phi_KL, (lambda phi)^*(z) = lambda (e^{z/lambda} - 1);
  * the closed-form Sinkhorn updates eq. (sinkhorn-iters-ot) for nu_- = 0;
  * the cell Y-update eq. (proxdiv-problem), solved per point by Newton;
  * the primal-dual gap eq. (PD-gap-KL).
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp


def kl(p, q) -> float:
    """KL(p|q) = sum [p log(p/q) - p + q] with 0 log 0 = 0 (eq. KL, Sec. 2.1).

    Pinned against scipy.special.kl_div, which evaluates the same integrand.
    """
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if np.any(q <= 0):
        # p must vanish where q does (absolute continuity), else +inf.
        if np.any(p[q <= 0] > 0):
            return np.inf
    out = q - p
    pos = p > 0
    out = out.copy()
    out[pos] += p[pos] * (np.log(p[pos]) - np.log(q[pos]))
    return float(out.sum())


def grid_points(n1: int, n2: int, h: float) -> np.ndarray:
    """Coordinates x = h (i1, i2) of an n1 x n2 grid, row-major, shape (n1*n2, 2)."""
    i1, i2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    return h * np.stack([i1.ravel(), i2.ravel()], axis=1).astype(np.float64)


def sq_cost(xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """c(x, y) = |x - y|^2, the cost used in all experiments (Sec. 4.1)."""
    d = xs[:, None, :] - ys[None, :, :]
    return np.einsum("ijk,ijk->ij", d, d)


def primal(pi, mu, nu, c, eps, lam, nu_minus=None) -> float:
    """E(pi | nu_-) = <c,pi> + eps KL(pi|mu x nu) + lam KL(P_X pi|mu)
    + lam KL(P_Y pi + nu_- | nu)   (Definition unbalanced-entropic-transport)."""
    pi = np.asarray(pi, dtype=np.float64)
    mu = np.ravel(mu)
    nu = np.ravel(nu)
    nm = 0.0 if nu_minus is None else np.ravel(nu_minus)
    prod = np.outer(mu, nu)
    return (float((c * pi).sum()) + eps * kl(pi, prod)
            + lam * kl(pi.sum(1), mu) + lam * kl(pi.sum(0) + nm, nu))


def dual(alpha, beta, mu, nu, c, eps, lam, nu_minus=None) -> float:
    """D(alpha, beta | nu_-) (Definition unbalanced-entropic-transport), with
    phi_i^*(-a) = lam (exp(-a/lam) - 1) for D_i = lam KL."""
    mu = np.ravel(mu)
    nu = np.ravel(nu)
    alpha = np.ravel(alpha)
    beta = np.ravel(beta)
    dens = np.exp((alpha[:, None] + beta[None, :] - c) / eps)
    val = eps * float(((1.0 - dens) * np.outer(mu, nu)).sum())
    val -= float((lam * (np.exp(-alpha / lam) - 1.0) * mu).sum())
    val -= float((lam * (np.exp(-beta / lam) - 1.0) * nu).sum())
    if nu_minus is not None:
        val -= float((beta * np.ravel(nu_minus)).sum())
    return val


def plan(alpha, beta, mu, nu, c, eps) -> np.ndarray:
    """pi = exp((alpha (+) beta - c)/eps) mu x nu, eq. (sinkhorn-primal)."""
    return np.exp((np.ravel(alpha)[:, None] + np.ravel(beta)[None, :] - c) / eps) \
        * np.outer(np.ravel(mu), np.ravel(nu))


def x_update(beta, nu, c, eps, lam) -> np.ndarray:
    """alpha(x) = -eps/(1+eps/lam) log int exp((beta - c(x,.))/eps) dnu,
    eq. (sinkhorn-iters-ot), identical to eq. (sinkhorn-X-iteration)."""
    kappa = lam / (lam + eps)
    t = (np.ravel(beta)[None, :] - c) / eps + np.log(np.ravel(nu))[None, :]
    return -eps * kappa * logsumexp(t, axis=1)


def y_log_integral(alpha, mu, c, eps) -> np.ndarray:
    """z(y) = log int exp((alpha - c(., y))/eps) dmu, defined in Sec. 4.1."""
    t = (np.ravel(alpha)[:, None] - c) / eps + np.log(np.ravel(mu))[:, None]
    return logsumexp(t, axis=0)


def y_update_root(z, log_r, eps, lam, max_steps: int = 200):
    """Solve eq. (proxdiv-problem) pointwise for beta.

    The equation log[r + exp(beta/eps + z)] + beta/lam = 0 is rewritten with
    q = -beta/lam as  q = logaddexp(log r, z - K q),  K = lam/eps.
    F(q) = logaddexp(log r, z - K q) - q is convex and strictly decreasing, and
    q* >= q0 = max(log r, z/(1+K)) (if q < log r then e^q < r; if q < z/(1+K)
    then z - Kq > q), so Newton started at q0 increases monotonically to the
    root.  Iterated until the step falls below 1e-15 (1 + |q|).

    For r = 0 (log r = -inf) the root is q = z/(1+K), i.e. beta = -eps kappa z,
    the closed form of eq. (sinkhorn-iters-ot).

    Returns (beta, steps_taken).
    """
    z = np.asarray(z, dtype=np.float64)
    lr = np.broadcast_to(np.asarray(log_r, dtype=np.float64), z.shape)
    K = lam / eps
    q = np.maximum(lr, z / (1.0 + K))
    active = np.ones(z.shape, dtype=bool)
    steps = 0
    for steps in range(1, max_steps + 1):
        w = z - K * q
        la = np.logaddexp(lr, w)
        F = la - q
        sig = np.exp(w - la)
        dq = F / (1.0 + K * sig)
        dq = np.where(active, dq, 0.0)
        q = q + dq
        active = active & (np.abs(dq) > 1e-15 * (1.0 + np.abs(q)))
        if not active.any():
            break
    return -lam * q, steps


def pd_gap_kl(alpha, px, mu, lam) -> float:
    """PD = lam KL(P_X pi | exp(-alpha/lam) mu), eq. (PD-gap-KL)."""
    return lam * kl(px, np.exp(-np.ravel(alpha) / lam) * np.ravel(mu))


def sinkhorn(mu, nu, c, eps, lam, tol=1e-13, max_iter=100000, beta0=None,
             nu_minus=None, step_tol=1e-15):
    """Dense log-domain unbalanced Sinkhorn (Definition sinkhorn; Sec. 4.1).

    alpha from eq. (sinkhorn-X-iteration); beta from eq. (sinkhorn-Y-iteration)
    through `y_update_root` (with nu_- = 0 this is eq. sinkhorn-iters-ot).
    Stops when PD/lam <= tol, PD from eq. (PD-gap-KL) evaluated for the pair
    (alpha^l, beta^l) (its P_X comes from the next X-half), or when alpha is
    stationary to `step_tol` relative (the KL gap is quadratic in the error,
    so tight pins pass tol=None and use this second rule).
    Returns dict(alpha, beta, iters, pd).
    """
    mu = np.ravel(mu).astype(np.float64)
    nu = np.ravel(nu).astype(np.float64)
    beta = np.zeros(nu.shape) if beta0 is None else np.ravel(beta0).astype(np.float64)
    if nu_minus is None:
        lr = np.full(nu.shape, -np.inf)
    else:
        with np.errstate(divide="ignore"):
            lr = np.log(np.ravel(nu_minus) / nu)
    alpha = x_update(beta, nu, c, eps, lam)
    pd = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        z = y_log_integral(alpha, mu, c, eps)
        beta, _ = y_update_root(z, lr, eps, lam)
        alpha_next = x_update(beta, nu, c, eps, lam)
        px = plan(alpha, beta, mu, nu, c, eps).sum(1)
        pd = pd_gap_kl(alpha, px, mu, lam) / lam
        if tol is not None and pd <= tol:
            break
        moved = np.max(np.abs(alpha_next - alpha)) / (1.0 + np.max(np.abs(alpha)))
        alpha = alpha_next
        if moved <= step_tol:
            break
    return dict(alpha=alpha, beta=beta, iters=it, pd=pd)
