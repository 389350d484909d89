"""Seeded synthetic marginals shared by the tests, the bench and the oracle checks.

This module holds no arithmetic of the transport method: it only draws the
input measures.  The paper evaluates on Gaussian-mixture images on [0,1]^2
with random means, variances and magnitudes (Sec. 4.4, "Test data"); those
images are not available, so the same kind of measure is drawn here from a
seeded NumPy PCG64 generator:

    f(x) = sum_k w_k exp(-|x - m_k|^2 / (2 sigma_k^2)),
    m_k ~ U([0.1, 0.9]^2),  sigma_k ~ U(0.03, 0.15),  w_k ~ U(0.2, 1),

evaluated at the grid points x = h (i1, i2), h = 1/n, then normalised to
max f = 1, lifted by a constant floor (so that every point carries mass, as
the full-support assumption of Sec. 3.2 requires) and scaled to a total mass.
"""
from __future__ import annotations

import numpy as np


def gaussian_mixture(n1: int, n2: int, components: int, floor: float,
                     mass: float, seed: int) -> np.ndarray:
    """Return an (n1, n2) float64 array of point masses summing to `mass`."""
    if n1 <= 0 or n2 <= 0:
        raise ValueError("grid sides must be positive")
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(0.1, 0.9, size=(components, 2))
    sigmas = rng.uniform(0.03, 0.15, size=components)
    weights = rng.uniform(0.2, 1.0, size=components)
    x1 = np.arange(n1, dtype=np.float64) / n1
    x2 = np.arange(n2, dtype=np.float64) / n2
    f = np.zeros((n1, n2), dtype=np.float64)
    for k in range(components):
        g1 = np.exp(-(x1 - means[k, 0]) ** 2 / (2.0 * sigmas[k] ** 2))
        g2 = np.exp(-(x2 - means[k, 1]) ** 2 / (2.0 * sigmas[k] ** 2))
        f += weights[k] * np.outer(g1, g2)
    f /= f.max()
    f += floor
    f *= mass / f.sum()
    return f


def uniform_masses(n1: int, n2: int, mass: float) -> np.ndarray:
    """Homogeneous measure on the grid (the toy problem of Sec. 4.2 uses it)."""
    return np.full((n1, n2), mass / (n1 * n2), dtype=np.float64)


# Workloads used throughout the tests and the bench.  Seeds follow the rule
# mu-seed = 10 c + 1, nu-seed = 10 c + 2 for workload number c.
WORKLOADS = {
    "grid32": dict(n=32, components=3, floor=1e-3, mass_mu=1.0, mass_nu=1.3,
                   lam=1.0, eps_h2=4.0, cell=4, seed=1),
    "grid256": dict(n=256, components=3, floor=1e-3, mass_mu=1.0, mass_nu=0.8,
                    lam=1.0, eps_h2=1.0, cell=4, seed=2),
    "grid1024": dict(n=1024, components=10, floor=1e-4, mass_mu=1.0, mass_nu=1.5,
                     lam=1.0, eps_h2=1.0, cell=8, seed=3),
    "grid512": dict(n=512, components=3, floor=1e-3, mass_mu=1.0, mass_nu=1.0,
                    lam=1.0, eps_h2=1.0, cell=4, seed=5),
}


def workload_marginals(name: str, n: int | None = None):
    """(mu, nu) for a named workload; `n` overrides the grid side."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    c = w["seed"]
    mu = gaussian_mixture(n, n, w["components"], w["floor"], w["mass_mu"], 10 * c + 1)
    nu = gaussian_mixture(n, n, w["components"], w["floor"], w["mass_nu"], 10 * c + 2)
    return mu, nu


def batched_problems(count: int = 64, seed: int = 4999, sides=(64, 128, 256, 512)):
    """Independent problems with sides drawn from `sides` and lambda log-uniform
    in [0.1, 10]; problem k uses seeds 4000+2k and 4001+2k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        n = int(rng.choice(np.asarray(sides)))
        lam = float(10.0 ** rng.uniform(-1.0, 1.0))
        mu = gaussian_mixture(n, n, 3, 1e-3, 1.0, 4000 + 2 * k)
        nu = gaussian_mixture(n, n, 3, 1e-3, 1.0, 4001 + 2 * k)
        out.append(dict(n=n, lam=lam, mu=mu, nu=nu))
    return out


# --------------------------------------------------------------------------
# Displaced Y support: y' = y + u_theta(y) with a smooth seeded field
# --------------------------------------------------------------------------
def cubic_bspline(t: np.ndarray) -> np.ndarray:
    """Centred uniform cubic B-spline kernel (support |t| < 2, partition of unity)."""
    a = np.abs(np.asarray(t, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a < 1.0
    m2 = (a >= 1.0) & (a < 2.0)
    out[m1] = 2.0 / 3.0 - a[m1] ** 2 + 0.5 * a[m1] ** 3
    out[m2] = (2.0 - a[m2]) ** 3 / 6.0
    return out


def displacement_basis(n: int, controls: int = 8) -> np.ndarray:
    """(n, controls) matrix B with B[i, a] the weight of control point a at the
    grid coordinate i/n: uniform cubic B-spline on [0, 1] with `controls`
    control points, the first and last lying one knot spacing outside [0, 1]
    (spacing 1/(controls - 3)), so that the rows sum to 1."""
    if controls < 4:
        raise ValueError("a cubic B-spline needs at least 4 control points")
    step = 1.0 / (controls - 3)
    x = np.arange(n, dtype=np.float64) / n
    a = np.arange(controls, dtype=np.float64)
    return cubic_bspline((x[:, None] - (a[None, :] - 1.0) * step) / step)


def displacement_theta(seed: int, h: float, controls: int = 8) -> np.ndarray:
    """Seeded control values theta, shape (2, controls, controls), U(-2h, 2h)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-2.0 * h, 2.0 * h, size=(2, controls, controls))


def displaced_points(n1: int, n2: int, h: float, theta: np.ndarray) -> np.ndarray:
    """y' = h (j1, j2) + u_theta(j), u_c = B1 theta_c B2^T; shape (n1, n2, 2).
    Since the basis rows sum to 1 and are nonnegative, |u_c| <= max |theta_c|."""
    G = theta.shape[1]
    B1 = displacement_basis(n1, G)
    B2 = displacement_basis(n2, G)
    j1, j2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    y = np.stack([h * j1, h * j2], axis=-1).astype(np.float64)
    y[..., 0] += B1 @ theta[0] @ B2.T
    y[..., 1] += B1 @ theta[1] @ B2.T
    return y
