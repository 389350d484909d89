"""Pins of the global-problem oracle against facts fixed by the paper and by
mathematics (closed forms, identities, limits, brute force)."""
import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.special import kl_div, logsumexp

from oracle import uot, grad


def test_kl_matches_library_integrand():
    rng = np.random.default_rng(0)
    p = rng.uniform(0, 2, 50)
    q = rng.uniform(0.1, 2, 50)
    p[3] = 0.0
    assert uot.kl(p, q) == pytest.approx(kl_div(p, q).sum(), rel=1e-14)
    # p/q below the double range must not turn the divergence into -inf
    assert uot.kl([1e-244], [1e240]) == pytest.approx(1e240, rel=1e-12)


def _two_dirac_closed_form(m1, m2, c, eps, lam):
    # dE/dp = c + eps log(p/(m1 m2)) + lam log(p/m1) + lam log(p/m2) = 0
    p = np.exp(((eps + lam) * np.log(m1 * m2) - c) / (eps + 2 * lam))
    return p, -lam * np.log(p / m1), -lam * np.log(p / m2)


@pytest.mark.parametrize("m1,m2,c,eps,lam", [(1.0, 1.3, 0.2, 0.05, 1.0),
                                             (0.4, 2.0, 1.5, 0.3, 0.7),
                                             (2.0, 2.0, 0.0, 1.0, 10.0)])
def test_two_dirac_closed_form(m1, m2, c, eps, lam):
    p, a, b = _two_dirac_closed_form(m1, m2, c, eps, lam)
    C = np.array([[c]])
    sol = uot.sinkhorn(np.array([m1]), np.array([m2]), C, eps, lam, tol=None)
    pi = uot.plan(sol["alpha"], sol["beta"], [m1], [m2], C, eps)
    assert pi[0, 0] == pytest.approx(p, rel=1e-12)
    assert sol["alpha"][0] == pytest.approx(a, rel=1e-10, abs=1e-12)
    assert sol["beta"][0] == pytest.approx(b, rel=1e-10, abs=1e-12)
    E = uot.primal(pi, [m1], [m2], C, eps, lam)
    D = uot.dual(sol["alpha"], sol["beta"], [m1], [m2], C, eps, lam)
    assert E == pytest.approx(D, rel=1e-11)


def test_zero_cost_product_plan():
    # c = 0: pi = s mu x nu with s = (|mu||nu|)^(-lam/(eps+2 lam))
    rng = np.random.default_rng(1)
    mu = rng.uniform(0.5, 1.5, 7)
    mu /= mu.sum()
    nu = rng.uniform(0.5, 1.5, 5)
    nu *= 1.3 / nu.sum()
    eps, lam = 4.0 / 1024, 1.0
    C = np.zeros((7, 5))
    sol = uot.sinkhorn(mu, nu, C, eps, lam, tol=None)
    pi = uot.plan(sol["alpha"], sol["beta"], mu, nu, C, eps)
    s = (mu.sum() * nu.sum()) ** (-lam / (eps + 2 * lam))
    assert s == pytest.approx(0.8772, abs=5e-4)
    np.testing.assert_allclose(pi, s * np.outer(mu, nu), rtol=1e-11)


def test_newton_quadratic_case_lambda_equals_eps():
    # lam = eps: e^q = r + e^(z - q)  ->  e^q = (r + sqrt(r^2 + 4 e^z)) / 2
    rng = np.random.default_rng(2)
    z = rng.uniform(-30, 30, 200)
    r = np.exp(rng.uniform(-40, 5, 200))
    eps = lam = 0.37
    beta, _ = uot.y_update_root(z, np.log(r), eps, lam)
    q = np.log((r + np.sqrt(r * r + 4 * np.exp(z))) / 2)
    np.testing.assert_allclose(-beta / lam, q, rtol=1e-13, atol=1e-13)


def test_newton_without_background_is_closed_form():
    # r = 0: beta = -eps/(1+eps/lam) z (eq. sinkhorn-iters-ot)
    z = np.linspace(-500, 500, 101)
    eps, lam = 1e-6, 1.0
    beta, _ = uot.y_update_root(z, np.full(z.shape, -np.inf), eps, lam)
    np.testing.assert_allclose(beta, -eps / (1 + eps / lam) * z, rtol=1e-15, atol=0)


@pytest.mark.parametrize("K", [1e-3, 1.0, 1e3, 1e6])
def test_newton_root_residual_and_monotone(K):
    rng = np.random.default_rng(3)
    z = rng.uniform(-20, 20, 500) * max(1.0, np.log10(K + 1))
    lr = rng.uniform(-40, 3, 500)
    eps, lam = 1.0, K
    beta, steps = uot.y_update_root(z, lr, eps, lam)
    q = -beta / lam
    # residual of eq. (proxdiv-problem): log[r + exp(beta/eps + z)] + beta/lam = 0
    res = np.logaddexp(lr, beta / eps + z) + beta / lam
    assert np.max(np.abs(res) / (1 + np.abs(q))) < 1e-12
    assert steps < 200


def _random_problem(n, m, seed, mass_mu=1.0, mass_nu=1.3):
    rng = np.random.default_rng(seed)
    xs = rng.uniform(0, 1, (n, 2))
    ys = rng.uniform(0, 1, (m, 2))
    mu = rng.uniform(0.2, 1, n)
    nu = rng.uniform(0.2, 1, m)
    return xs, ys, mu * mass_mu / mu.sum(), nu * mass_nu / nu.sum()


def test_pd_identity_with_background():
    # After an exact Y-update, E(pi|nu_-) - D(alpha,beta|nu_-) =
    # lam KL(P_X pi | exp(-alpha/lam) mu)   (eq. PD-gap / PD-gap-KL)
    xs, ys, mu, nu = _random_problem(9, 11, 4)
    rng = np.random.default_rng(5)
    nu_minus = rng.uniform(0, 0.2, 11) * nu
    C = uot.sq_cost(xs, ys)
    eps, lam = 0.05, 0.8
    alpha = rng.normal(0, 0.1, 9)
    z = uot.y_log_integral(alpha, mu, C, eps)
    beta, _ = uot.y_update_root(z, np.log(nu_minus / nu), eps, lam)
    pi = uot.plan(alpha, beta, mu, nu, C, eps)
    E = uot.primal(pi, mu, nu, C, eps, lam, nu_minus)
    D = uot.dual(alpha, beta, mu, nu, C, eps, lam, nu_minus)
    assert E - D == pytest.approx(uot.pd_gap_kl(alpha, pi.sum(1), mu, lam), rel=1e-9)
    # and the Y optimality condition eq. (optimality-conditions-KL)
    np.testing.assert_allclose(np.exp(-beta / lam), (pi.sum(0) + nu_minus) / nu, rtol=1e-12)


def test_brute_force_small_problem():
    # minimise E over log pi with a generic quasi-Newton method (no Sinkhorn)
    xs, ys, mu, nu = _random_problem(4, 4, 6)
    C = uot.sq_cost(xs, ys)
    eps, lam = 0.1, 0.5
    prod = np.outer(mu, nu)

    def f(lv):
        pi = np.exp(lv.reshape(4, 4))
        px, py = pi.sum(1), pi.sum(0)
        val = ((C * pi).sum() + eps * (pi * (lv.reshape(4, 4) - np.log(prod)) - pi + prod).sum()
               + lam * (px * np.log(px / mu) - px + mu).sum()
               + lam * (py * np.log(py / nu) - py + nu).sum())
        g = pi * (C + eps * (lv.reshape(4, 4) - np.log(prod))
                  + lam * np.log(px / mu)[:, None] + lam * np.log(py / nu)[None, :])
        return val, g.ravel()

    res = minimize(f, np.log(prod).ravel(), jac=True, method="L-BFGS-B",
                   options=dict(ftol=1e-16, gtol=1e-13, maxiter=20000))
    sol = uot.sinkhorn(mu, nu, C, eps, lam, tol=None)
    pi = uot.plan(sol["alpha"], sol["beta"], mu, nu, C, eps)
    assert res.fun == pytest.approx(uot.primal(pi, mu, nu, C, eps, lam), rel=1e-9)
    np.testing.assert_allclose(np.exp(res.x.reshape(4, 4)), pi, rtol=2e-5)


def test_swap_symmetry():
    xs, ys, mu, nu = _random_problem(6, 8, 7)
    C = uot.sq_cost(xs, ys)
    eps, lam = 0.08, 2.0
    s1 = uot.sinkhorn(mu, nu, C, eps, lam, tol=None)
    s2 = uot.sinkhorn(nu, mu, C.T, eps, lam, tol=None)
    p1 = uot.plan(s1["alpha"], s1["beta"], mu, nu, C, eps)
    p2 = uot.plan(s2["alpha"], s2["beta"], nu, mu, C.T, eps)
    np.testing.assert_allclose(p1, p2.T, rtol=1e-9)
    assert uot.primal(p1, mu, nu, C, eps, lam) == pytest.approx(
        uot.primal(p2, nu, mu, C.T, eps, lam), rel=1e-12)


def _balanced_sinkhorn(mu, nu, C, eps, iters=20000):
    # textbook log-domain balanced Sinkhorn (independent of the oracle)
    f = np.zeros(mu.size)
    g = np.zeros(nu.size)
    for _ in range(iters):
        f = -eps * logsumexp((g[None, :] - C) / eps + np.log(nu)[None, :], axis=1)
        g = -eps * logsumexp((f[:, None] - C) / eps + np.log(mu)[:, None], axis=0)
    return np.exp((f[:, None] + g[None, :] - C) / eps) * np.outer(mu, nu)


def test_balanced_limit():
    xs, ys, mu, nu = _random_problem(6, 6, 8, 1.0, 1.0)
    C = uot.sq_cost(xs, ys)
    eps = 0.3
    ref = _balanced_sinkhorn(mu, nu, C, eps, iters=3000)
    errs = []
    for lam in (10.0, 100.0, 1000.0):
        sol = uot.sinkhorn(mu, nu, C, eps, lam, tol=None, max_iter=400000, step_tol=1e-13)
        pi = uot.plan(sol["alpha"], sol["beta"], mu, nu, C, eps)
        errs.append(np.abs(pi - ref).sum())
    assert errs[2] < 2e-4
    # O(1/lambda): a factor 10 in lambda shrinks the error by about 10
    assert 5 < errs[0] / errs[1] < 20 and 5 < errs[1] / errs[2] < 20


def test_envelope_gradients_match_finite_differences():
    xs, ys, mu, nu = _random_problem(5, 6, 9)
    eps, lam = 0.1, 0.7
    W, a, b, pi = grad.solve_value(mu, nu, xs, ys, eps, lam)
    dmu, dnu = grad.grads_from_pair(a, b, pi, mu, nu, eps, lam)
    dy = grad.grad_ypos(pi, xs, ys)
    rng = np.random.default_rng(10)
    for _ in range(3):
        xi_m = rng.normal(size=mu.size)
        xi_n = rng.normal(size=nu.size)
        xi_y = rng.normal(size=ys.shape)
        t = 1e-5
        wp = grad.solve_value(mu * (1 + t * xi_m), nu * (1 + t * xi_n), xs, ys + t * xi_y, eps, lam)[0]
        wm = grad.solve_value(mu * (1 - t * xi_m), nu * (1 - t * xi_n), xs, ys - t * xi_y, eps, lam)[0]
        fd = (wp - wm) / (2 * t)
        an = (dmu * mu * xi_m).sum() + (dnu * nu * xi_n).sum() + (dy * xi_y).sum()
        assert fd == pytest.approx(an, rel=1e-6, abs=1e-9)
