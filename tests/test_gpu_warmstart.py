"""Global Sinkhorn warm start on the GPU against the oracle (reading R11):
the global UOT Sinkhorn, the potential interpolation, the DD state built from
a pair of potentials, and the multiscale driver with global layers."""
import numpy as np
import pytest

from oracle import dd, uot
from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.inputs import gaussian_mixture

pytestmark = pytest.mark.gpu


def marg(n, seed, mass=1.0):
    return gaussian_mixture(n, n, 3, 1e-3, mass, seed)


def gcfg(n, eps, s=2, cap=32, precision=64):
    return B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=eps, lam=1.0, cell=s,
                                   precision=precision, init=B.INIT_BLOCK, lenience=0.0,
                                   box_cap=cap, box_margin=2, trunc=1e-15, fixed_inner_iters=20)


def dense_cost(n):
    pts = uot.grid_points(n, n, 1.0 / n)
    return uot.sq_cost(pts, pts)


@pytest.mark.parametrize("iters,tol", [(30, 0.0), (5000, 1e-7)])
def test_global_sinkhorn_matches_oracle(iters, tol):
    n = 24
    mu, nu = marg(n, 901), marg(n, 902, 1.3)
    eps = 2.0 / n ** 2
    rng = np.random.default_rng(903)
    beta0 = 0.01 * rng.normal(size=(n, n))
    print(f"[warmstart] global sinkhorn n={n} iters={iters} tol={tol}", flush=True)
    got = B.dd_uot_global_sinkhorn(gcfg(n, eps), mu, nu, beta0, max_iter=iters, tol=tol)
    ref = uot.sinkhorn(mu, nu, dense_cost(n), eps, 1.0, tol=tol, max_iter=iters,
                       beta0=beta0, step_tol=-1.0)
    assert got["iters"] == ref["iters"]
    sa = np.abs(ref["alpha"]).max()
    np.testing.assert_allclose(got["alpha"].ravel(), ref["alpha"], rtol=0, atol=1e-11 * sa)
    np.testing.assert_allclose(got["beta"].ravel(), ref["beta"], rtol=0, atol=1e-11 * sa)
    assert got["pd"] == pytest.approx(ref["pd"], rel=1e-8, abs=1e-14)
    if tol > 0:
        assert got["pd"] <= tol


def test_interpolation_matches_oracle():
    rng = np.random.default_rng(904)
    for shape in [(7, 5), (1, 4), (16, 16)]:
        ac = rng.normal(size=shape)
        print(f"[warmstart] interpolate {shape}", flush=True)
        got = B.dd_uot_interpolate_potential(ac)
        ref = dd.interpolate_potential(ac, 2 * shape[0], 2 * shape[1])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14 * np.abs(ac).max())


def compare_states(h, p, st, tol=1e-10, label=""):
    px, py = B.dd_uot_marginals(h, 0, p.n1, p.n2)
    np.testing.assert_allclose(px, st.px, rtol=0, atol=tol * st.px.max(), err_msg=label)
    P = dd.aggregate(p, st.boxes)
    np.testing.assert_allclose(py, P, rtol=0, atol=tol * P.max(), err_msg=label)
    for b in range(p.nb1 * p.nb2):
        o1, o2, arr = B.dd_uot_basic_marginal(h, 0, b)
        r1, r2, ref = st.boxes[b]
        if ref.size == 0:
            assert arr.size == 0, f"{label} basic cell {b}"
            continue
        assert (o1, o2, arr.shape) == (r1, r2, ref.shape), f"{label} box of basic cell {b}"
        np.testing.assert_allclose(arr, ref, rtol=0, atol=tol * ref.max(), err_msg=label)


@pytest.mark.parametrize("cap", [32, 9])
def test_state_from_potentials_matches_oracle(cap):
    n, s = 32, 4
    mu, nu = marg(n, 911), marg(n, 912, 1.3)
    eps = 1.0 / n ** 2
    sol = uot.sinkhorn(mu, nu, dense_cost(n), eps, 1.0, tol=1e-9, max_iter=3000)
    a, b = sol["alpha"].reshape(n, n), sol["beta"].reshape(n, n)
    c = gcfg(n, eps, s, cap)
    p = dd.make_problem(mu, nu, eps, 1.0, 1.0 / n, s)
    print(f"[warmstart] init_duals n={n} s={s} cap={cap}", flush=True)
    h = B.dd_uot_init_duals(c, mu, nu, a, b)
    try:
        st = dd.init_from_duals(p, a, b, 1e-15)
        compare_states(h, p, st, label="init")
        # the in-LDS layout only decides where a cell's arrays live: with side
        # 9 the wider boxes are solved from the cell workspace, no box is cut
        wide = sum(1 for _, _, arr in st.boxes if arr.size and max(arr.shape) > 9)
        print(f"[warmstart] {wide} basic boxes wider than 9", flush=True)
        assert wide > 0
        s_gpu = B.dd_uot_score(h, 0)
        assert s_gpu["tracked"] == pytest.approx(dd.tracked_score(p, st), rel=1e-11)
        # the first (greedy) half-iteration follows the oracle
        B.dd_uot_iterate(h, 1)
        opt = dd.Options(fixed_iters=20, lenience=0.0, margin=2, trunc=1e-15,
                         translate=True)
        out = dd.half_iteration(p, st, "A", opt)
        assert out["theta"] == 1.0
        compare_states(h, p, st, tol=1e-9, label="after one half-iteration")
    finally:
        B.dd_uot_destroy(h)


def oracle_multiscale_global(mu, nu, c, ms):
    """The driver's schedule with global layers, written with the oracle's
    pieces (uot.sinkhorn per eps stage, interpolate_potential for the next
    layer's warm beta, init_from_duals on the last global layer, refine,
    DD half-iterations, certificate)."""
    L = ms.levels
    mus, nus = [mu], [nu]
    for _ in range(L - 1):
        mus.insert(0, dd.coarsen(mus[0]))
        nus.insert(0, dd.coarsen(nus[0]))
    first = 0
    while first < L - 1 and mus[first].shape[0] < ms.dd_from:
        first += 1
    mass = mu.sum()
    alpha = beta = None
    p = st = None
    for l in range(first):
        n = mus[l].shape[0]
        h = c.h * 2 ** (L - 1 - l)
        C = uot.sq_cost(uot.grid_points(n, n, h), uot.grid_points(n, n, h))
        beta = np.zeros(n * n) if l == 0 else \
            dd.interpolate_potential(beta.reshape(n // 2, n // 2), n, n).ravel()
        e, e_end = ms.eps_start_h2 * h * h, ms.eps_end_h2 * h * h
        while True:
            sol = uot.sinkhorn(mus[l], nus[l], C, e, c.lambda_, tol=ms.global_tol * mass,
                               max_iter=ms.global_max_iter, beta0=beta, step_tol=-1.0)
            alpha, beta = sol["alpha"], sol["beta"]
            if e <= e_end * (1 + 1e-12):
                break
            e = max(e * 0.5, e_end)
        if l == first - 1:
            p = dd.make_problem(mus[l], nus[l], e, c.lambda_, h, min(c.cell, ms.coarse_cell))
            st = dd.init_from_duals(p, alpha.reshape(n, n), beta.reshape(n, n), c.trunc)
    trace = []
    for l in range(first, L):
        n = mus[l].shape[0]
        h = c.h * 2 ** (L - 1 - l)
        fin = l == L - 1
        s = c.cell if fin else min(c.cell, ms.coarse_cell)
        opt = dd.Options(err=c.sinkhorn_err, max_iter=c.sinkhorn_max_iter if fin else
                         max(c.sinkhorn_max_iter, ms.coarse_max_iter), trunc=c.trunc,
                         lenience=c.lenience if fin else ms.coarse_lenience,
                         margin=c.box_margin, getweights="swift", translate=True)
        pn = dd.make_problem(mus[l], nus[l], ms.eps_start_h2 * h * h, c.lambda_, h, s)
        st = dd.refine(p, st, pn, c.trunc)
        p = pn
        e_end = c.eps if fin else ms.eps_end_h2 * h * h
        e = p.eps
        while True:
            done = 0
            while True:
                dd.run(p, st, ms.halves_per_stage, opt)
                done += ms.halves_per_stage
                if done + ms.halves_per_stage > ms.stage_max_halves:
                    break
                if dd.certificate(p, st.abar)["rel"] <= ms.stage_gap:
                    break
            if e <= e_end * (1 + 1e-12):
                break
            e = max(e * 0.5, e_end)
            dd.set_eps(p, st, e)
        if fin:
            trace.append(dd.certificate(p, st.abar)["rel"])
            done = 0
            while trace[-1] > ms.target_rel_gap and done < ms.final_max_halves:
                k = min(ms.check_every, ms.final_max_halves - done)
                dd.run(p, st, k, opt)
                done += k
                trace.append(dd.certificate(p, st.abar)["rel"])
    return p, st, trace


def test_multiscale_with_global_layers_follows_the_oracle():
    n = 32
    mu, nu = marg(n, 931), marg(n, 932, 1.3)
    c = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=1.0 / n ** 2, lam=1.0, cell=4,
                                precision=64, box_cap=32, sinkhorn_max_iter=200, lenience=0.0)
    ms = B.dd_uot_default_multiscale(levels=3, coarse_cell=2, dd_from=16, global_max_iter=60,
                                     global_tol=1e-7, final_max_halves=8, check_every=4,
                                     target_rel_gap=1e-12, stage_max_halves=8,
                                     coarse_max_iter=400)
    print("[warmstart] multiscale 8 (global) -> 16 -> 32 against the oracle", flush=True)
    h, tr = B.dd_uot_solve_multiscale(c, ms, mu, nu)
    try:
        p, st, otr = oracle_multiscale_global(mu, nu, c, ms)
        print(tr, otr, flush=True)
        assert tr.shape[0] == len(otr)
        np.testing.assert_allclose(tr[:, 2], otr, rtol=1e-6)
        compare_states(h, p, st, tol=1e-8, label="final")
    finally:
        B.dd_uot_destroy(h)
