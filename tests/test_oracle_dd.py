"""Pins of the domain-decomposition oracle (Sec. 3, Sec. 4)."""
import numpy as np
import pytest

from oracle import dd, uot
from paper_2410_08859_amd.inputs import gaussian_mixture, uniform_masses


def small_problem(n=8, s=2, eps_h2=4.0, lam=1.0, seed=1, h=None):
    mu = gaussian_mixture(n, n, 3, 1e-3, 1.0, 10 * seed + 1)
    nu = gaussian_mixture(n, n, 3, 1e-3, 1.3, 10 * seed + 2)
    hh = 1.0 / n if h is None else h
    return dd.make_problem(mu, nu, eps_h2 / n ** 2, lam, hh, s)


def global_optimum(p):
    pts = uot.grid_points(p.n1, p.n2, p.h)
    C = uot.sq_cost(pts, pts)
    sol = uot.sinkhorn(p.mu, p.nu, C, p.eps, p.lam, tol=None, step_tol=1e-15)
    pi = uot.plan(sol["alpha"], sol["beta"], p.mu, p.nu, C, p.eps)
    return pi, sol, C


def test_partitions_cover_basic_cells_once():
    p = small_problem(16, 2)
    for part, ncell in (("A", 16), ("B", 25)):
        cells = dd.composite_cells(p, part)
        assert len(cells) == ncell
        ids = sorted(b for c in cells for b in c["basic"])
        assert ids == list(range(p.nb1 * p.nb2))
        for c in cells:
            o1, o2, l1, l2 = c["rect"]
            idx = set(dd.rect_index(c["rect"], p.n2).tolist())
            assert idx == set(np.concatenate([dd.rect_index(dd.basic_rect(p, b), p.n2)
                                              for b in c["basic"]]).tolist())


def test_toy_partition_has_singletons():
    mu = uniform_masses(1, 32, 1.0)
    p = dd.make_problem(mu, mu.copy(), 2.0 / 32 ** 2, 1.0, 1.0 / 32, 1, 1)
    B = dd.composite_cells(p, "B")
    assert [len(c["basic"]) for c in B] == [1] + [2] * 15 + [1]
    assert len(dd.composite_cells(p, "A")) == 16


def test_init_marginals():
    p = small_problem()
    st = dd.init_block(p)
    np.testing.assert_allclose(dd.aggregate(p, st.boxes), p.nu, rtol=1e-15)
    st = dd.init_product(p)
    np.testing.assert_allclose(dd.aggregate(p, st.boxes), p.mu.sum() * p.nu, rtol=1e-14)
    np.testing.assert_allclose(st.px, p.nu.sum() * p.mu, rtol=1e-15)


def test_block_init_piece_closed_form():
    # H_i of the block start written out: <c,pi> + eps[|nu(X_i)|(-log|mu_i| - 1) +
    # |mu_i||nu|] + lam |mu_i| (t log t - t + 1), t = |nu(X_i)|/|mu_i|
    p = small_problem(8, 2)
    st = dd.init_block(p)
    for b in range(p.nb1 * p.nb2):
        rect = dd.basic_rect(p, b)
        idx = dd.rect_index(rect, p.n2)
        m, v = p.mu.ravel()[idx], p.nu.ravel()[idx]
        C = dd.rect_cost(p, rect, rect)
        t = v.sum() / m.sum()
        h = ((C * np.outer(m, v)).sum() / m.sum()
             + p.eps * (v.sum() * (-np.log(m.sum()) - 1) + m.sum() * p.nu.sum())
             + p.lam * m.sum() * (t * np.log(t) - t + 1))
        assert st.hbar[b] == pytest.approx(h, rel=1e-13)


def test_cell_piece_formula_for_diagonal_scaling_plan():
    # For pi = exp((a + b - c)/eps) mu x nu on X_i x box:
    # <c,pi> + eps KL(pi|mu_i x nu) = <a, P_X pi> + <b, P_Y pi> - eps|pi| + eps|mu_i||nu|
    p = small_problem(8, 2)
    rng = np.random.default_rng(3)
    rect, box = (2, 2, 2, 2), (1, 0, 5, 6)
    xi, yi = dd.rect_index(rect, p.n2), dd.rect_index(box, p.n2)
    mu_x, nu_y = p.mu.ravel()[xi], p.nu.ravel()[yi]
    C = dd.rect_cost(p, rect, box)
    a = rng.normal(0, 0.01, xi.size)
    b = rng.normal(0, 0.01, yi.size)
    pi = uot.plan(a, b, mu_x, nu_y, C, p.eps)
    px, py = pi.sum(1), pi.sum(0)
    formula = ((a * px).sum() + (b * py).sum() - p.eps * pi.sum()
               + p.eps * mu_x.sum() * p.nu.sum() + p.lam * uot.kl(px, mu_x))
    definition = dd.cell_piece(pi, mu_x, nu_y, p.nu.sum(), C, p.eps, p.lam)
    assert formula == pytest.approx(definition, rel=1e-12)


def test_resplit_sums():
    p = small_problem(8, 2)
    st = dd.init_block(p)
    opt = dd.Options(margin=2, trunc=0.0)
    P = dd.aggregate(p, st.boxes)
    for cell in dd.composite_cells(p, "B"):
        r = dd.process_cell(p, cell, st.boxes, P, opt)
        tot = sum(r["cand"][b] for b in cell["basic"]).ravel()
        np.testing.assert_allclose(tot[r["dom"]], r["pi"].sum(0), rtol=1e-13)
        assert np.all(tot[~r["dom"]] == 0.0)
        for b in cell["basic"]:
            rows = np.isin(r["xi"], dd.rect_index(dd.basic_rect(p, b), p.n2))
            assert r["cand"][b].sum() == pytest.approx(r["px"][rows].sum(), rel=1e-13)


def test_global_optimum_is_a_fixed_point_of_the_cell_step():
    # nu_{-J} = P_Y pi - nu_J at the optimum: the cell problem returns pi^dagger
    # restricted to X_J x Y (Sec. 3.1, cell subproblem)
    p = small_problem(8, 2)
    pi, _, _ = global_optimum(p)
    st = dd.init_product(p)
    for b in range(p.nb1 * p.nb2):
        rows = dd.rect_index(dd.basic_rect(p, b), p.n2)
        st.boxes[b] = (0, 0, pi[rows].sum(0).reshape(p.n1, p.n2))
    opt = dd.Options(trunc=0.0, getweights="greedy", err=1e-14, max_iter=5000)
    ref = [arr.copy() for _, _, arr in st.boxes]
    dd.half_iteration(p, st, "A", opt)
    for b in range(p.nb1 * p.nb2):
        np.testing.assert_allclose(st.boxes[b][2], ref[b], rtol=1e-6, atol=1e-14)
    np.testing.assert_allclose(st.px, pi.sum(1).reshape(p.mu.shape), rtol=1e-6)


@pytest.mark.parametrize("gw", ["swift", "safe", "line", "opt"])
def test_monotone_scores(gw):
    # Safe decrement proof (Sec. 3.4): with safe weights the exact score of the
    # mixed plan never rises.  The tracked score Ebar (reading R8) bounds E from
    # above and never rises under safe or swift; swift compares tracked scores,
    # so after a safe step it may accept a greedy plan whose exact score lies
    # above the (smaller) exact score of the mixture.
    p = small_problem(8, 2)
    st = dd.init_product(p, dense_plan=True)
    opt = dd.Options(trunc=0.0, getweights=gw, err=1e-13, max_iter=5000)
    E = [dd.exact_score(p, st)]
    Eb = [dd.tracked_score(p, st)]
    assert Eb[0] == pytest.approx(E[0], rel=1e-13)
    for _ in range(8):
        dd.run(p, st, 1, opt)
        E.append(dd.exact_score(p, st))
        Eb.append(dd.tracked_score(p, st))
    E, Eb = np.array(E), np.array(Eb)
    if gw == "safe":
        assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))
    assert np.all(np.diff(Eb) <= 1e-12 * np.abs(Eb[:-1]))
    assert np.all(E <= Eb + 1e-12 * np.abs(Eb))
    if gw == "swift":
        greedy_steps = [h["theta"] == 1.0 for h in st.history]
        # after a greedy step the tracked score is exact
        for k, g in enumerate(greedy_steps):
            if g:
                assert Eb[k + 1] == pytest.approx(E[k + 1], rel=1e-11)


def test_sequential_monotone():
    p = small_problem(8, 2)
    st = dd.init_product(p, dense_plan=True)
    opt = dd.Options(trunc=0.0, err=1e-13, max_iter=5000)
    E = [dd.exact_score(p, st)]
    for _ in range(4):
        dd.run(p, st, 1, opt, sequential=True)
        E.append(dd.exact_score(p, st))
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[0]))


def test_dd_converges_to_global_optimum():
    # Props. (convergence, parallel) + unique optimum: DD limit = pi^dagger
    p = small_problem(8, 2)
    pi, sol, C = global_optimum(p)
    st = dd.init_product(p, dense_plan=True)
    opt = dd.Options(trunc=0.0, getweights="swift", err=1e-15, max_iter=20000)
    dd.run(p, st, 160, opt)
    np.testing.assert_allclose(st.plan, pi, rtol=5e-6, atol=1e-15)
    np.testing.assert_allclose(st.px.ravel(), pi.sum(1), rtol=5e-6)
    np.testing.assert_allclose(dd.aggregate(p, st.boxes).ravel(), pi.sum(0), rtol=5e-6)
    cert = dd.certificate(p, st.abar)
    W = uot.primal(pi, p.mu, p.nu, C, p.eps, p.lam)
    assert cert["rel"] < 1e-12
    assert cert["dual"] <= W * (1 + 1e-13) and cert["primal"] >= W * (1 - 1e-13)
    assert dd.tracked_score(p, st) == pytest.approx(W, rel=1e-9)


def test_certificate_gap_identity():
    # PD of the certificate pair equals E(pi_hat) - D(alpha_bar, beta_hat)
    p = small_problem(8, 2)
    st = dd.init_block(p)
    dd.run(p, st, 3, dd.Options(margin=2))
    cert = dd.certificate(p, st.abar)
    assert cert["primal"] - cert["dual"] == pytest.approx(cert["pd"], rel=1e-8)
    assert cert["pd"] > 0


def test_polished_bounds_bracket_the_optimum_and_tighten():
    # weak duality (Definition unbalanced-entropic-transport): every pair of
    # the global Sinkhorn iteration gives D <= W <= E; the iteration raises D
    # (block coordinate ascent), so more polishing never loosens the bounds,
    # and they close in on the optimal value W
    p = small_problem(8, 2)
    _, sol, C = global_optimum(p)
    W = uot.dual(sol["alpha"], sol["beta"], p.mu, p.nu, C, p.eps, p.lam)
    st = dd.init_block(p)
    dd.run(p, st, 3, dd.Options(margin=2, trunc=0.0, err=1e-6, max_iter=2000))
    gaps = []
    prev_d, prev_e = -np.inf, np.inf
    for m in (0, 2, 10, 200):
        c = dd.certificate(p, st.abar, polish=m)
        assert c["dual_polished"] <= W * (1 + 1e-12) + 1e-15
        assert c["primal_polished"] >= W * (1 - 1e-12) - 1e-15
        assert c["dual_polished"] >= prev_d - 1e-15 and c["primal_polished"] <= prev_e + 1e-15
        if m == 0:
            assert c["dual_polished"] == c["dual"] and c["primal_polished"] == c["primal"]
        prev_d, prev_e = c["dual_polished"], c["primal_polished"]
        gaps.append((c["primal_polished"] - c["dual_polished"]) / abs(W))
    assert gaps[-1] < 1e-6 * gaps[0] and gaps[-1] < 1e-9


def test_zero_cost_dd_reaches_product_plan():
    # h = 0 makes c = 0; the optimum is s mu x nu, s = (|mu||nu|)^(-lam/(eps+2lam))
    p = small_problem(8, 2, h=0.0)
    p.eps = 4.0 / 64
    st = dd.init_product(p, dense_plan=True)
    dd.run(p, st, 40, dd.Options(trunc=0.0, err=1e-15, max_iter=20000))
    s = (p.mu.sum() * p.nu.sum()) ** (-p.lam / (p.eps + 2 * p.lam))
    # the cell stopping rule bounds KL(P_X pi | e^{-alpha/lam} mu) <= Err |mu_J|,
    # which is quadratic in the relative marginal error: Err = 1e-15 leaves
    # up to sqrt(2e-15) ~ 4.5e-8 (a warm-started cell at the fixed point stops
    # at its first check)
    np.testing.assert_allclose(st.plan, s * np.outer(p.mu.ravel(), p.nu.ravel()), rtol=5e-8)


def toy(gw, iters):
    # Sec. 4.2 toy: N = 32 on {0, 1/N, ..}, mu = nu uniform, lam = 1, eps = 2/N^2,
    # A = pairs, B = staggered with two singletons, start mu x nu
    N = 32
    mu = uniform_masses(1, N, 1.0)
    p = dd.make_problem(mu, mu.copy(), 2.0 / N ** 2, 1.0, 1.0 / N, 1, 1)
    st = dd.init_product(p, dense_plan=True)
    opt = dd.Options(trunc=0.0, getweights=gw, err=1e-7, max_iter=1500)
    E = [dd.exact_score(p, st)]
    for _ in range(iters):
        dd.run(p, st, 1, opt)
        E.append(dd.exact_score(p, st))
    return np.array(E), p


def test_toy_getweights_behaviour():
    # Sec. 4.2: greedy does not converge (cells overshoot together and the
    # score rises), safe is very slow, swift makes steady progress.
    # Qualitative only: the paper's figures carry no numbers.
    Eg, p = toy("greedy", 4)
    Es, _ = toy("safe", 8)
    Ew, _ = toy("swift", 8)
    pts = uot.grid_points(p.n1, p.n2, p.h)
    C = uot.sq_cost(pts, pts)
    sol = uot.sinkhorn(p.mu, p.nu, C, p.eps, p.lam, tol=None, step_tol=1e-14)
    W = uot.primal(uot.plan(sol["alpha"], sol["beta"], p.mu, p.nu, C, p.eps),
                   p.mu, p.nu, C, p.eps, p.lam)
    gap_g, gap_s, gap_w = Eg - W, Es - W, Ew - W
    assert np.any(np.diff(Eg) > 0)             # greedy raises the score
    assert gap_w[-1] < 0.1 * gap_w[0]          # swift converges
    assert gap_s[-1] > 3 * gap_w[-1]           # safe lags behind
    assert gap_g[-1] > 10 * gap_w[-1]          # greedy does not converge


def test_translation_shift_is_the_line_maximiser_and_keeps_the_solution():
    p = small_problem(16, 4, eps_h2=1.0, lam=1.0)
    st = dd.init_block(p)
    opt = dd.Options(margin=2)
    P = dd.aggregate(p, st.boxes)
    cell = dd.composite_cells(p, "A")[1]
    box = dd.cell_box(p, cell, st.boxes, opt)
    xi, yi = dd.rect_index(cell["rect"], p.n2), dd.rect_index(box, p.n2)
    mu_x, nu_y = p.mu.ravel()[xi], p.nu.ravel()[yi]
    C = dd.rect_cost(p, cell["rect"], box)
    r, beta0, _ = dd.cell_inputs(p, cell, box, st.boxes, P)
    alpha = uot.x_update(beta0, nu_y, C, p.eps, p.lam)
    s = dd.translation_shift(alpha, beta0, mu_x, nu_y, r, p.lam)
    D = lambda d_: uot.dual(alpha + s + d_, beta0 - s - d_, mu_x, nu_y, C, p.eps, p.lam, r * nu_y)
    for d_ in (1e-3, -1e-3, 1e-5, -1e-5):
        assert D(d_) <= D(0.0)
    assert D(0.0) >= uot.dual(alpha, beta0, mu_x, nu_y, C, p.eps, p.lam, r * nu_y)
    # same converged cell solution with and without the step
    sols = []
    for tr in (False, True):
        o = dd.Options(margin=2, translate=tr, err=1e-14, max_iter=200000)
        sols.append(dd.solve_cell(mu_x, nu_y, r, beta0, C, p.eps, p.lam, 1e-14 * mu_x.sum(), o))
    assert sols[1]["iters"] < sols[0]["iters"]
    np.testing.assert_allclose(sols[1]["px"], sols[0]["px"], rtol=1e-6)


def test_dd_with_displaced_support_converges_to_global_optimum():
    # moved Y points y' (cost |x - y'|^2, no longer separable): the DD limit is
    # still the unique optimum of the global problem with the same cost
    from paper_2410_08859_amd.inputs import displaced_points, displacement_theta
    n = 8
    p0 = small_problem(n, 2)
    y = displaced_points(n, n, 1.0 / n, displacement_theta(53, 1.0 / n))
    p = dd.make_problem(p0.mu, p0.nu, p0.eps, p0.lam, p0.h, 2, ypos=y)
    C = dd.full_cost(p)
    pts = uot.grid_points(n, n, p.h)
    np.testing.assert_allclose(C, uot.sq_cost(pts, y.reshape(-1, 2)))
    assert not np.allclose(C, uot.sq_cost(pts, pts))
    sol = uot.sinkhorn(p.mu, p.nu, C, p.eps, p.lam, tol=None, step_tol=1e-15)
    pi = uot.plan(sol["alpha"], sol["beta"], p.mu, p.nu, C, p.eps)
    st = dd.init_product(p, dense_plan=True)
    opt = dd.Options(trunc=0.0, getweights="swift", err=1e-15, max_iter=20000,
                     translate=True)
    dd.run(p, st, 160, opt)
    np.testing.assert_allclose(st.plan, pi, rtol=5e-6, atol=1e-15)
    cert = dd.certificate(p, st.abar)
    assert cert["rel"] < 1e-12


def _coarse_pair(n=16, s=2):
    pf = small_problem(n, s)
    pc = dd.make_problem(dd.coarsen(pf.mu), dd.coarsen(pf.nu), pf.eps * 4, pf.lam, pf.h * 2, s)
    return pc, pf


def test_refined_product_plan_is_the_fine_product_plan():
    # mu_c x nu_c split in proportion to the fine masses is mu_f x nu_f
    pc, pf = _coarse_pair()
    st = dd.refine(pc, dd.init_product(pc), pf, 0.0)
    ref = dd.init_product(pf)
    np.testing.assert_allclose(st.px, ref.px, rtol=1e-13)
    for (a1, a2, a), (b1, b2, b) in zip(st.boxes, ref.boxes):
        assert (a1, a2, a.shape) == (b1, b2, b.shape)
        np.testing.assert_allclose(a, b, rtol=1e-13)
    assert st.force_greedy


def test_refined_block_start_with_double_cell_is_the_fine_block_start():
    # cell side doubles: one fine basic cell per coarse one, nu on the block
    pf = small_problem(16, 4)
    pc = dd.make_problem(dd.coarsen(pf.mu), dd.coarsen(pf.nu), pf.eps * 4, pf.lam, pf.h * 2, 2)
    st = dd.refine(pc, dd.init_block(pc), pf, 0.0)
    ref = dd.init_block(pf)
    np.testing.assert_allclose(st.px, ref.px, rtol=1e-13)
    for (a1, a2, a), (b1, b2, b) in zip(st.boxes, ref.boxes):
        assert (a1, a2, a.shape) == (b1, b2, b.shape)
        np.testing.assert_allclose(a, b, rtol=1e-13)


def test_refinement_keeps_mass_and_the_prolonged_y_marginal():
    pc, pf = _coarse_pair()
    stc = dd.init_block(pc)
    dd.run(pc, stc, 3, dd.Options(margin=2, trunc=0.0, translate=True))
    st = dd.refine(pc, stc, pf, 0.0)
    Pc = dd.aggregate(pc, stc.boxes)
    Pf = dd.aggregate(pf, st.boxes)
    np.testing.assert_allclose(dd.coarsen(Pf), Pc, rtol=1e-12)
    np.testing.assert_allclose(Pf, np.kron(Pc / pc.nu, np.ones((2, 2))) * pf.nu, rtol=1e-12)
    assert st.px.sum() == pytest.approx(stc.px.sum(), rel=1e-13)


@pytest.mark.parametrize("part", ["A", "B"])
def test_staggered_batches_partition_the_cells_without_neighbours(part):
    p = small_problem(24, 2)   # 12 basic cells per axis: B has border singletons
    batches = dd.staggered_batches(p, part)
    cells = dd.composite_cells(p, part)
    got = sorted(tuple(c["basic"]) for b in batches for c in b)
    assert got == sorted(tuple(c["basic"]) for c in cells)
    for b in batches:
        for i, c in enumerate(b):
            for d in b[i + 1:]:
                (a1, a2, l1, l2), (b1, b2, m1, m2) = c["rect"], d["rect"]
                # rectangles of one batch do not touch (not even at a corner)
                assert a1 + l1 < b1 or b1 + m1 < a1 or a2 + l2 < b2 or b2 + m2 < a2


def test_staggered_scores_decrease_and_reach_the_optimum():
    p = small_problem(8, 2)
    pi, sol, C = global_optimum(p)
    st = dd.init_product(p, dense_plan=True)
    opt = dd.Options(trunc=0.0, getweights="staggered", err=1e-15, max_iter=20000,
                     lenience=0.0)
    prev = dd.tracked_score(p, st)
    for _ in range(120):
        out = dd.half_iteration(p, st, "A" if st.k % 2 == 0 else "B", opt)
        assert len(out) == 4
        cur = dd.tracked_score(p, st)
        assert cur <= prev + 1e-12 * abs(prev)
        prev = cur
    np.testing.assert_allclose(st.plan, pi, rtol=5e-6, atol=1e-15)
    assert dd.certificate(p, st.abar)["rel"] < 1e-12


# ---- global Sinkhorn warm start and potential-based refinement (R11) --------
def test_interpolated_potential_is_exact_for_affine_potentials():
    # a coarse potential sampled at the block centres 2I + 1/2 of an affine
    # function gives that affine function at every fine point, also past the
    # first and last centres (linear continuation)
    nc1, nc2 = 5, 7
    I1, I2 = np.meshgrid(np.arange(nc1), np.arange(nc2), indexing="ij")
    f = lambda u, v: 0.3 - 1.7 * u + 0.45 * v
    ac = f(2 * I1 + 0.5, 2 * I2 + 0.5)
    af = dd.interpolate_potential(ac, 2 * nc1, 2 * nc2)
    i1, i2 = np.meshgrid(np.arange(2 * nc1), np.arange(2 * nc2), indexing="ij")
    np.testing.assert_allclose(af, f(i1, i2), rtol=0, atol=1e-13)
    # a single coarse point: constant
    np.testing.assert_array_equal(dd.interpolate_potential(np.full((1, 3), 2.5), 2, 6), 2.5)


def test_interpolated_potential_keeps_the_coarse_values_between_centres():
    # midway between two centres the value is their mean; a nonlinear coarse
    # potential is reproduced at the centres' neighbours with weights 3/4, 1/4
    rng = np.random.default_rng(5)
    ac = rng.normal(size=(4, 4))
    af = dd.interpolate_potential(ac, 8, 8)
    # fine index 2I + 1 lies 1/4 of the way from centre I to centre I + 1
    np.testing.assert_allclose(af[3, 5], (0.75 * (0.75 * ac[1, 2] + 0.25 * ac[1, 3]) +
                                          0.25 * (0.75 * ac[2, 2] + 0.25 * ac[2, 3])), rtol=1e-14)


def test_state_from_optimal_potentials_has_the_optimal_score():
    # the plan of the optimal pair split by basic cells: the tracked score is
    # the exact primal of that plan, which equals the optimal dual value
    # (strong duality, Sec. 2.2), and the marginals are the plan's
    p = small_problem(8, 2)
    pi, sol, C = global_optimum(p)
    st = dd.init_from_duals(p, sol["alpha"].reshape(8, 8), sol["beta"].reshape(8, 8), 0.0)
    assert st.force_greedy
    E = uot.primal(pi, p.mu, p.nu, C, p.eps, p.lam)
    D = uot.dual(sol["alpha"], sol["beta"], p.mu, p.nu, C, p.eps, p.lam)
    assert dd.tracked_score(p, st) == pytest.approx(E, rel=1e-12)
    assert dd.tracked_score(p, st) == pytest.approx(D, rel=1e-9)
    np.testing.assert_allclose(st.px, pi.sum(1).reshape(8, 8), rtol=1e-12)
    np.testing.assert_allclose(dd.aggregate(p, st.boxes), pi.sum(0).reshape(8, 8), rtol=1e-12)


def test_state_from_potentials_truncates_and_boxes_tightly():
    p = small_problem(16, 4, eps_h2=1.0)
    pi, sol, C = global_optimum(p)
    a, b = sol["alpha"].reshape(16, 16), sol["beta"].reshape(16, 16)
    trunc = 1e-9
    st = dd.init_from_duals(p, a, b, trunc)
    for bi, (o1, o2, arr) in enumerate(st.boxes):
        full = pi[dd.rect_index(dd.basic_rect(p, bi), p.n2)].sum(0).reshape(16, 16)
        kept = arr > 0
        assert np.all(arr[kept] >= trunc)
        np.testing.assert_allclose(arr[kept], full[o1:o1 + arr.shape[0], o2:o2 + arr.shape[1]][kept],
                                   rtol=1e-13)
        # the box is the bbox of the entries >= trunc, whatever its size
        big = full >= trunc
        r1, r2 = np.nonzero(big)
        assert (o1, o2, arr.shape) == (r1.min(), r2.min(),
                                       (r1.max() + 1 - r1.min(), r2.max() + 1 - r2.min()))
        assert np.count_nonzero(kept) == np.count_nonzero(big)
    # px is the X-marginal of the kept cell plans: at most the full row sums
    assert np.all(st.px <= pi.sum(1).reshape(16, 16) * (1 + 1e-13))


def test_optimal_state_is_a_fixed_point_of_a_dd_half_iteration():
    # optimal plan split by cells (Sec. 3: pi^dagger is a fixed point of
    # DomDecIter): a greedy half-iteration from it keeps it
    p = small_problem(8, 2)
    pi, sol, C = global_optimum(p)
    st = dd.init_from_duals(p, sol["alpha"].reshape(8, 8), sol["beta"].reshape(8, 8), 0.0)
    ref = [arr.copy() for _, _, arr in st.boxes]
    opt = dd.Options(trunc=0.0, getweights="greedy", err=1e-14, max_iter=5000)
    out = dd.half_iteration(p, st, "B", opt)
    assert out["theta"] == 1.0
    P = dd.aggregate(p, st.boxes)
    np.testing.assert_allclose(P, pi.sum(0).reshape(8, 8), rtol=1e-6)
    for (o1, o2, arr), r in zip(st.boxes, ref):
        assert np.abs(arr).sum() == pytest.approx(r.sum(), rel=1e-6)


def _mixed_tracked(p, st, cells, res, theta, P, Pg):
    """Tracked score of the mixture with weight theta (untruncated): the
    pieces and the aggregated Y-marginal are linear in theta."""
    hb = st.hbar.copy()
    for c, r in zip(cells, res):
        if r is None:
            continue
        for b in c["basic"]:
            hb[b] = (1 - theta) * st.hbar[b] + theta * r["pieces"][b]
    return float(hb.sum()) + p.lam * uot.kl((1 - theta) * P + theta * Pg, p.nu)


def test_line_weight_minimises_the_tracked_score_of_the_mixture():
    # GetWeights line (Proposition converging-getweights, reading R12): the
    # weight is the minimiser over [1/n, 1] of the mixture's tracked score, so
    # it does at least as well as both swift candidates and as any nearby
    # weight (checked by evaluating the score itself, not its derivative)
    p = small_problem(16, 2, eps_h2=2.0)
    st = dd.init_product(p)
    opt = dd.Options(trunc=0.0, err=1e-12, max_iter=3000, margin=2)
    dd.run(p, st, 1, dd.Options(trunc=0.0, err=1e-12, max_iter=3000, margin=2,
                                getweights="greedy"))
    found_interior = False
    for part in ("B", "A", "B"):
        cells = dd.composite_cells(p, part)
        P = dd.aggregate(p, st.boxes)
        res = [dd.process_cell(p, c, st.boxes, P, opt, st.abar, st.warm) for c in cells]
        cand = list(st.boxes)
        for c, r in zip(cells, res):
            for b in c["basic"]:
                cand[b] = dd.truncate_to_box(r["box"][0], r["box"][1], r["cand"][b], 0.0)
        Pg = dd.aggregate(p, cand)
        n = len(res)
        dH = sum(r["pieces"][b] - st.hbar[b] for c, r in zip(cells, res) for b in c["basic"])
        z = dd.line_weight(p, P, Pg, dH, n)
        assert 1.0 / n <= z <= 1.0
        f = lambda th: _mixed_tracked(p, st, cells, res, th, P, Pg)
        fz = f(z)
        assert fz <= f(1.0 / n) + 1e-13 * abs(fz) and fz <= f(1.0) + 1e-13 * abs(fz)
        if 1.0 / n < z < 1.0:
            found_interior = True
            for dz in (1e-3, 1e-5):
                assert fz <= f(min(z + dz, 1.0)) + 1e-13 * abs(fz)
                assert fz <= f(max(z - dz, 1.0 / n)) + 1e-13 * abs(fz)
        dd.half_iteration(p, st, part, dd.Options(trunc=0.0, err=1e-12, max_iter=3000,
                                                   margin=2, getweights="line"))
        assert st.history[-1]["theta"] == pytest.approx(z, rel=1e-12)
    assert found_interior


def test_opt_weights_minimise_the_tracked_score_of_the_mixture():
    # GetWeights opt (eq. opt-weights-problem, reading R14): the per-cell
    # weights minimise the mixture's tracked score over [1/n, 1]^J, so they do
    # at least as well as the uniform line weight, greedy and safe, satisfy
    # the bound-constrained optimality conditions, and no single weight can be
    # moved to improve (checked on the score itself)
    p = small_problem(16, 2, eps_h2=2.0)
    st = dd.init_product(p)
    opt = dd.Options(trunc=0.0, err=1e-12, max_iter=3000, margin=2)
    dd.run(p, st, 1, dd.Options(trunc=0.0, err=1e-12, max_iter=3000, margin=2,
                                getweights="greedy"))
    for part in ("B", "A"):
        cells = dd.composite_cells(p, part)
        P = dd.aggregate(p, st.boxes)
        res = [dd.process_cell(p, c, st.boxes, P, opt, st.abar, st.warm) for c in cells]
        deltas, dHs = [], []
        for c, r in zip(cells, res):
            dl = np.zeros((p.n1, p.n2))
            for b in c["basic"]:
                o1, o2, arr = dd.truncate_to_box(r["box"][0], r["box"][1], r["cand"][b], 0.0)
                if arr.size:
                    dl[o1:o1 + arr.shape[0], o2:o2 + arr.shape[1]] += arr
                o1, o2, arr = st.boxes[b]
                if arr.size:
                    dl[o1:o1 + arr.shape[0], o2:o2 + arr.shape[1]] -= arr
            deltas.append(dl)
            dHs.append(sum(r["pieces"][b] - st.hbar[b] for b in c["basic"]))
        n = len(cells)
        D = np.stack([x.ravel() for x in deltas])
        dH = np.array(dHs)
        f = lambda th: float(th @ dH) + p.lam * uot.kl(P.ravel() + th @ D, p.nu.ravel())
        z = dd.line_weight(p, P, P + D.sum(0).reshape(P.shape), float(dH.sum()), n)
        th = dd.opt_weights(p, P, deltas, dHs, n, z)
        fz = f(th)
        for ref in (np.full(n, z), np.ones(n), np.full(n, 1.0 / n)):
            assert fz <= f(ref) + 1e-13 * abs(fz)
        g = dH + p.lam * (D @ (np.log(P.ravel() + th @ D) - np.log(p.nu.ravel())))
        scale = np.abs(dH).max()
        lo, hi = th <= 1.0 / n + 1e-12, th >= 1.0 - 1e-12
        assert np.all(g[lo] >= -1e-7 * scale) and np.all(g[hi] <= 1e-7 * scale)
        mid = ~lo & ~hi
        assert np.all(np.abs(g[mid]) <= 1e-7 * scale)
        rng = np.random.default_rng(5)
        for J in rng.choice(n, 6, replace=False):
            for dz in (1e-3, -1e-3):
                t2 = th.copy()
                t2[J] = min(1.0, max(1.0 / n, t2[J] + dz))
                assert fz <= f(t2) + 1e-13 * abs(fz)
        assert np.ptp(th) > 0      # the weights differ between cells
        dd.half_iteration(p, st, part, dd.Options(trunc=0.0, err=1e-12, max_iter=3000, margin=2,
                                                   getweights="opt"))
        np.testing.assert_allclose(st.history[-1]["thetas"], th, rtol=1e-12, atol=0)


def test_balancing_moves_mass_horizontally_to_the_targets():
    # Sec. 4.1 "Balancing" (reading R13): nu_J is kept pointwise, every basic
    # cell ends with m_i = mubar(X_i) |nu_J| / mubar(X_J), where mubar is the
    # X-marginal after one more X-half, and a receiver's column at y is its
    # kernel column e^{(alpha - c)/eps} mu restricted to its rows, rescaled
    p = small_problem(16, 2, eps_h2=1.0)
    st = dd.init_block(p)
    P = dd.aggregate(p, st.boxes)
    # a solve stopped early leaves P_X away from mubar, so there is mass to move
    opt = dd.Options(trunc=0.0, err=1e-10, max_iter=3, margin=2, translate=True)
    cell = dd.composite_cells(p, "A")[5]
    plain = dd.process_cell(p, cell, st.boxes, P, opt)
    opt.balance = True
    bal = dd.process_cell(p, cell, st.boxes, P, opt)
    basics = cell["basic"]
    tot = sum(plain["cand"][b].sum() for b in basics)
    np.testing.assert_allclose(sum(bal["cand"][b] for b in basics),
                               sum(plain["cand"][b] for b in basics), rtol=1e-12, atol=1e-300)
    C = dd.rect_cost(p, cell["rect"], plain["box"])[:, plain["dom"]]
    mu_x = p.mu.ravel()[plain["xi"]]
    nu_y = p.nu.ravel()[plain["yi"]]
    a2 = uot.x_update(plain["beta"], nu_y, C, p.eps, p.lam)
    mubar = np.exp(-a2 / p.lam) * mu_x
    moved = False
    for b in basics:
        rows = np.isin(plain["xi"], dd.rect_index(dd.basic_rect(p, b), p.n2))
        target = mubar[rows].sum() * tot / mubar.sum()
        assert bal["cand"][b].sum() == pytest.approx(target, rel=1e-11)
        moved |= abs(plain["cand"][b].sum() - target) > 1e-6 * target
        gain = (bal["pi"][rows] - plain["pi"][rows]).sum(0)
        if np.all(gain >= 0) and gain.sum() > 0:
            # receiver: the added mass follows the kernel column of its rows
            lk = (plain["alpha"][rows][:, None] - C[rows]) / p.eps + np.log(mu_x[rows])[:, None]
            k = np.exp(lk - lk.max(0)[None, :])
            np.testing.assert_allclose(bal["pi"][rows] - plain["pi"][rows],
                                       gain[None, :] * k / k.sum(0)[None, :], rtol=1e-9,
                                       atol=1e-14 * plain["pi"][rows].max())
        # P_X and the pieces follow the balanced plan
        np.testing.assert_allclose(bal["px"][rows], bal["pi"][rows].sum(1), rtol=1e-12)
    assert moved
