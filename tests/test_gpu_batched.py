"""Several independent problems of different sizes in one handle: every launch
covers all problems' cells, GetWeights decides per problem.  Each problem must
follow its own oracle trajectory, and match a handle that holds it alone."""
import numpy as np
import pytest

from oracle import dd
from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.inputs import batched_problems, gaussian_mixture

pytestmark = pytest.mark.gpu

SPECS = [  # (n, s, lam, eps_h2, init)
    (16, 2, 0.5, 4.0, B.INIT_PRODUCT),
    (32, 4, 1.0, 4.0, B.INIT_PRODUCT),
    (32, 4, 5.0, 2.0, B.INIT_PRODUCT),
    (24, 2, 2.0, 3.0, B.INIT_PRODUCT),
]


def problem_data(k, n):
    mu = gaussian_mixture(n, n, 3, 1e-3, 1.0, 700 + 2 * k)
    nu = gaussian_mixture(n, n, 3, 1e-3, 1.2, 701 + 2 * k)
    return mu, nu


def make_cfgs(precision, fixed=8, balance=(0, 0, 0, 0)):
    cfgs = []
    for (n, s, lam, e, init), bal in zip(SPECS, balance):
        cfgs.append(B.dd_uot_default_config(
            n1=n, n2=n, h=1.0 / n, eps=e / n ** 2, lam=lam, cell=s, precision=precision,
            init=init, fixed_inner_iters=fixed, lenience=0.0, box_cap=32, getweights=B.GW_SWIFT,
            balance=bal))
    return cfgs


@pytest.mark.parametrize("balance", [(0, 0, 0, 0), (1, 0, 1, 1)])
def test_batched_fp64_follows_each_oracle(balance):
    # balance: per problem; a handle mixing both runs the balancing kernel
    # variant, which leaves the problems without it untouched
    cfgs = make_cfgs(64, balance=balance)
    data = [problem_data(k, c.n1) for k, c in enumerate(cfgs)]
    h = B.dd_uot_init_batch(cfgs, [d[0] for d in data], [d[1] for d in data])
    try:
        assert B.dd_uot_num_problems(h) == len(cfgs)
        probs, states = [], []
        for k, c in enumerate(cfgs):
            p = dd.make_problem(data[k][0], data[k][1], c.eps, c.lambda_, c.h, c.cell)
            probs.append(p)
            states.append(dd.init_product(p))
        opts = [dd.Options(fixed_iters=8, lenience=0.0, trunc=1e-15, margin=2, translate=True,
                           balance=bool(b)) for b in balance]
        for step in range(4):
            print(f"[batched] step {step}", flush=True)
            B.dd_uot_iterate(h, 1)
            for k, (p, st) in enumerate(zip(probs, states)):
                ost = dd.half_iteration(p, st, "A" if step % 2 == 0 else "B", opts[k])
                rec = B.dd_uot_history(h, k)[-1]
                assert rec[0] == ost["theta"]
                assert rec[1] == pytest.approx(ost["e_cur"], rel=1e-10)
                assert rec[2] == pytest.approx(ost["e_greedy"], rel=1e-10)
                px, py = B.dd_uot_marginals(h, k, p.n1, p.n2)
                np.testing.assert_allclose(px, st.px, rtol=0, atol=1e-10 * st.px.max())
                P = dd.aggregate(p, st.boxes)
                np.testing.assert_allclose(py, P, rtol=0, atol=1e-10 * P.max())
    finally:
        B.dd_uot_destroy(h)


def test_batched_matches_single_handles_fp32():
    cfgs = make_cfgs(32)
    data = [problem_data(k, c.n1) for k, c in enumerate(cfgs)]
    hb = B.dd_uot_init_batch(cfgs, [d[0] for d in data], [d[1] for d in data])
    singles = [B.dd_uot_init(c, d[0], d[1]) for c, d in zip(cfgs, data)]
    try:
        B.dd_uot_iterate(hb, 5)
        for k, hs in enumerate(singles):
            B.dd_uot_iterate(hs, 5)
            n = cfgs[k].n1
            pb = B.dd_uot_marginals(hb, k, n, n)
            ps = B.dd_uot_marginals(hs, 0, n, n)
            # the same arithmetic per cell and a deterministic (fixed-point)
            # aggregation: the batched handle reproduces each single handle
            for a, b in zip(pb, ps):
                np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * b.max())
            np.testing.assert_allclose(B.dd_uot_history(hb, k)[:, :3], B.dd_uot_history(hs, 0)[:, :3],
                                       rtol=1e-12)
    finally:
        B.dd_uot_destroy(hb)
        for hs in singles:
            B.dd_uot_destroy(hs)


def test_batched_workload_64_problems_runs():
    # the batched workload: 64 problems, sides 64..512, lambda in [0.1, 10], FP32
    probs = batched_problems(64)
    cfgs = [B.dd_uot_default_config(n1=q["n"], n2=q["n"], h=1.0 / q["n"], eps=1.0 / q["n"] ** 2,
                                    lam=q["lam"], cell=4, precision=32, sinkhorn_max_iter=50,
                                    box_cap=48) for q in probs]
    h = B.dd_uot_init_batch(cfgs, [q["mu"] for q in probs], [q["nu"] for q in probs])
    try:
        st = B.dd_uot_iterate(h, 4)
        assert st["n_cells"] > 0
        assert st["n_overflow"] == sum(B.dd_uot_history(h, k)[:, 7].sum() for k in range(64))
        for k in (0, 17, 63):
            s = B.dd_uot_score(h, k)
            assert np.isfinite(s["tracked"]) and s["pd_gap"] >= -1e-12 * abs(s["dual"])
            assert abs(s["mass_x"] - s["mass_y"]) <= 1e-5 * s["mass_x"]
    finally:
        B.dd_uot_destroy(h)


def test_graph_replays_match_eager_steps():
    # hipGraph of an A+B pair replayed between eager work (scores, odd
    # counts, an eps change); every replay must match the eager handle
    cfgs = make_cfgs(64)
    data = [problem_data(k, c.n1) for k, c in enumerate(cfgs)]
    he = B.dd_uot_init_batch(cfgs, [d[0] for d in data], [d[1] for d in data])
    hg = B.dd_uot_init_batch(cfgs, [d[0] for d in data], [d[1] for d in data])
    B.dd_uot_set_graph(hg, True)
    try:
        for chunk in (2, 3, 4, 1, 2):
            print(f"[graph] chunk {chunk}", flush=True)
            B.dd_uot_iterate(he, chunk)
            B.dd_uot_iterate(hg, chunk)
            if chunk == 4:
                for h in (he, hg):
                    B.dd_uot_set_eps(h, 1, 0.8 * cfgs[1].eps)
            for k, c in enumerate(cfgs):
                n = c.n1
                se, sg = B.dd_uot_score(he, k), B.dd_uot_score(hg, k)
                assert sg["half_iters"] == se["half_iters"]
                assert sg["tracked"] == pytest.approx(se["tracked"], rel=1e-12)
                for a, b in zip(B.dd_uot_marginals(hg, k, n, n), B.dd_uot_marginals(he, k, n, n)):
                    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * b.max())
                np.testing.assert_allclose(B.dd_uot_history(hg, k), B.dd_uot_history(he, k),
                                           rtol=1e-12, atol=0)
    finally:
        B.dd_uot_destroy(he)
        B.dd_uot_destroy(hg)


@pytest.mark.parametrize("balance", [0, 1])
def test_autotuned_threads_per_cell_keep_the_trajectory(balance):
    # the autotuner picks 64, 128 or 256 threads per cell for tiles of at
    # most 64 points; any choice must follow the same trajectory
    cfgs = make_cfgs(64, balance=(balance,) * 4)
    data = [problem_data(k, c.n1) for k, c in enumerate(cfgs)]
    ha = B.dd_uot_init_batch(cfgs, [d[0] for d in data], [d[1] for d in data])
    hb = B.dd_uot_init_batch(cfgs, [d[0] for d in data], [d[1] for d in data])
    try:
        B.dd_uot_iterate(ha, 1)
        B.dd_uot_iterate(hb, 1)
        nt, ms = B.dd_uot_autotune(ha)
        print(f"[autotune] chose {nt} threads, ms {ms}", flush=True)
        assert nt in (64, 128, 256) and ms[[64, 128, 256].index(nt)] >= 0
        assert np.all(ms >= 0)   # every size is admissible for tiles of <= 64 points
        B.dd_uot_iterate(ha, 4)
        B.dd_uot_iterate(hb, 4)
        for k, c in enumerate(cfgs):
            n = c.n1
            for a, b in zip(B.dd_uot_marginals(ha, k, n, n), B.dd_uot_marginals(hb, k, n, n)):
                np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * b.max())
            np.testing.assert_allclose(B.dd_uot_history(ha, k)[:, :3], B.dd_uot_history(hb, k)[:, :3],
                                       rtol=1e-12)
    finally:
        B.dd_uot_destroy(ha)
        B.dd_uot_destroy(hb)


@pytest.mark.parametrize("precision,balance", [(64, 0), (32, 0), (64, 1)])
def test_two_launch_tiers_keep_the_trajectory(precision, balance):
    # cells whose Y-box exceeds fast_cap run in a second launch with the
    # larger LDS layout; the arithmetic is the same, so the trajectory is too
    cfgs = make_cfgs(precision, balance=(balance,) * 4)
    tiered = []
    for c in make_cfgs(precision, balance=(balance,) * 4):
        c.fast_cap = 12
        tiered.append(c)
    data = [problem_data(k, c.n1) for k, c in enumerate(cfgs)]
    ha = B.dd_uot_init_batch(cfgs, [d[0] for d in data], [d[1] for d in data])
    hb = B.dd_uot_init_batch(tiered, [d[0] for d in data], [d[1] for d in data])
    try:
        print(f"[tiers] FP{precision} caps {B.dd_uot_launch_caps(ha)} vs {B.dd_uot_launch_caps(hb)}",
              flush=True)
        assert B.dd_uot_launch_caps(hb) == (12, 32)
        fa, ca = B.dd_uot_launch_caps(ha)
        assert ca == 32 and 1 <= fa <= 32
        B.dd_uot_iterate(ha, 6)
        B.dd_uot_iterate(hb, 6)
        # the same arithmetic in both handles (fixed-point aggregation)
        tol = 1e-12
        wide = 0
        for k, c in enumerate(cfgs):
            n = c.n1
            for a, b in zip(B.dd_uot_marginals(ha, k, n, n), B.dd_uot_marginals(hb, k, n, n)):
                np.testing.assert_allclose(a, b, rtol=0, atol=tol * b.max())
            np.testing.assert_allclose(B.dd_uot_history(ha, k)[:, :3], B.dd_uot_history(hb, k)[:, :3],
                                       rtol=tol, atol=0)
            for b in range(0, (n // c.cell) ** 2):
                o1, o2, arr = B.dd_uot_basic_marginal(hb, k, b)
                wide += int(max(arr.shape, default=0) > 12)
        assert wide > 0   # the second tier had cells to solve
    finally:
        B.dd_uot_destroy(ha)
        B.dd_uot_destroy(hb)


def test_three_problems_of_the_batched_workload_follow_their_oracles():
    # the bench's batched workload (64 problems, sides 64..512, lambda in
    # [0.1, 10], eps = h^2, FP32, GetWeights line): one half-iteration of
    # the whole batch; problems 3, 20 and 25 (64^2, lambda 0.67, 9.3, 0.13)
    # against the FP64 oracle, within the FP32 bound (1e-5 relative)
    probs = batched_problems(64)
    cfgs = [B.dd_uot_default_config(n1=q["n"], n2=q["n"], h=1.0 / q["n"], eps=1.0 / q["n"] ** 2,
                                    lam=q["lam"], cell=4, precision=32, sinkhorn_max_iter=100,
                                    box_cap=48, getweights=B.GW_LINE, lenience=0.0) for q in probs]
    h = B.dd_uot_init_batch(cfgs, [q["mu"] for q in probs], [q["nu"] for q in probs])
    try:
        print("[batched] one half-iteration of 64 problems", flush=True)
        B.dd_uot_iterate(h, 1)
        for k in (3, 20, 25):
            q, c = probs[k], cfgs[k]
            n = q["n"]
            assert n == 64
            p = dd.make_problem(q["mu"], q["nu"], c.eps, c.lambda_, c.h, c.cell)
            st = dd.init_block(p)
            opt = dd.Options(err=c.sinkhorn_err, max_iter=c.sinkhorn_max_iter, trunc=c.trunc,
                             lenience=0.0, margin=c.box_margin, getweights="line", translate=True)
            out = dd.half_iteration(p, st, "A", opt)
            rec = B.dd_uot_history(h, k)[-1]
            print(f"[batched] problem {k}: lambda {q['lam']:.3g} theta {rec[0]:.6g} / "
                  f"{out['theta']:.6g}, inner {rec[4]:.0f} / {out['point_iters']}", flush=True)
            assert rec[3] == out["n_updated"]
            assert rec[0] == pytest.approx(out["theta"], rel=1e-5)
            assert rec[1] == pytest.approx(out["e_cur"], rel=1e-5)
            assert rec[2] == pytest.approx(out["e_greedy"], rel=1e-5)
            px, py = B.dd_uot_marginals(h, k, n, n)
            P = dd.aggregate(p, st.boxes)
            assert np.abs(px - st.px).sum() <= 1e-5 * np.abs(st.px).sum()
            assert np.abs(py - P).sum() <= 1e-5 * np.abs(P).sum()
    finally:
        B.dd_uot_destroy(h)
