"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 cell arithmetic must follow the oracle's trajectory half-iteration by
half-iteration within 1e-10 relative; FP32 cell log-sum-exp (with FP64 bases
and reductions) must match scores and marginals within 1e-5 relative.
"""
import numpy as np
import pytest

from oracle import dd
from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.inputs import gaussian_mixture, workload_marginals

pytestmark = pytest.mark.gpu

GW = {0: "greedy", 1: "safe", 2: "swift", 3: "staggered", 4: "line", 5: "opt"}


def config(n, s, eps, lam, h, **kw):
    return B.dd_uot_default_config(n1=n, n2=n, h=h, eps=eps, lam=lam, cell=s, **kw)


def oracle_options(cfg):
    return dd.Options(err=cfg.sinkhorn_err, max_iter=cfg.sinkhorn_max_iter,
                      fixed_iters=cfg.fixed_inner_iters, trunc=cfg.trunc, lenience=cfg.lenience,
                      margin=cfg.box_margin, getweights=GW[cfg.getweights],
                      translate=bool(cfg.translate), balance=bool(cfg.balance),
                      support=bool(cfg.support_only))


def oracle_start(p, cfg):
    return dd.init_product(p) if cfg.init == B.INIT_PRODUCT else dd.init_block(p)


def rel_close(a, b, rtol, what):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max() / scale
    assert err <= rtol, f"{what}: max |gpu - oracle| / max|oracle| = {err:.3e} > {rtol:.1e}"


def l1_rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).sum() / np.abs(np.asarray(b)).sum()


def run_pair(mu, nu, cfg, n_half, check_every=True, rtol=1e-10, theta_rtol=1e-15):
    n, n2 = cfg.n1, cfg.n2
    p = dd.make_problem(mu, nu, cfg.eps, cfg.lambda_, cfg.h, cfg.cell)
    st = oracle_start(p, cfg)
    opt = oracle_options(cfg)
    h = B.dd_uot_init(cfg, mu, nu)
    try:
        print(f"[parity] n={n}x{n2} s={cfg.cell} h={cfg.h:g} prec={cfg.precision} init={cfg.init} "
              f"fixed={cfg.fixed_inner_iters} gw={cfg.getweights}", flush=True)
        for k in range(n_half):
            ost = dd.half_iteration(p, st, "A" if k % 2 == 0 else "B", opt)
            B.dd_uot_iterate(h, 1)
            if not check_every and k != n_half - 1:
                continue
            rec = B.dd_uot_history(h, 0)[-1]
            assert rec[0] == pytest.approx(ost["theta"], rel=theta_rtol), f"theta at step {k}"
            assert rec[3] == ost["n_updated"]
            rel_close(rec[1], ost["e_cur"], rtol, f"tracked score at step {k}")
            rel_close(rec[2], ost["e_greedy"], rtol, f"greedy score at step {k}")
            if cfg.precision == 64:
                assert int(rec[4]) == ost["point_iters"], f"inner iterations at step {k}"
            px, py = B.dd_uot_marginals(h, 0, n, n2)
            P = dd.aggregate(p, st.boxes)
            if cfg.precision == 64:
                rel_close(px, st.px, rtol, f"P_X at step {k}")
                rel_close(py, P, rtol, f"P_Y at step {k}")
                a, _ = B.dd_uot_potentials(h, 0, n, n2, beta=False)
                rel_close(a, st.abar, rtol, f"alpha_bar at step {k}")
            else:
                assert l1_rel(px, st.px) < rtol, f"P_X at step {k}: {l1_rel(px, st.px):.2e}"
                assert l1_rel(py, P) < rtol, f"P_Y at step {k}: {l1_rel(py, P):.2e}"
        return h, p, st
    except BaseException:
        B.dd_uot_destroy(h)
        raise


def compare_boxes(h, p, st, rtol):
    for b in range(p.nb1 * p.nb2):
        o1, o2, arr = B.dd_uot_basic_marginal(h, 0, b)
        e1, e2, ref = st.boxes[b]
        assert (o1, o2, arr.shape) == (e1, e2, ref.shape), f"box of basic cell {b}"
        if ref.size:
            rel_close(arr, ref, rtol, f"nu_{b}")


@pytest.fixture(scope="module")
def grid32():
    mu, nu = workload_marginals("grid32")
    return mu, nu


@pytest.mark.parametrize("translate", [0, 1])
def test_fp64_product_start_fixed_inner(grid32, translate):
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=64, init=B.INIT_PRODUCT,
                 fixed_inner_iters=20, lenience=0.0, box_cap=32, translate=translate)
    h, p, st = run_pair(mu, nu, cfg, 6)
    try:
        compare_boxes(h, p, st, 1e-10)
    finally:
        B.dd_uot_destroy(h)


def test_fp64_block_start_boxes_and_truncation(grid32):
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=64, init=B.INIT_BLOCK,
                 sinkhorn_err=1e-9, sinkhorn_max_iter=150, lenience=0.0, box_cap=32, box_margin=2)
    h, p, st = run_pair(mu, nu, cfg, 8)
    try:
        compare_boxes(h, p, st, 1e-10)
    finally:
        B.dd_uot_destroy(h)


@pytest.mark.parametrize("gw", [B.GW_SAFE, B.GW_GREEDY, B.GW_LINE])
def test_fp64_other_getweights(grid32, gw):
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=64, init=B.INIT_PRODUCT,
                 fixed_inner_iters=10, lenience=0.0, box_cap=32, getweights=gw)
    # greedy collapses the plan on this problem (Sec. 4.2 divergence), which
    # amplifies rounding differences; compare the steps before the collapse.
    # line: both sides find the root of the same derivative f', whose sums are
    # taken in different orders; the root moves by their rounding over f''
    # (weights equal to ~2e-10 after six warm-started steps)
    steps = {B.GW_SAFE: 4, B.GW_GREEDY: 3, B.GW_LINE: 6}[gw]
    h, _, _ = run_pair(mu, nu, cfg, steps, theta_rtol=1e-15 if gw != B.GW_LINE else 1e-9)
    if gw == B.GW_LINE:
        thetas = B.dd_uot_history(h, 0)[:, 0]
        print(f"[parity] line weights {thetas}", flush=True)
        assert np.any((thetas > 1.0 / 16) & (thetas < 1.0))   # an interior minimiser
    B.dd_uot_destroy(h)


@pytest.mark.parametrize("precision,lam,init", [(64, 10.0, B.INIT_BLOCK), (64, 1.0, B.INIT_PRODUCT),
                                                 (32, 10.0, B.INIT_BLOCK)])
def test_balancing_follows_the_oracle(grid32, precision, lam, init):
    # balancing step (Sec. 4.1): mass moved along X between the basic cells
    # of every composite cell, in proportion to e^{-alpha'/lambda} mu
    mu, nu = grid32
    n = 32
    kw = dict(precision=precision, init=init, fixed_inner_iters=20, lenience=0.0, box_cap=32,
              box_margin=2)
    cfg = config(n, 4, 4.0 / n ** 2, lam, 1.0 / n, balance=1, **kw)
    rtol = 1e-10 if precision == 64 else 1e-5
    h, p, st = run_pair(mu, nu, cfg, 6, rtol=rtol)
    h0 = B.dd_uot_init(config(n, 4, 4.0 / n ** 2, lam, 1.0 / n, **kw), mu, nu)
    try:
        if precision == 64:
            compare_boxes(h, p, st, 1e-10)
        B.dd_uot_iterate(h0, 6)
        px, _ = B.dd_uot_marginals(h, 0, n, n)
        px0, _ = B.dd_uot_marginals(h0, 0, n, n)
        moved = l1_rel(px0, px)
        print(f"[parity] balancing changed P_X by {moved:.2e} (L1, relative)", flush=True)
        assert moved > 1e-4   # the step is not vacuous on this problem
    finally:
        B.dd_uot_destroy(h)
        B.dd_uot_destroy(h0)


@pytest.mark.parametrize("n1,n2,s,h", [(24, 40, 2, 1 / 32), (16, 16, 1, 1 / 16), (16, 16, 2, 0.0)])
def test_fp64_grid_shapes_and_vanishing_cost(n1, n2, s, h):
    # a rectangular grid (its own B offsets on each axis), one-point basic
    # cells (2 x 2 tiles), and h = 0 (the cost vanishes, no windows)
    mu = gaussian_mixture(n1, n2, 3, 1e-3, 1.0, 1001)
    nu = gaussian_mixture(n1, n2, 3, 1e-3, 1.3, 1002)
    cfg = B.dd_uot_default_config(n1=n1, n2=n2, h=h, eps=4.0 / 32 ** 2, lam=1.0, cell=s,
                                  precision=64, init=B.INIT_BLOCK, fixed_inner_iters=20,
                                  lenience=0.0, box_cap=32 if n1 != 16 else 16, box_margin=2)
    h_, p, st = run_pair(mu, nu, cfg, 4)
    try:
        compare_boxes(h_, p, st, 1e-10)
    finally:
        B.dd_uot_destroy(h_)


@pytest.mark.parametrize("precision", [64, 32])
def test_largest_box_cap_fits_and_keeps_the_trajectory(precision):
    # the largest box side whose cell layout fits the LDS of one workgroup:
    # one more is rejected before any launch; at the largest, a trajectory
    # whose boxes stay small is that of a small cap
    n = 64
    mu = gaussian_mixture(n, n, 3, 1e-3, 1.0, 1011)
    nu = gaussian_mixture(n, n, 3, 1e-3, 1.3, 1012)
    kw = dict(precision=precision, init=B.INIT_BLOCK, fixed_inner_iters=10, lenience=0.0,
              box_margin=2)
    big = None
    for cap in range(128, 31, -1):
        try:
            big = B.dd_uot_init(config(n, 4, 2.0 / n ** 2, 1.0, 1.0 / n, box_cap=cap, **kw), mu, nu)
            break
        except B.DDUOTError as e:
            assert e.code == B.EINVAL and "LDS" in str(e)
    assert big is not None and cap < 128
    print(f"[parity] FP{precision}: largest box cap {cap}, launch caps {B.dd_uot_launch_caps(big)}",
          flush=True)
    small = B.dd_uot_init(config(n, 4, 2.0 / n ** 2, 1.0, 1.0 / n, box_cap=64, **kw), mu, nu)
    try:
        B.dd_uot_iterate(big, 3)
        B.dd_uot_iterate(small, 3)
        assert B.dd_uot_score(small, 0)["overflow"] == 0 and B.dd_uot_score(big, 0)["overflow"] == 0
        for a, b in zip(B.dd_uot_marginals(big, 0, n, n), B.dd_uot_marginals(small, 0, n, n)):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * b.max())
        np.testing.assert_allclose(B.dd_uot_history(big, 0)[:, :3], B.dd_uot_history(small, 0)[:, :3],
                                   rtol=1e-12, atol=0)
    finally:
        B.dd_uot_destroy(big)
        B.dd_uot_destroy(small)


def test_fp32_matches_fp64_oracle(grid32):
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=32, init=B.INIT_PRODUCT,
                 fixed_inner_iters=20, lenience=0.0, box_cap=32)
    h, _, _ = run_pair(mu, nu, cfg, 6, rtol=1e-5)
    B.dd_uot_destroy(h)


def test_certificate_and_backward_match_oracle(grid32):
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=64, init=B.INIT_PRODUCT,
                 sinkhorn_err=1e-10, lenience=0.0, box_cap=32)
    h, p, st = run_pair(mu, nu, cfg, 4, check_every=False)
    try:
        s = B.dd_uot_score(h, 0)
        cert = dd.certificate(p, st.abar)
        for key, ref in (("pd_gap", cert["pd"]), ("dual", cert["dual"]), ("primal", cert["primal"])):
            print(f"[parity] certificate {key}: rel {abs(s[key] - ref) / abs(ref):.2e}", flush=True)
            assert s[key] == pytest.approx(ref, rel=1e-10), key
        assert s["tracked"] == pytest.approx(dd.tracked_score(p, st), rel=1e-10)
        _, bh = B.dd_uot_potentials(h, 0, n, n)
        rel_close(bh, cert["beta_hat"], 1e-10, "beta_hat")
        dmu, dnu = B.dd_uot_backward(h, 0, n, n)
        eps, lam = p.eps, p.lam
        ref_mu = eps * p.nu.sum() - eps * cert["px"] / p.mu - lam * (np.exp(-st.abar / lam) - 1)
        ref_nu = eps * p.mu.sum() - eps * cert["py"] / p.nu - lam * (np.exp(-cert["beta_hat"] / lam) - 1)
        rel_close(dmu, ref_mu, 1e-10, "dW/dmu")
        rel_close(dnu, ref_nu, 1e-10, "dW/dnu")
    finally:
        B.dd_uot_destroy(h)


def test_polished_bounds_sparsity_and_counts_match_oracle(grid32):
    # the polished score bounds (global Sinkhorn pairs from alpha_bar), the
    # sparsity count of Sec. 4.2 and the safe / unconverged counts of the
    # recorded steps, against the oracle's state and certificate
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=64, init=B.INIT_BLOCK,
                 sinkhorn_err=1e-8, sinkhorn_max_iter=40, lenience=0.0, box_cap=32,
                 getweights=B.GW_SWIFT)
    h, p, st = run_pair(mu, nu, cfg, 5, check_every=False)
    try:
        for m in (0, 7):
            B.dd_uot_set_polish(h, m)
            s = B.dd_uot_score(h, 0)
            cert = dd.certificate(p, st.abar, polish=m)
            tracked = dd.tracked_score(p, st)
            print(f"[parity] polish {m}: rel gap {s['rel_gap_polished']:.3e}", flush=True)
            assert s["polish_iters"] == m
            assert s["dual_polished"] == pytest.approx(cert["dual_polished"], rel=1e-10)
            assert s["primal_polished"] == pytest.approx(min(tracked, cert["primal_polished"]),
                                                         rel=1e-10)
            ref = (min(tracked, cert["primal_polished"]) - cert["dual_polished"]) / \
                abs(cert["dual_polished"])
            assert s["rel_gap_polished"] == pytest.approx(ref, rel=1e-6, abs=1e-12)
        assert s["dual_polished"] >= s["dual"] and s["primal_polished"] <= s["tracked"]
        assert s["nnz"] == sum(int(np.count_nonzero(arr > 1e-14)) for _, _, arr in st.boxes)
        assert s["n_safe"] == sum(1 for x in st.history if x["theta"] < 1.0)
        assert s["n_unconverged"] == sum(x["n_unconverged"] for x in st.history)
        assert s["n_unconverged"] > 0
    finally:
        B.dd_uot_destroy(h)


def gpu_state_of(st, k):
    """The oracle's state in the layout of dd_uot_set_state."""
    boxes = np.array([[o1, o2, arr.shape[0], arr.shape[1]] for o1, o2, arr in st.boxes],
                     dtype=np.int32).reshape(-1, 4)
    vals = np.concatenate([arr.ravel() for _, _, arr in st.boxes] + [np.zeros(0)])
    warm = np.zeros(len(st.boxes), dtype=np.int32) if st.warm is None else st.warm.astype(np.int32)
    return dict(boxes=boxes, values=vals, px=st.px, hbar=st.hbar, abar=st.abar, warm=warm, k=k)


def test_fp64_opt_weights_match_the_oracle_minimiser(grid32):
    # GetWeights opt (eq. opt-weights-problem): the device's rounds of
    # projected diagonal Newton with exact searches against the oracle's
    # bounded minimiser, one step at a time from the oracle's state
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=64, init=B.INIT_PRODUCT,
                 fixed_inner_iters=15, lenience=0.0, box_cap=32, getweights=B.GW_OPT, trunc=0.0)
    p = dd.make_problem(mu, nu, cfg.eps, cfg.lambda_, cfg.h, cfg.cell)
    st = dd.init_product(p)
    opt = oracle_options(cfg)
    h = B.dd_uot_init(cfg, mu, nu)
    try:
        for k in range(4):
            if k > 0:
                B.dd_uot_set_state(h, gpu_state_of(st, k))
            out = dd.half_iteration(p, st, "A" if k % 2 == 0 else "B", opt)
            B.dd_uot_iterate(h, 1)
            rec = B.dd_uot_history(h, 0)[-1]
            s = B.dd_uot_score(h, 0)
            ref = dd.tracked_score(p, st)
            print(f"[parity] opt step {k}: mean weight {rec[0]:.6f} vs {out['theta']:.6f}, "
                  f"weights in [{out['thetas'].min():.3g}, {out['thetas'].max():.3g}], tracked "
                  f"{s['tracked']:.12g} vs {ref:.12g}", flush=True)
            # the optimal value is unique; the weights of this ill-conditioned
            # minimiser move by ~1e-4 for score changes of ~1e-10
            assert s["tracked"] == pytest.approx(ref, rel=1e-9)
            assert rec[0] == pytest.approx(out["theta"], rel=1e-3)
            px, py = B.dd_uot_marginals(h, 0, n, n)
            rel_close(px, st.px, 1e-6, f"P_X at {k}")
            rel_close(py, dd.aggregate(p, st.boxes), 1e-6, f"P_Y at {k}")
    finally:
        B.dd_uot_destroy(h)


@pytest.mark.parametrize("precision", [64, 32])
def test_boxes_wider_than_the_lds_layout_follow_the_oracle(grid32, precision):
    # B cells gather basic boxes grown inside four different A boxes; with an
    # in-LDS layout of side 12 their union no longer fits, so those cells run
    # the variant whose box arrays live in the cell workspace: every cell is
    # solved, on the same trajectory as the oracle (which has no box limit)
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=precision, init=B.INIT_BLOCK,
                 sinkhorn_err=1e-8, sinkhorn_max_iter=150, lenience=0.0, box_cap=12, box_margin=2,
                 fixed_inner_iters=20 if precision == 32 else 0)
    h, p, st = run_pair(mu, nu, cfg, 4, rtol=1e-10 if precision == 64 else 1e-5)
    try:
        hist = B.dd_uot_history(h, 0)
        assert np.all(hist[:, 7] == 0)
        assert list(hist[:, 3].astype(int)) == [x["n_updated"] for x in st.history]
        wide = sum(1 for _, _, arr in st.boxes if arr.size and max(arr.shape) > 12)
        print(f"[parity] FP{precision}: {wide} basic boxes wider than the layout", flush=True)
        assert wide > 0
        assert B.dd_uot_score(h, 0)["overflow"] == 0
        if precision == 64:   # FP32 may round entries near the truncation level either way
            compare_boxes(h, p, st, 1e-10)
    finally:
        B.dd_uot_destroy(h)


@pytest.mark.parametrize("balance", [0, 1])
def test_fp64_staggered_batches(grid32, balance):
    # staggered GetWeights: four batch steps per half-iteration, each with its
    # own record, theta and scores (with balancing: the paper's production
    # setting)
    mu, nu = grid32
    n = 32
    cfg = config(n, 4, 4.0 / n ** 2, 1.0, 1.0 / n, precision=64, init=B.INIT_BLOCK,
                 fixed_inner_iters=20, lenience=0.0, box_cap=32, box_margin=2,
                 getweights=B.GW_STAGGERED, balance=balance)
    p = dd.make_problem(mu, nu, cfg.eps, cfg.lambda_, cfg.h, cfg.cell)
    st = dd.init_block(p)
    opt = oracle_options(cfg)
    h = B.dd_uot_init(cfg, mu, nu)
    try:
        for k in range(4):
            print(f"[parity] staggered half-iteration {k}", flush=True)
            outs = dd.half_iteration(p, st, "A" if k % 2 == 0 else "B", opt)
            B.dd_uot_iterate(h, 1)
            recs = B.dd_uot_history(h, 0)[-4:]
            assert len(B.dd_uot_history(h, 0)) == 4 * (k + 1)
            for rec, ost in zip(recs, outs):
                assert rec[0] == pytest.approx(ost["theta"], rel=1e-15)
                assert rec[3] == ost["n_updated"]
                rel_close(rec[1], ost["e_cur"], 1e-10, f"tracked score at {k}")
                rel_close(rec[2], ost["e_greedy"], 1e-10, f"greedy score at {k}")
            px, py = B.dd_uot_marginals(h, 0, n, n)
            rel_close(px, st.px, 1e-10, f"P_X at {k}")
            rel_close(py, dd.aggregate(p, st.boxes), 1e-10, f"P_Y at {k}")
        compare_boxes(h, p, st, 1e-10)
    finally:
        B.dd_uot_destroy(h)
