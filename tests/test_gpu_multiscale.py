"""Multiscale refinement on the GPU against the oracle's refinement (reading
R10), and the coarse-to-fine driver end to end."""
import numpy as np
import pytest

from oracle import dd
from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.inputs import gaussian_mixture

pytestmark = pytest.mark.gpu


def cfg(n, s, eps, precision=64, cap=32):
    return B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=eps, lam=1.0, cell=s,
                                   precision=precision, init=B.INIT_BLOCK, lenience=0.0,
                                   box_cap=cap, box_margin=2, trunc=1e-15, fixed_inner_iters=20)


@pytest.mark.parametrize("sc,sf", [(2, 2), (2, 4)])
def test_refine_matches_oracle(sc, sf):
    nf = 32
    muf = gaussian_mixture(nf, nf, 3, 1e-3, 1.0, 801)
    nuf = gaussian_mixture(nf, nf, 3, 1e-3, 1.3, 802)
    muc, nuc = dd.coarsen(muf), dd.coarsen(nuf)
    nc = nf // 2
    ec, ef = 2.0 / nc ** 2, 2.0 / nf ** 2
    cc, cf = cfg(nc, sc, ec), cfg(nf, sf, ef)
    print(f"[multiscale] refine {nc}->{nf}, cells {sc}->{sf}", flush=True)
    pc = dd.make_problem(muc, nuc, ec, 1.0, 1.0 / nc, sc)
    pf = dd.make_problem(muf, nuf, ef, 1.0, 1.0 / nf, sf)
    stc = dd.init_block(pc)
    opt = dd.Options(fixed_iters=20, lenience=0.0, cap=32, margin=2, trunc=1e-15, translate=True)
    dd.run(pc, stc, 3, opt)
    hc = B.dd_uot_init(cc, muc, nuc)
    hf = None
    try:
        B.dd_uot_iterate(hc, 3)
        hf = B.dd_uot_refine(hc, cf, muf, nuf)
        stf = dd.refine(pc, stc, pf, 1e-15, 32)
        px, _ = B.dd_uot_marginals(hf, 0, nf, nf)
        np.testing.assert_allclose(px, stf.px, rtol=0, atol=1e-10 * stf.px.max())
        for b in range(pf.nb1 * pf.nb2):
            o1, o2, arr = B.dd_uot_basic_marginal(hf, 0, b)
            r1, r2, ref = stf.boxes[b]
            if ref.size == 0:
                assert arr.size == 0
                continue
            assert (o1, o2, arr.shape) == (r1, r2, ref.shape), f"box of basic cell {b}"
            np.testing.assert_allclose(arr, ref, rtol=0, atol=1e-10 * ref.max())
        # the next (forced greedy) half-iteration follows the oracle
        B.dd_uot_iterate(hf, 1)
        out = dd.half_iteration(pf, stf, "A", opt)
        assert out["theta"] == 1.0
        px, py = B.dd_uot_marginals(hf, 0, nf, nf)
        np.testing.assert_allclose(px, stf.px, rtol=0, atol=1e-10 * stf.px.max())
        P = dd.aggregate(pf, stf.boxes)
        np.testing.assert_allclose(py, P, rtol=0, atol=1e-10 * P.max())
    finally:
        B.dd_uot_destroy(hc)
        B.dd_uot_destroy(hf)


def test_multiscale_driver_reduces_the_gap():
    n = 128
    mu = gaussian_mixture(n, n, 3, 1e-3, 1.0, 811)
    nu = gaussian_mixture(n, n, 3, 1e-3, 1.3, 812)
    c = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=1.0 / n ** 2, lam=1.0, cell=4,
                                precision=64, box_cap=48, sinkhorn_max_iter=500)
    ms = B.dd_uot_default_multiscale(levels=3, final_max_halves=24, check_every=4,
                                     target_rel_gap=1e-9)
    print("[multiscale] driver 32 -> 128", flush=True)
    h, tr = B.dd_uot_solve_multiscale(c, ms, mu, nu)
    try:
        assert tr.shape[0] >= 2
        print(tr, flush=True)
        assert np.all(np.diff(tr[:, 1]) > 0)
        assert tr[-1, 2] < tr[0, 2]
        s = B.dd_uot_score(h, 0)
        assert s["rel_pd_gap"] == pytest.approx(tr[-1, 2], rel=1e-12)
        assert abs(s["mass_x"] - s["mass_y"]) <= 1e-9 * s["mass_x"]
    finally:
        B.dd_uot_destroy(h)
