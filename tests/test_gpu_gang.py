"""Gangs: a wide cell (box wider than the in-LDS layout) solved by several
workgroups together, through the C ABI.

The gang path does the arithmetic of the one-workgroup path; only the order
of some sums differs (the members' partial sums of the X pass 2 and of the
Y sums are added in member order).  FP64 follows the oracle within 1e-10
relative whatever the gang size, FP32 within the FP32 parity bound (1e-5
relative, L1); at 256^2, where most cells are wide, gangs of every size
follow the one-workgroup path within the same bounds.
"""
import numpy as np
import pytest

from oracle import dd
from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.inputs import workload_marginals

pytestmark = pytest.mark.gpu


def l1_rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).sum() / np.abs(np.asarray(b)).sum())


def max_rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("G,wpc", [(1, 1), (8, 2), (16, 1)])
def test_gangs_follow_the_oracle(precision, G, wpc):
    mu, nu = workload_marginals("grid32")
    n = 32
    cfg = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=4.0 / n ** 2, lam=1.0, cell=4,
                                  precision=precision, init=B.INIT_BLOCK, sinkhorn_err=1e-8,
                                  sinkhorn_max_iter=150, lenience=0.0, box_cap=12, box_margin=2,
                                  getweights=B.GW_LINE,
                                  fixed_inner_iters=20 if precision == 32 else 0)
    p = dd.make_problem(mu, nu, cfg.eps, cfg.lambda_, cfg.h, cfg.cell)
    st = dd.init_block(p)
    opt = dd.Options(err=cfg.sinkhorn_err, max_iter=cfg.sinkhorn_max_iter,
                     fixed_iters=cfg.fixed_inner_iters, trunc=cfg.trunc, lenience=0.0,
                     margin=cfg.box_margin, getweights="line", translate=True)
    h = B.dd_uot_init(cfg, mu, nu)
    try:
        g, nwg = B.dd_uot_set_gang(h, G, wpc)
        print(f"[gang] FP{precision} G={g} workgroups={nwg}", flush=True)
        assert g == G and nwg > 0 and nwg % (8 * G) == 0
        rtol = 1e-10 if precision == 64 else 1e-5
        for k in range(4):
            ost = dd.half_iteration(p, st, "A" if k % 2 == 0 else "B", opt)
            B.dd_uot_iterate(h, 1)
            rec = B.dd_uot_history(h, 0)[-1]
            assert rec[3] == ost["n_updated"]
            assert rec[1] == pytest.approx(ost["e_cur"], rel=rtol), f"tracked score at {k}"
            assert rec[2] == pytest.approx(ost["e_greedy"], rel=rtol), f"greedy score at {k}"
            px, py = B.dd_uot_marginals(h, 0, n, n)
            P = dd.aggregate(p, st.boxes)
            if precision == 64:
                assert int(rec[4]) == ost["point_iters"], f"inner iterations at {k}"
                assert max_rel(px, st.px) <= rtol, f"P_X at {k}"
                assert max_rel(py, P) <= rtol, f"P_Y at {k}"
            else:
                assert l1_rel(px, st.px) <= rtol, f"P_X at {k}"
                assert l1_rel(py, P) <= rtol, f"P_Y at {k}"
        boxes, iters, _ = B.dd_uot_cell_stats(h, 1)
        wide = int((np.maximum(boxes[:, 2], boxes[:, 3]) > 12).sum())
        print(f"[gang] {wide} wide cells in the last B step", flush=True)
        assert wide > 0 and np.all(iters > 0)
        assert B.dd_uot_score(h, 0)["overflow"] == 0
    finally:
        B.dd_uot_destroy(h)


@pytest.mark.parametrize("precision", [64, 32])
def test_gang_sizes_agree_at_256(precision):
    # eps = h^2 with a small layout: most cells are wide and their boxes span
    # tens of rows, so every member of a 16-gang holds rows
    mu, nu = workload_marginals("grid256")
    n = 256
    cfg = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=1.0 / n ** 2, lam=1.0, cell=4,
                                  precision=precision, init=B.INIT_BLOCK, sinkhorn_err=1e-6,
                                  sinkhorn_max_iter=300, lenience=0.0, box_cap=16, box_margin=2,
                                  getweights=B.GW_LINE,
                                  fixed_inner_iters=30 if precision == 32 else 0)
    runs = {}
    for G, wpc in [(0, 2), (4, 2), (16, 1)]:
        h = B.dd_uot_init(cfg, mu, nu)
        try:
            g, nwg = B.dd_uot_set_gang(h, G, wpc)
            print(f"[gang] 256^2 FP{precision} G={g} workgroups={nwg}", flush=True)
            B.dd_uot_iterate(h, 6)
            boxes, iters, _ = B.dd_uot_cell_stats(h, 1)
            runs[G] = dict(hist=B.dd_uot_history(h, 0), marg=B.dd_uot_marginals(h, 0, n, n),
                           wide=int((np.maximum(boxes[:, 2], boxes[:, 3]) > 16).sum()),
                           score=B.dd_uot_score(h, 0))
        finally:
            B.dd_uot_destroy(h)
    ref = runs[0]
    print(f"[gang] wide cells in the last B step: {ref['wide']}", flush=True)
    assert ref["wide"] > 100
    for G in (4, 16):
        r = runs[G]
        assert r["wide"] == ref["wide"]
        if precision == 64:
            np.testing.assert_array_equal(r["hist"][:, 3], ref["hist"][:, 3])
            np.testing.assert_array_equal(r["hist"][:, 4], ref["hist"][:, 4])
            np.testing.assert_allclose(r["hist"][:, :3], ref["hist"][:, :3], rtol=1e-10)
            for a, b in zip(r["marg"], ref["marg"]):
                assert max_rel(a, b) <= 1e-10
        else:
            np.testing.assert_allclose(r["hist"][:, 1:3], ref["hist"][:, 1:3], rtol=1e-5)
            for a, b in zip(r["marg"], ref["marg"]):
                assert l1_rel(a, b) <= 1e-5
        assert r["score"]["rel_pd_gap"] == pytest.approx(ref["score"]["rel_pd_gap"], rel=1e-3, abs=1e-9)


def test_gang_setter_shapes_and_limits():
    mu, nu = workload_marginals("grid32")
    n = 32
    cfg = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=4.0 / n ** 2, lam=1.0, cell=4,
                                  precision=32, box_cap=12)
    h = B.dd_uot_init(cfg, mu, nu)
    try:
        for G, wpc in [(1, 1), (2, 2), (4, 1), (8, 2), (16, 2), (32, 1)]:
            g, nwg = B.dd_uot_set_gang(h, G, wpc)
            assert g == G and nwg % (8 * G) == 0 and nwg >= 8 * G
        assert B.dd_uot_set_gang(h, 0, 1) == (0, 0)
        with pytest.raises(B.DDUOTError):
            B.dd_uot_set_gang(h, -1, 1)
        with pytest.raises(B.DDUOTError):
            B.dd_uot_set_gang(h, 8, 0)
    finally:
        B.dd_uot_destroy(h)
    # the balancing step keeps the one-workgroup path
    cb = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=4.0 / n ** 2, lam=1.0, cell=4,
                                 precision=32, box_cap=12, balance=1)
    h = B.dd_uot_init(cb, mu, nu)
    try:
        assert B.dd_uot_set_gang(h, 8, 2) == (0, 0)
    finally:
        B.dd_uot_destroy(h)


def test_gang_autotuner_keeps_the_trajectory():
    # the autotuner times the wide cells' launch shapes on the current state,
    # leaves the state as it was, and the tuned handle follows the untuned one
    mu, nu = workload_marginals("grid256")
    n = 256
    cfg = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=1.0 / n ** 2, lam=1.0, cell=4,
                                  precision=64, init=B.INIT_BLOCK, sinkhorn_err=1e-6,
                                  sinkhorn_max_iter=300, lenience=0.0, box_cap=16, box_margin=2,
                                  getweights=B.GW_LINE)
    ha = B.dd_uot_init(cfg, mu, nu)
    hb = B.dd_uot_init(cfg, mu, nu)
    try:
        B.dd_uot_iterate(ha, 3)
        B.dd_uot_iterate(hb, 3)
        g, w, ms = B.dd_uot_autotune_gang(hb)
        print(f"[gang] autotune: G={g} per CU {w}; ms {np.round(ms, 2).tolist()}", flush=True)
        assert ms[0] > 0 and (g, w) in [(0, 0), (2, 2), (4, 1), (4, 2), (8, 1), (8, 2), (16, 2)]
        assert ms[[0, 1, 2, 3, 4, 5, 6].index(
            [(0, 0), (2, 2), (4, 1), (4, 2), (8, 1), (8, 2), (16, 2)].index((g, w)))] == ms[ms > 0].min()
        B.dd_uot_iterate(ha, 3)
        B.dd_uot_iterate(hb, 3)
        np.testing.assert_array_equal(B.dd_uot_history(hb, 0)[:, 3], B.dd_uot_history(ha, 0)[:, 3])
        np.testing.assert_allclose(B.dd_uot_history(hb, 0)[:, :3], B.dd_uot_history(ha, 0)[:, :3],
                                   rtol=1e-10)
        for a, b in zip(B.dd_uot_marginals(hb, 0, n, n), B.dd_uot_marginals(ha, 0, n, n)):
            assert max_rel(a, b) <= 1e-10
    finally:
        B.dd_uot_destroy(ha)
        B.dd_uot_destroy(hb)
