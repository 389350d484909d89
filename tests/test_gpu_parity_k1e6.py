"""FP32 steps where the bench's state lives: K = lambda/eps ~ 1e6, Y-boxes
grown past the in-LDS layout (so both the in-LDS kernel and the gang kernel
solve cells), the shifted sums' retry and exact recomputation paths taken.

Step parity: before each of 8 half-iterations from the block start, the FP32
handle is loaded with the FP64 oracle's state, and the step's tracked and
greedy scores, P_X and P_Y are compared with the oracle's step within the
FP32 bound (1e-5 relative).  A second FP32 handle runs the 8 steps on its
own; its marginals stay within the same bound of the oracle's trajectory.
(With the pass exponents formed in FP32, the cancellation between a large
potential and a large transport cost made the one-step error grow with the
box width, to 1e-5 at the sixth step here; they are formed in FP64.)
"""
import numpy as np
import pytest

from oracle import dd
from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.inputs import workload_marginals

pytestmark = pytest.mark.gpu


def as_device_state(st, n1, n2):
    """The oracle's state in the layout of dd_uot_set_state."""
    boxes, vals = [], []
    for o1, o2, arr in st.boxes:
        l1, l2 = arr.shape if arr.size else (0, 0)
        boxes.append((o1, o2, l1, l2))
        vals.append(np.ascontiguousarray(arr, dtype=np.float64).ravel())
    return dict(boxes=np.asarray(boxes, dtype=np.int32), values=np.concatenate(vals),
                px=st.px.reshape(n1, n2), hbar=st.hbar, abar=st.abar.reshape(n1, n2),
                warm=np.asarray(st.warm, dtype=np.int32), k=st.k)


def test_fp32_steps_at_k_1e6_with_boxes_past_the_layout_follow_the_oracle():
    mu, nu = workload_marginals("grid256")
    n, lam = 256, 16.0
    cap = 24
    cfg = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=1.0 / n ** 2, lam=lam, cell=8,
                                  precision=32, init=B.INIT_BLOCK, fixed_inner_iters=20,
                                  sinkhorn_err=1e-6, lenience=0.0, box_cap=cap, box_margin=2,
                                  getweights=B.GW_LINE)
    assert lam / cfg.eps > 1e6
    p = dd.make_problem(mu, nu, cfg.eps, lam, cfg.h, cfg.cell)
    st = dd.init_block(p)
    opt = dd.Options(err=cfg.sinkhorn_err, max_iter=cfg.sinkhorn_max_iter, fixed_iters=20,
                     trunc=cfg.trunc, lenience=0.0, margin=2, getweights="line", translate=True)
    h = B.dd_uot_init(cfg, mu, nu)      # stepped from the oracle's state every time
    hf = B.dd_uot_init(cfg, mu, nu)     # free-running FP32 trajectory
    try:
        widest, falls = 0, 0.0
        for k in range(8):
            part = k % 2
            if k > 0:
                B.dd_uot_set_state(h, as_device_state(st, n, n))
            out = dd.half_iteration(p, st, "A" if part == 0 else "B", opt)
            B.dd_uot_iterate(h, 1)
            B.dd_uot_iterate(hf, 1)
            rec = B.dd_uot_history(h, 0)[-1]
            falls += rec[11]
            boxes, _, _ = B.dd_uot_cell_stats(h, part)
            side = np.maximum(boxes[:, 2], boxes[:, 3])
            widest = max(widest, int(side.max()))
            P = dd.aggregate(p, st.boxes)
            px, py = B.dd_uot_marginals(h, 0, n, n)
            ex = np.abs(px - st.px).sum() / st.px.sum()
            ey = np.abs(py - P).sum() / P.sum()
            fx, fy = B.dd_uot_marginals(hf, 0, n, n)
            free = max(np.abs(fx - st.px).sum() / st.px.sum(), np.abs(fy - P).sum() / P.sum())
            print(f"[k1e6] step {k}: theta {rec[0]:.6g} / {out['theta']:.6g}, wide cells "
                  f"{int((side > cap).sum())} (widest {int(side.max())}), fallbacks {rec[11]:.0f}; "
                  f"step error P_X {ex:.2e} P_Y {ey:.2e}; free-running {free:.2e}", flush=True)
            assert rec[3] == out["n_updated"]
            assert rec[0] == pytest.approx(out["theta"], rel=1e-5), f"theta at {k}"
            assert rec[1] == pytest.approx(out["e_cur"], rel=1e-5), f"tracked score at {k}"
            assert rec[2] == pytest.approx(out["e_greedy"], rel=1e-5), f"greedy score at {k}"
            assert ex <= 1e-5 and ey <= 1e-5, f"marginals at {k}"
            assert free <= 1e-5, f"free-running marginals at {k}"
        assert falls > 0          # retries / exact recomputations ran
        assert widest > cap       # the gang kernel solved cells
    finally:
        B.dd_uot_destroy(h)
        B.dd_uot_destroy(hf)
