"""State export and import through the C ABI (checkpoint / resume).

A state read from one handle and loaded into a fresh handle of the same
problem continues on exactly the same trajectory; a state moved from an
FP64 handle into an FP32 one gives one FP32 step from the same state, whose
difference to the FP64 step is the FP32 error of that step.
"""
import numpy as np
import pytest

from oracle import dd
from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.inputs import workload_marginals

pytestmark = pytest.mark.gpu


def cfg(n, precision, **kw):
    return B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=4.0 / n ** 2, lam=1.0, cell=4,
                                   precision=precision, init=B.INIT_BLOCK, sinkhorn_err=1e-8,
                                   sinkhorn_max_iter=200, lenience=0.0, box_cap=32,
                                   getweights=B.GW_LINE, **kw)


def test_resume_from_exported_state_follows_the_same_trajectory():
    mu, nu = workload_marginals("grid32")
    n = 32
    nb = (n // 4) ** 2
    a = B.dd_uot_init(cfg(n, 64), mu, nu)
    b = B.dd_uot_init(cfg(n, 64), mu, nu)
    try:
        print("[state] export after 3 half-iterations", flush=True)
        B.dd_uot_iterate(a, 3)
        st = B.dd_uot_get_state(a, n, n, nb)
        assert st["k"] == 3 and np.all(st["warm"] == 1)
        assert st["values"].size == sum(int(x[2] * x[3]) for x in st["boxes"])
        B.dd_uot_set_state(b, st)
        back = B.dd_uot_get_state(b, n, n, nb)
        for key in ("boxes", "values", "px", "hbar", "abar", "warm"):
            np.testing.assert_array_equal(back[key], st[key], err_msg=key)
        B.dd_uot_iterate(a, 3)
        B.dd_uot_iterate(b, 3)
        ra, rb = B.dd_uot_history(a, 0)[-3:], B.dd_uot_history(b, 0)[-3:]
        np.testing.assert_allclose(rb[:, :9], ra[:, :9], rtol=1e-12, atol=0)
        for x, y in zip(B.dd_uot_marginals(a, 0, n, n), B.dd_uot_marginals(b, 0, n, n)):
            np.testing.assert_allclose(y, x, rtol=0, atol=1e-13 * x.max())
        # the oracle resumes the same state on the same path (first step)
        p = dd.make_problem(mu, nu, 4.0 / n ** 2, 1.0, 1.0 / n, 4)
        boxes = []
        off = 0
        for o1, o2, l1, l2 in st["boxes"]:
            boxes.append((int(o1), int(o2), st["values"][off:off + l1 * l2].reshape(l1, l2).copy()))
            off += l1 * l2
        ost = dd.State(boxes, st["px"].copy(), st["hbar"].copy(), st["abar"].copy(),
                       warm=st["warm"].astype(bool), k=3)
        c = cfg(n, 64)
        opt = dd.Options(err=c.sinkhorn_err, max_iter=c.sinkhorn_max_iter, trunc=c.trunc,
                         lenience=0.0, margin=c.box_margin, getweights="line", translate=True)
        out = dd.half_iteration(p, ost, "B", opt)
        assert rb[0, 0] == pytest.approx(out["theta"], rel=1e-9)
        assert rb[0, 1] == pytest.approx(out["e_cur"], rel=1e-10)
        assert rb[0, 2] == pytest.approx(out["e_greedy"], rel=1e-10)
    finally:
        B.dd_uot_destroy(a)
        B.dd_uot_destroy(b)


def test_fp64_state_into_fp32_handle_gives_the_fp32_error_of_one_step():
    mu, nu = workload_marginals("grid32")
    n = 32
    nb = (n // 4) ** 2
    h64 = B.dd_uot_init(cfg(n, 64, fixed_inner_iters=20), mu, nu)
    h32 = B.dd_uot_init(cfg(n, 32, fixed_inner_iters=20), mu, nu)
    try:
        print("[state] FP64 -> FP32", flush=True)
        B.dd_uot_iterate(h64, 4)
        st = B.dd_uot_get_state(h64, n, n, nb)
        B.dd_uot_set_state(h32, st)
        B.dd_uot_iterate(h64, 1)
        B.dd_uot_iterate(h32, 1)
        r64, r32 = B.dd_uot_history(h64, 0)[-1], B.dd_uot_history(h32, 0)[-1]
        assert r32[3] == r64[3]
        assert r32[2] == pytest.approx(r64[2], rel=1e-5)
        for x64, x32 in zip(B.dd_uot_marginals(h64, 0, n, n), B.dd_uot_marginals(h32, 0, n, n)):
            err = np.abs(x32 - x64).sum() / np.abs(x64).sum()
            print(f"[state] FP32 step error (rel L1) {err:.2e}", flush=True)
            assert err <= 1e-5
    finally:
        B.dd_uot_destroy(h64)
        B.dd_uot_destroy(h32)
