"""The global Sinkhorn without allocations, through the C ABI.

On caller-owned device buffers it must give what the allocating entry point
gives on the same inputs (the same kernels in the same order: the same bits),
on two calls in a row, the second on a smaller grid (the library's scratch
keeps the first call's contents), and refuse what its scratch cannot hold.
"""
import numpy as np
import pytest
import torch

from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.inputs import workload_marginals

pytestmark = pytest.mark.gpu


def cfg_for(n):
    return B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=2.0 / n ** 2, lam=1.0, cell=4,
                                   precision=64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def test_noalloc_matches_the_allocating_entry_point_twice():
    stream = torch.cuda.current_stream().cuda_stream
    for n, iters, tol in ((128, 40, 0.0), (64, 300, 1e-9)):
        print(f"[noalloc] {n}x{n}, at most {iters} iterations, tol {tol:g}", flush=True)
        mu, nu = workload_marginals("grid256", n)
        cfg = cfg_for(n)
        beta0 = 1e-3 * np.cos(np.arange(n * n) / 7.0).reshape(n, n)
        ref = B.dd_uot_global_sinkhorn(cfg, mu, nu, beta0=beta0, max_iter=iters, tol=tol,
                                       stream=stream)
        m, v, b = dev(mu), dev(nu), dev(beta0)
        a = torch.full((n * n,), float("nan"), dtype=torch.float64, device="cuda")
        out = B.dd_uot_global_sinkhorn_noalloc(cfg, m, v, a, b, max_iter=iters, tol=tol,
                                               stream=stream)
        torch.cuda.synchronize()
        assert out["iters"] == ref["iters"]
        assert out["pd"] == ref["pd"]
        np.testing.assert_array_equal(a.cpu().numpy().reshape(n, n), ref["alpha"])
        np.testing.assert_array_equal(b.cpu().numpy().reshape(n, n), ref["beta"])
        # the inputs are left as they were
        np.testing.assert_array_equal(m.cpu().numpy().reshape(n, n), mu)
        np.testing.assert_array_equal(v.cpu().numpy().reshape(n, n), nu)


def test_noalloc_refuses_what_it_cannot_take():
    n = 512   # above the scratch's 256 x 256 points
    cfg = cfg_for(n)
    z = torch.ones(n * n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.DDUOTError, match="scratch"):
        B.dd_uot_global_sinkhorn_noalloc(cfg, z, z, z.clone(), z.clone(), max_iter=2)
    n = 32
    cfg = cfg_for(n)
    mu, nu = workload_marginals("grid32")
    bad = mu.copy()
    bad[3, 4] = 0.0
    with pytest.raises(B.DDUOTError, match="finite"):
        B.dd_uot_global_sinkhorn_noalloc(cfg, dev(bad), dev(nu), dev(np.zeros(n * n)),
                                         dev(np.zeros(n * n)), max_iter=2)
    host = torch.ones(n * n, dtype=torch.float64)
    with pytest.raises(B.DDUOTError, match="device memory"):
        B.dd_uot_global_sinkhorn_noalloc(cfg, host, host, host.clone(), host.clone(), max_iter=2)
