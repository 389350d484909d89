"""The C ABI with device memory: marginals given as device pointers, outputs
written into device buffers, the gradient seed applied on the device.

Inputs in device memory give the same solve as the same values in host
memory (bit for bit: the library reads them once into its own buffers);
outputs written into device buffers equal those copied to the host.
"""
import numpy as np
import pytest
import torch

from paper_2410_08859_amd import binding as B
from paper_2410_08859_amd.autograd import uot_value
from paper_2410_08859_amd.inputs import workload_marginals

pytestmark = pytest.mark.gpu


def cfg32():
    n = 32
    return B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=4.0 / n ** 2, lam=1.0, cell=4,
                                   precision=64, sinkhorn_err=1e-8, sinkhorn_max_iter=200,
                                   lenience=0.0, box_cap=32, getweights=B.GW_LINE)


def test_device_inputs_and_outputs_match_host_ones():
    mu, nu = workload_marginals("grid32")
    n = 32
    c = cfg32()
    stream = torch.cuda.current_stream().cuda_stream
    dmu_in = torch.from_numpy(mu.ravel().copy()).cuda()
    dnu_in = torch.from_numpy(nu.ravel().copy()).cuda()
    print("[boundary] device inputs", flush=True)
    hh = B.dd_uot_init(c, mu, nu, stream=stream)
    hd = B.dd_uot_init(c, dmu_in, dnu_in, stream=stream)
    try:
        B.dd_uot_iterate(hh, 4)
        B.dd_uot_iterate(hd, 4)
        np.testing.assert_array_equal(B.dd_uot_history(hd, 0), B.dd_uot_history(hh, 0))
        # marginals into device tensors
        px_h, py_h = B.dd_uot_marginals(hh, 0, n, n)
        bufs = (torch.empty(n * n, dtype=torch.float64, device="cuda"),
                torch.empty(n * n, dtype=torch.float64, device="cuda"))
        px_d, py_d = B.dd_uot_marginals(hd, 0, n, n, out=bufs)
        assert px_d.is_cuda and px_d.shape == (n, n)
        np.testing.assert_array_equal(px_d.cpu().numpy(), px_h)
        np.testing.assert_array_equal(py_d.cpu().numpy(), py_h)
        # gradient scaled by the seed on the device, host and device outputs
        B.dd_uot_score(hh, 0)
        B.dd_uot_score(hd, 0)
        g1 = B.dd_uot_backward(hh, 0, n, n)
        g3 = B.dd_uot_backward(hh, 0, n, n, gout=-2.5)
        dev = (torch.empty(n * n, dtype=torch.float64, device="cuda"),
               torch.empty(n * n, dtype=torch.float64, device="cuda"))
        g3d = B.dd_uot_backward(hd, 0, n, n, gout=-2.5, out=dev)
        for a, b, bd in zip(g1, g3, g3d):
            np.testing.assert_array_equal(b, -2.5 * a)
            np.testing.assert_array_equal(bd.cpu().numpy(), b)
    finally:
        B.dd_uot_destroy(hh)
        B.dd_uot_destroy(hd)


def test_autograd_on_device_tensors_matches_host_tensors():
    mu, nu = workload_marginals("grid32")
    c = cfg32()
    vals, grads = [], []
    for device in ("cpu", "cuda"):
        m = torch.tensor(mu, dtype=torch.float64, device=device, requires_grad=True)
        v = torch.tensor(nu, dtype=torch.float64, device=device, requires_grad=True)
        w = uot_value(m, v, c, 6)
        (3.0 * w).backward()
        assert m.grad.device.type == device
        vals.append(float(w.detach()))
        grads.append((m.grad.cpu().numpy(), v.grad.cpu().numpy()))
    assert vals[1] == vals[0]
    for a, b in zip(grads[1], grads[0]):
        np.testing.assert_array_equal(a, b)
