"""The closure gradient entry point that allocates nothing (fdtd_closure_grad_static)
against the handle's fdtd_closure_grad, through the C ABI: bitwise equal gradients and
losses on two calls in a row, the second with fewer rows, with the outputs filled with
NaN beforehand; and the row limit of its fixed scratch array."""
import ctypes as C

import numpy as np
import pytest

from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import closure as CL

pytestmark = pytest.mark.gpu


def _static(torch, p_dev, X, T, g, loss, n=None):
    L = B.lib()
    return L.fdtd_closure_grad_static(0, C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                      C.c_void_p(p_dev.data_ptr()), C.c_void_p(X.data_ptr()),
                                      C.c_void_p(T.data_ptr()), X.shape[0] if n is None else n,
                                      C.c_void_p(g.data_ptr()), C.c_void_p(loss.data_ptr()))


def test_static_gradient_is_bitwise_the_handle_gradient(gpu_lib):
    import torch
    rng = np.random.default_rng(2211)
    params = CL.init_params(17)
    params[-129:] += rng.normal(0.0, 0.05, 129).astype(np.float32)   # a non-trivial last layer
    c = B.Closure(max_rows=8192)
    c.set_params(params)
    p_dev = torch.tensor(params, dtype=torch.float32, device="cuda")
    for n in (8192, 1000, 777):
        X = torch.tensor(rng.uniform(-1.0, 1.0, (n, B.NIN)).astype(np.float32), device="cuda")
        T = torch.tensor((0.1 * rng.standard_normal(n)).astype(np.float32), device="cuda")
        loss_h, g_h = c.grad(X, T)
        g = torch.full((B.NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        B.check(_static(torch, p_dev, X, T, g, loss), "grad_static")
        torch.cuda.synchronize()
        gs = g.cpu().numpy()
        assert np.all(np.isfinite(gs))
        assert np.array_equal(gs, g_h), n
        assert float(loss.cpu()[0]) == loss_h
        assert np.abs(g_h).max() > 0
    c.close()


def test_static_gradient_row_limit(gpu_lib):
    import torch
    n = 8192 + 1
    X = torch.zeros((n, B.NIN), dtype=torch.float32, device="cuda")
    T = torch.zeros(n, dtype=torch.float32, device="cuda")
    p_dev = torch.zeros(B.NPARAM, dtype=torch.float32, device="cuda")
    g = torch.full((B.NPARAM,), 7.0, dtype=torch.float32, device="cuda")
    loss = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    assert _static(torch, p_dev, X, T, g, loss) == B.ERANGE
    assert _static(torch, p_dev, X, T, g, loss, n=0) == B.ERANGE
    torch.cuda.synchronize()
    assert bool(torch.all(g == 7.0)) and float(loss.cpu()[0]) == 7.0
