"""The allocation-free gradient entry point (mk_mlp_grad_static, whose workspace is a
file-scope device array) against mk_mlp_grad with a caller workspace, through the C-ABI:
two calls in a row, the second with a smaller minibatch, and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2305_17813_amd import native
from parity import say

pytestmark = pytest.mark.gpu

N_PARAMS, N_IN, N_OUT = 5187, 12, 3
MAX_SAMPLES = 16384  # MK_MLP_GRAD_STATIC_MAX
MK_ERR_INVALID_ARG, MK_ERR_CAPACITY = 1, 3


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _problem(seed, n):
    rng = np.random.default_rng(seed)
    f = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda().contiguous()
    return (f(rng.normal(0, 0.3, N_PARAMS)), f(rng.normal(0, 1, (n, N_IN))),
            f(rng.normal(0, 1, (n, N_OUT))), f((rng.random((n, N_OUT)) < 0.8).astype(np.float32)))


def _with_workspace(L, s, p, X, T, M):
    n = X.shape[0]
    ws = torch.empty(L.mk_mlp_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    g = torch.full((N_PARAMS,), float("nan"), device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    st = L.mk_mlp_grad(_p(p), _p(X), _p(T), _p(M), n, _p(g), _p(ws), ws.numel(), _p(loss), s)
    assert st == 0, st
    return g, loss


def _static(L, s, p, X, T, M):
    g = torch.full((N_PARAMS,), float("nan"), device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    st = L.mk_mlp_grad_static(_p(p), _p(X), _p(T), _p(M), X.shape[0], _p(g), _p(loss), s)
    assert st == 0, st
    return g, loss


def test_static_workspace_gradient_equals_the_workspace_entry_point():
    L = native.load()
    torch.cuda.set_device(0)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for seed, n in [(11, 5000), (12, 300)]:  # the second call is smaller than the first
        say(f"case: mk_mlp_grad_static n={n}")
        p, X, T, M = _problem(seed, n)
        g_ref, loss_ref = _with_workspace(L, s, p, X, T, M)
        g, loss = _static(L, s, p, X, T, M)
        torch.cuda.synchronize()
        # both run the same deterministic gradient kernels: equal bit for bit
        assert torch.equal(g, g_ref)
        assert bool(torch.isfinite(g).all())
        # the loss is a sum of block partials added in arrival order
        assert abs(float(loss) - float(loss_ref)) <= 1e-12 * max(1.0, abs(float(loss_ref)))


def test_static_workspace_gradient_rejects_sizes_beyond_its_limit():
    L = native.load()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p, X, T, M = _problem(13, 4)
    g = torch.zeros(N_PARAMS, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    # the size check comes before any launch, so the short inputs are never read
    assert L.mk_mlp_grad_static(_p(p), _p(X), _p(T), _p(M), MAX_SAMPLES + 1, _p(g), _p(loss), s) \
        == MK_ERR_CAPACITY
    assert L.mk_mlp_grad_static(_p(p), _p(X), _p(T), _p(M), 0, _p(g), _p(loss), s) == MK_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((g == 0).all())
