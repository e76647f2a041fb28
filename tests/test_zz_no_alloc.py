"""GPU: the allocation-free loss gradient of the selector's perceptron
(tiledqr_mlp_loss_grad_noalloc) against the allocating entry point
(tiledqr_mlp_loss_grad), through the C ABI.

Both run the same two kernels in the same fixed reduction order, so the
gradient and the loss must agree bit for bit.  Two calls in a row, the second
on fewer samples, show that the shared device array keeps no stale partial
sums from the first; a call above the array's sample limit is rejected on
the host.
"""

import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _grad(torch, lib, fn, P, X, t):
    nparam = P.numel()
    g = torch.full((nparam,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = fn(ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(t.data_ptr()),
            t.numel(), ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr()), stream)
    lib.check(st, fn.__name__)
    torch.cuda.synchronize()
    return g.cpu().numpy(), loss.cpu().numpy()


def test_noalloc_gradient_matches_allocating_entry_point(torch_cuda):
    torch = torch_cuda
    from paper_1104_4475_amd import _lib
    nparam = _lib.tiledqr_mlp_nparam()
    nmax = _lib.tiledqr_mlp_noalloc_max_samples()
    assert nmax == 16384
    rng = np.random.default_rng(41)
    P = torch.from_numpy(rng.standard_normal(nparam).astype(np.float32) * 0.2).cuda()
    # The second call is smaller: stale partial sums of the first would show.
    for n in (5000, 777, nmax):
        _say("noalloc gradient, n = %d" % n)
        X = torch.from_numpy(np.concatenate([rng.uniform(0, 7, (n, 3)), rng.integers(0, 2, (n, 10))],
                                            axis=1).astype(np.float32)).cuda().contiguous()
        t = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
        g_ref, l_ref = _grad(torch, _lib, _lib.tiledqr_mlp_loss_grad, P, X, t)
        g_na, l_na = _grad(torch, _lib, _lib.tiledqr_mlp_loss_grad_noalloc, P, X, t)
        assert np.all(np.isfinite(g_ref)) and np.isfinite(l_ref[0])
        assert np.array_equal(g_na.view(np.uint32), g_ref.view(np.uint32)), \
            "max |diff| %g" % np.max(np.abs(g_na - g_ref))
        assert l_na.view(np.uint32)[0] == l_ref.view(np.uint32)[0]


def test_noalloc_rejects_sizes_above_its_limit(torch_cuda):
    torch = torch_cuda
    from paper_1104_4475_amd import _lib
    nparam = _lib.tiledqr_mlp_nparam()
    n = _lib.tiledqr_mlp_noalloc_max_samples() + 1
    P = torch.zeros(nparam, dtype=torch.float32, device="cuda")
    X = torch.zeros((n, 13), dtype=torch.float32, device="cuda")
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    g = torch.zeros(nparam, dtype=torch.float32, device="cuda")
    st = _lib.tiledqr_mlp_loss_grad_noalloc(ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                            ctypes.c_void_p(t.data_ptr()), n, ctypes.c_void_p(g.data_ptr()), None,
                                            None)
    assert st == _lib.TQR_EINVAL
