"""The allocation-free backward entry point (ph_mlp_backward_noalloc) against ph_mlp_backward:
the same gradient and loss bit for bit, on two calls in a row (the second with fewer rows, so
the fixed scratch still holds the first call's larger partials), called through the C ABI."""
import ctypes

import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import rel_l2

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def test_noalloc_backward_equals_allocating_backward(gpu_lib):
    import torch
    print("no-alloc backward: 8192 rows then 777 rows", flush=True)
    lib = gpu_lib.load()
    rng = np.random.default_rng(31)
    p = _t(omlp.init_params(11) * 0.9)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for m in (gpu_lib.MLP_NOALLOC_MAX_ROWS, 777):
        X = _t(rng.normal(size=(m, 8)))
        y = _t((rng.uniform(size=m) < 0.3).astype(np.float32))
        g_ref, l_ref = gpu_lib.mlp_backward(p, X, y, 2.5)
        g = torch.full((gpu_lib.MLP_NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        st = lib.ph_mlp_backward_noalloc(ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()), ctypes.c_float(2.5), ctypes.c_int64(m),
                                         ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr()), stream)
        assert st == gpu_lib.PH_OK
        torch.cuda.synchronize()
        assert np.array_equal(g.cpu().numpy().view(np.uint32), g_ref.cpu().numpy().view(np.uint32)), m
        assert np.array_equal(loss.cpu().numpy().view(np.uint32), l_ref.cpu().numpy().view(np.uint32)), m
        # and against the FP64 oracle, to the bar of the allocating call's own test
        loss64, g64 = omlp.loss_and_grad(p.cpu().numpy().astype(np.float64), X.cpu().numpy().astype(np.float64),
                                         y.cpu().numpy().astype(np.float64), 2.5)
        assert rel_l2(g.cpu().numpy().astype(np.float64), g64) <= 1e-4
    # sizes beyond the fixed scratch are refused before any launch
    big = gpu_lib.MLP_NOALLOC_MAX_ROWS + 1
    Xb = torch.zeros((big, 8), dtype=torch.float32, device="cuda")
    yb = torch.zeros(big, dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.PhError) as e:
        gpu_lib.mlp_backward_noalloc(p, Xb, yb, 1.0, g, loss)
    assert e.value.status == gpu_lib.PH_EINVAL
    with pytest.raises(gpu_lib.PhError) as e:
        gpu_lib.mlp_backward_noalloc(p, Xb[:0], yb[:0], 1.0, g, loss)
    assert e.value.status == gpu_lib.PH_EINVAL
