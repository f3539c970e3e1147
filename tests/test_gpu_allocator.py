"""The caller's device memory provider (rmg_create's allocator): a handle whose buffers all come
from PyTorch's caching allocator computes bit for bit what a hipMalloc handle computes, its
buffers show in torch's accounting while it lives, and every one is returned when it closes."""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu


def solve(w, torch_allocator, **opts):
    import torch

    h = harness.gpu_problem(w, torch_allocator=torch_allocator, **opts)
    b = harness.to_dev(synth.rhs(w))
    x = torch.zeros_like(b)
    out = h.solve(b, x, rtol=1e-8, maxit=100)
    torch.cuda.synchronize()
    return h, x.cpu().numpy(), out


@pytest.mark.parametrize("case", ["c2_small", "c5_small", "hybrid"])
def test_torch_allocator(hip_device, case):
    import torch

    if case == "hybrid":
        o, e = synth.tensor_layout([[10] * 3] * 3)
        w = synth.Workload("fd7_10", 3, 1, o, e, 63, 3, 2, "fd7", seed=0)
        opts = dict(setup=True, smoother=4, jacobi_omega=1.0, hybrid=1, cycle_gamma=2)
    else:
        w = synth.workload(case)
        opts = {}
    h0, x0, out0 = solve(w, False, **opts)
    h0.close()
    del h0  # with it the harness's own input tensors
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    h1, x1, out1 = solve(w, True, **opts)
    held = torch.cuda.memory_allocated() - before
    assert held > 0  # the library's buffers came from torch
    np.testing.assert_array_equal(x1, x0)
    assert out1["iterations"] == out0["iterations"] and out1["history"] == out0["history"]
    assert out1["setup_ms"] > 0.0
    h1.close()
    h1.__dict__.pop("_keep", None)  # the harness's input tensor (element coefficients), not a library buffer
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
