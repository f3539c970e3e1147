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


def test_provider_failure_mid_setup(hip_device):
    """A provider that runs dry partway through setup: the setup fails with RMG_ERR_OOM, the
    handle can still be closed, and every buffer it did get is returned."""
    import torch

    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    state = {"left": None}

    def alloc(nbytes, ctx):
        if state["left"] is not None:
            if state["left"] == 0:
                return None
            state["left"] -= 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=0, stream=torch.cuda.current_stream(0))

    def free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    prov = regmg.Allocator(regmg.ALLOC_FN(alloc), regmg.FREE_FN(free), None)
    h = regmg.Handle(0, allocator=prov)
    h.build_regions(w.dim, w.ndof, w.extents, w.origins, w.dirichlet_mask)
    h.assemble_q1(regmg.PDE_LAPLACE, w.h)
    state["left"] = 25  # a few buffers more, then nothing
    with pytest.raises(regmg.RmgError) as e:
        h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree)
    assert e.value.status == "RMG_ERR_OOM"
    state["left"] = None  # the provider recovers: a new setup succeeds and solves
    h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree)
    b = harness.to_dev(synth.rhs(w))
    x = torch.zeros_like(b)
    assert h.solve(b, x)["converged"]
    h.close()
    del b, x
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
