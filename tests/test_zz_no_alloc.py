"""The entry point that allocates no device memory: rmg_convergence_factor_noalloc against
rmg_convergence_factor on the same handle (same kernels, same order: bit for bit), on two calls
in a row whose second has a smaller finest level (the shared per-GPU work array keeps the first
call's contents), then a problem too large for the array."""
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu


def test_noalloc_matches_allocating_entry_point(hip_device):
    import torch

    from paper_2103_11962_amd import regmg

    for name, opts in (("c2_mid", dict(stencil_kernel=2)), ("c2_small", dict(precision=1)), ("c1_small", {})):
        w = synth.workload(name)
        print(f"[no-alloc] {name} {opts}", flush=True)
        h = harness.gpu_problem(w, **opts)
        n0 = regmg.kernel_launches()
        rho = h.convergence_factor_noalloc(7)
        n1 = regmg.kernel_launches()
        rho_ref = h.convergence_factor(7)
        assert rho == rho_ref, (name, rho, rho_ref)
        assert 0.0 < rho < 1.0 and n1 > n0
        torch.cuda.synchronize()
        h.close()
    w = synth.workload("c2_octant")  # 4.4M regional rows: beyond the 1,048,576-dof array
    h = harness.gpu_problem(w)
    with pytest.raises(regmg.RmgError) as e:
        h.convergence_factor_noalloc(2)
    assert e.value.status == "RMG_ERR_ARG" and "scratch" in str(e.value)
    h.close()
