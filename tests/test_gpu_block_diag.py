"""Nodal-block D~ of elasticity (block_diag = 1; Section 3.2 smoother setup, block reading) against
the oracle with block_diag: the eigenvalue estimates, the smoother, the V-cycle (FP64 Chebyshev
and Jacobi) and PCG (same iteration count, history 1e-10, iterate 1e-10, true residual 1e-8),
element by element; the FP32 V-cycle to its mixed-precision bound; and the option's checks.
"""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3(hip_device):
    w = synth.workload("c3_small")
    lay, levels, opt = harness.oracle_problem(w, block_diag=True)
    return w, lay, levels, opt


def test_block_eigenvalues_and_smoother(c3):
    import torch

    from oracle import regional

    w, lay, levels, opt = c3
    h = harness.gpu_problem(w, block_diag=1)
    for l, L in enumerate(levels[:-1]):
        lam = h.level_info(l)["lambda"]
        assert abs(lam - L.lam) <= 1e-12 * L.lam, (l, lam, L.lam)
    b = synth.rhs(w)
    br = lay.to_regional(b)
    u = torch.empty(lay.n_regional, dtype=torch.float64, device="cuda:0")
    h.smooth(0, harness.to_dev(lay.flatten(br)), u)
    h.close()
    ref = regional.chebyshev(levels[0], lay.zeros_regional(), br, br, opt)
    harness.assert_close(u.cpu().numpy(), lay.flatten(ref), 1e-12, what="block Chebyshev")


def test_block_vcycle_and_pcg(c3):
    import torch

    from oracle import regional

    w, lay, levels, opt = c3
    h = harness.gpu_problem(w, block_diag=1)
    b = synth.rhs(w)
    z = torch.empty(lay.n_composite, dtype=torch.float64, device="cuda:0")
    h.apply_vcycle(harness.to_dev(b), z)
    ref = lay.to_composite_owner(regional.vcycle(levels, lay.to_regional(b), opt)).reshape(-1)
    harness.assert_close(z.cpu().numpy(), ref, 1e-12, what="block V-cycle")
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8, maxit=100)
    h.close()
    rp = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-8, maxit=100)
    assert out["converged"] and rp.converged and out["iterations"] == rp.iterations
    np.testing.assert_allclose(out["history"], rp.history, rtol=1e-10, atol=0)
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(rp.x).reshape(-1), 1e-10, what="block PCG")
    assert out["true_relres"] <= 1e-8
    # the point diagonal's solve, for the record
    hp = harness.gpu_problem(w)
    xp = torch.zeros_like(x)
    outp = hp.solve(harness.to_dev(b), xp, rtol=1e-8, maxit=100)
    hp.close()
    print(f"[gpu-block-diag] c3_small PCG iterations: block {out['iterations']}, point {outp['iterations']}",
          flush=True)


def test_block_jacobi_vcycle(hip_device):
    import torch

    from oracle import regional

    w = synth.workload("c3_small")
    lay, levels, opt = harness.oracle_problem(w, block_diag=True, smoother="jacobi", jacobi_omega=0.6)
    h = harness.gpu_problem(w, block_diag=1, smoother=1, jacobi_omega=0.6)
    b = synth.rhs(w)
    z = torch.empty(lay.n_composite, dtype=torch.float64, device="cuda:0")
    h.apply_vcycle(harness.to_dev(b), z)
    h.close()
    ref = lay.to_composite_owner(regional.vcycle(levels, lay.to_regional(b), opt)).reshape(-1)
    harness.assert_close(z.cpu().numpy(), ref, 1e-12, what="block Jacobi V-cycle")


def test_block_fp32_vcycle_solve(c3):
    import torch

    from oracle import regional
    from paper_2103_11962_amd import regmg

    w, lay, levels, opt = c3
    h = harness.gpu_problem(w, block_diag=1, precision=regmg.PREC_FP32)
    b = synth.rhs(w)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8, maxit=100)
    h.close()
    ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-12, maxit=200)
    assert out["converged"] and out["true_relres"] <= 1e-8, out
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(ref.x).reshape(-1), 1e-6, floor=1.0)


@pytest.mark.parametrize("name,kw", [("c2_small", dict(block_diag=1)),
                                     ("c3_small", dict(block_diag=1, smoother=2)),
                                     ("c3_small", dict(block_diag=2))])
def test_block_diag_checks(hip_device, name, kw):
    from paper_2103_11962_amd import regmg

    w = synth.workload(name)
    h = harness.gpu_problem(w, setup=False)
    with pytest.raises(regmg.RmgError) as e:
        h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, **kw)
    assert e.value.status == "RMG_ERR_ARG"
    h.close()
