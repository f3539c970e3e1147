"""Edge cases of the regional method on the GPU, each against the oracle: one region (no
interfaces), a zero right-hand side, the shallowest hierarchy (two levels), Dirichlet data on one
face only, CG stopped by maxit, the smallest coarsenable regions (one coarse cell per region,
also with learned weights), and uneven 2D regions listed in a shuffled order."""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu


def solve_both(w, rtol=1e-8, maxit=100, raise_on_fail=True, **opts):
    import torch

    from oracle import regional

    lay, levels, opt = harness.oracle_problem(w)
    b = synth.rhs(w)
    ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=rtol, maxit=maxit)
    h = harness.gpu_problem(w, **opts)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=rtol, maxit=maxit, raise_on_fail=raise_on_fail)
    h.close()
    return out, x.cpu().numpy(), ref, lay.to_composite_owner(ref.x).reshape(-1)


def box_workload(name, slabs, mask, nlevels, degree, pde="laplace", seed=0):
    o, e = synth.tensor_layout(slabs)
    dim = len(slabs)
    h = 1.0 / (int((o + e).max(axis=0)[0]) - 1)
    return synth.Workload(name, dim, 1, o, e, mask, nlevels, degree, pde, h=h, seed=seed)


@pytest.mark.parametrize("kernel", [1, 2])
def test_single_region(hip_device, kernel):
    w = box_workload("one", [[28], [28], [28]], 63, 3, 3)
    out, x, ref, xref = solve_both(w, stencil_kernel=kernel)
    assert out["iterations"] == ref.iterations
    harness.assert_close(x, xref, 1e-10)


def test_zero_rhs(hip_device):
    import torch

    w = synth.workload("c2_small")
    h = harness.gpu_problem(w)
    b = torch.zeros(int(np.prod(w.composite_shape_xyz)), dtype=torch.float64, device="cuda:0")
    x = torch.ones_like(b)
    out = h.solve(b, x)
    assert out["converged"] and out["iterations"] == 0 and torch.count_nonzero(x) == 0
    h.close()


def test_two_levels(hip_device):
    w = synth.workload("c2_small")
    w = synth.Workload(w.name, w.dim, w.ndof, w.origins, w.extents, w.dirichlet_mask, 2, w.cheb_degree, w.pde,
                       h=w.h, seed=w.seed)
    out, x, ref, xref = solve_both(w)
    assert out["iterations"] == ref.iterations
    harness.assert_close(x, xref, 1e-10)


def test_dirichlet_on_one_face(hip_device):
    w = box_workload("face", [[10, 10], [10, 10], [10, 10]], 1, 3, 3)  # x-low face only
    out, x, ref, xref = solve_both(w, stencil_kernel=1)
    assert out["iterations"] == ref.iterations
    harness.assert_close(x, xref, 1e-10)


def test_maxit_returns_last_iterate(hip_device):
    w = synth.workload("c2_small")
    out, x, ref, xref = solve_both(w, rtol=1e-14, maxit=3, raise_on_fail=False)
    assert out["status"] == "RMG_ERR_NOT_CONVERGED" and not out["converged"] and not ref.converged
    assert out["iterations"] == ref.iterations == 3
    harness.assert_close(x, xref, 1e-10)


def test_smallest_regions(hip_device):
    """Regions of 4^3 nodes: one coarse cell each, coarse regions of 2^3."""
    w = box_workload("tiny", [[4, 4, 4], [4, 4], [4, 4, 4]], 63, 2, 2)
    out, x, ref, xref = solve_both(w)
    assert out["iterations"] == ref.iterations
    harness.assert_close(x, xref, 1e-10)


def test_smallest_regions_learned_weights(hip_device):
    from oracle import learned
    from oracle.regions import Layout
    from paper_2103_11962_amd import regmg

    w = box_workload("tiny_c5", [[4, 4, 4], [4, 4], [4, 4, 4]], 63, 2, 2, pde="diffusion", seed=2)
    lay = Layout(w.dim, w.origins, w.extents, w.dirichlet_mask)
    theta = synth.mlp_params(seed=4)
    W = learned.node_weights(lay, lay.coarsen(), theta.astype(np.float64), synth.jump_coefficients(w))
    Wr = np.concatenate([Wk.reshape(-1, 8) for Wk in W])
    h = harness.gpu_problem(w, setup=False)
    h.set_learned_prolongator(theta)
    h.setup_hierarchy(nlevels=2, cheb_degree=2, judge_cycles=0)
    assert h.prolongator_info()["kind"] == regmg.P_LEARNED
    Wg = h.prolongator_weights(lay.n_regional)
    assert np.abs(Wg - Wr).max() <= 1e-5 and np.all(Wg[Wr == 0.0] == 0.0)
    h.close()


def test_uneven_2d_regions_in_shuffled_order(hip_device):
    o, e = synth.tensor_layout([[10, 19, 28], [19, 10]])
    perm = np.random.default_rng(0).permutation(len(o))
    w = synth.Workload("shuffled", 2, 1, o[perm], e[perm], 15, 3, 2, "fd5", seed=0)
    out, x, ref, xref = solve_both(w)
    assert out["iterations"] == ref.iterations
    harness.assert_close(x, xref, 1e-10)


@pytest.mark.parametrize("call", ["composite_stencil", "region_stencil"])
def test_rejected_operator_leaves_no_stale_hierarchy(hip_device, call):
    """An operator call rejected on its arguments changes nothing: the hierarchy (and its recorded
    CG graphs) still solves bit for bit as before.  One rejected only after it has started
    replacing level 0 (non-finite values found on the device) leaves no hierarchy: the next solve
    reports RMG_ERR_NOT_SETUP instead of replaying kernels over the old operator's buffers."""
    import torch

    from paper_2103_11962_amd import regmg

    w = synth.workload("c1_small")
    h = harness.gpu_problem(w, use_graph=1)
    b = harness.to_dev(synth.rhs(w))
    x0 = torch.zeros_like(b)
    out0 = h.solve(b, x0)  # records the CG graphs
    good = synth.fd5_composite_stencil(w)
    with pytest.raises(regmg.RmgError) as e:
        if call == "composite_stencil":
            h.set_composite_stencil(3, good)  # wrong stencil size for 2D
        else:
            h.set_region_stencil(w.nreg, 5, np.zeros((5, 10)))  # no such region
    assert e.value.status == "RMG_ERR_ARG"
    x1 = torch.zeros_like(b)
    out1 = h.solve(b, x1)
    assert torch.equal(x1, x0) and out1["iterations"] == out0["iterations"]
    bad = good.copy()
    bad[2, 50] = np.nan
    with pytest.raises(regmg.RmgError) as e:
        if call == "composite_stencil":
            h.set_composite_stencil(5, bad)
        else:
            h.set_region_stencil(0, 5, np.full((5, int(np.prod(w.extents[0]))), np.nan))
    assert e.value.status == "RMG_ERR_NUMERIC"
    x2 = torch.zeros_like(b)
    with pytest.raises(regmg.RmgError) as e:
        h.solve(b, x2)
    assert e.value.status == "RMG_ERR_NOT_SETUP"
    # a valid operator and a new set-up bring the solve back
    h.set_composite_stencil(5, good)
    h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, use_graph=1)
    x3 = torch.zeros_like(b)
    out3 = h.solve(b, x3)
    assert torch.equal(x3, x0) and out3["iterations"] == out0["iterations"]
    h.close()
