"""Region-local Gauss-Seidel (Section 3.4, Algorithm 1) on the GPU against the oracle.

The device sweep walks each region's hyperplanes x + 2y + 4z (x + y for the five-point stencil)
in order, which is the lexicographic sweep's arithmetic; the oracle solves the same triangular
systems with a library routine.  Checked: the smoother's whole regional output (every copy of
every interface dof), the V-cycle with forward and symmetric sweeps on 2D five-/nine-point,
3D Laplace, jump-coefficient and elasticity levels and uneven regions, PCG, and MG as a solver
in the Table 1 setting, whose regional history must equal the oracle's regional history and stay
close to the composite (true Gauss-Seidel) one.
"""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu

CASES = ["c1_small", "c2_small", "c3_small", "c4_small", "c5_small", "uneven2d_small", "uneven3d_small",
         "uneven_tiny3d", "uneven_tiny2d"]
NAMES = {2: "gs", 3: "sgs", 4: "symgs"}


@pytest.mark.parametrize("name", CASES)
def test_gs_smoother_regional_output(hip_device, name):
    import torch

    from oracle import regional

    w = synth.workload(name)
    print(f"[gs] smoother {name}", flush=True)
    lay, levels, opt = harness.oracle_problem(w, smoother="gs", jacobi_omega=0.9)
    br = lay.to_regional(synth.rhs(w))
    ref = regional.gauss_seidel(levels[0], lay.zeros_regional(), br, br, opt)
    h = harness.gpu_problem(w, smoother=2, jacobi_omega=0.9)
    u = torch.empty(lay.n_regional, dtype=torch.float64, device="cuda:0")
    h.smooth(0, harness.to_dev(lay.flatten(br)), u)
    got = u.cpu().numpy()
    harness.assert_close(got, lay.flatten(ref), 1e-12)
    # copies of an interface dof agree after the averaging
    avg = lay.flatten(lay.to_regional(lay.to_composite_avg(lay.unflatten(got))))
    assert np.abs(got - avg).max() <= 1e-15 * np.abs(got).max()
    h.close()


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("smoother", [2, 3, 4])
def test_gs_vcycle(hip_device, name, smoother):
    import torch

    from oracle import regional

    w = synth.workload(name)
    print(f"[gs] vcycle {name} smoother {smoother}", flush=True)
    lay, levels, opt = harness.oracle_problem(w, smoother=NAMES[smoother], jacobi_omega=1.0)
    b = synth.rhs(w)
    h = harness.gpu_problem(w, smoother=smoother, jacobi_omega=1.0)
    z = torch.empty(lay.n_composite, dtype=torch.float64, device="cuda:0")
    h.apply_vcycle(harness.to_dev(b), z)
    ref = lay.to_composite_owner(regional.vcycle(levels, lay.to_regional(b), opt)).reshape(-1)
    harness.assert_close(z.cpu().numpy(), ref, 1e-12)
    h.close()


def test_symmetric_gs_pcg(hip_device):
    import torch

    from oracle import regional

    w = synth.workload("c2_small")
    lay, levels, opt = harness.oracle_problem(w, smoother="sgs", jacobi_omega=1.0)
    b = synth.rhs(w)
    ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-8, maxit=100)
    h = harness.gpu_problem(w, smoother=3, jacobi_omega=1.0)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8, maxit=100)
    assert out["iterations"] == ref.iterations and ref.converged
    np.testing.assert_allclose(out["history"], ref.history, rtol=1e-8)
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(ref.x).reshape(-1), 1e-10)
    h.close()


def test_table1_structure_gauss_seidel(hip_device):
    """2D 730^2 in 3x3 regions, 4 levels, one forward sweep (omega 1) before and after the coarse
    correction, MG as a solver to 1e-12: the GPU's regional history is the oracle's regional
    history cycle by cycle, and it stays within a factor 2 of true Gauss-Seidel's."""
    import torch

    from oracle import assembly, composite, regional
    from oracle.regions import Layout

    o, e = synth.tensor_layout([[244] * 3, [244] * 3])
    w = synth.Workload("table1", 2, 1, o, e, 15, 4, 1, "fd5", seed=0)
    lay = Layout(2, o, e, 15)
    opt = regional.Options(nlevels=4, degree=1, smoother="gs", jacobi_omega=1.0)
    lv = regional.setup(lay, assembly.regional_fd5(lay), opt)
    clv = composite.setup(lay, assembly.composite_fd5(lay), opt)
    b = synth.rhs(w)
    h = harness.gpu_problem(w, nlevels=4, cheb_degree=1, smoother=2, jacobi_omega=1.0)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-12, maxit=300, method="mg")
    assert out["converged"]
    n = out["iterations"]
    xr, hr = regional.stationary(lv, lay.to_regional(b), lay.zeros_regional(), opt, n)
    _, hc = composite.stationary(clv, b.reshape(-1), np.zeros(b.size), opt, n)
    hg = np.asarray(out["history"][: n + 1])
    hr, hc = np.asarray(hr), np.asarray(hc)
    # cycle by cycle; near 1e-12 the two differ by the rounding of the FP64 residual evaluation
    # (a few 1e-17 relative to the initial residual), hence the absolute floor
    np.testing.assert_allclose(hg, hr, rtol=1e-8, atol=1e-15)
    assert hr[-1] <= 1e-12 < hr[-2]
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(xr).reshape(-1), 1e-10)
    ratio = hr[1:] / hc[1:]
    assert np.all(ratio > 0.5) and np.all(ratio < 2.0), ratio
    print(f"[table1 gs] {n} cycles; regional/composite residual ratio {ratio.min():.3f} .. {ratio.max():.3f}",
          flush=True)
    h.close()


def test_table1_rectangular_gauss_seidel(hip_device):
    """Table 1(b)'s Gauss-Seidel column setting: 700 x 720 nodes in 3x3 regions (extents not
    3^k + 1), 4 levels, one forward sweep before and after the coarse correction, MG as a solver
    to 1e-12; the GPU's regional history is the oracle's regional history cycle by cycle."""
    import torch

    from oracle import regional

    w = synth.workload("table1_rect")
    lay, levels, opt = harness.oracle_problem(w, smoother="gs", jacobi_omega=1.0)
    b = synth.rhs(w)
    print("[table1-rect gs] GPU solve", flush=True)
    h = harness.gpu_problem(w, smoother=2, jacobi_omega=1.0)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-12, maxit=300, method="mg")
    assert out["converged"]
    n = out["iterations"]
    xr, hr = regional.stationary(levels, lay.to_regional(b), lay.zeros_regional(), opt, n)
    hr = np.asarray(hr)
    np.testing.assert_allclose(np.asarray(out["history"][: n + 1]), hr, rtol=1e-8, atol=1e-15)
    assert hr[-1] <= 1e-12 < hr[-2]
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(xr).reshape(-1), 1e-10)
    print(f"[table1-rect gs] {n} cycles", flush=True)
    h.close()


def test_gs_option_errors(hip_device):
    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    h = harness.gpu_problem(w, setup=False)
    for bad in (dict(smoother=5), dict(smoother=2, precision=1), dict(smoother=4, jacobi_omega=2.0)):
        with pytest.raises(regmg.RmgError) as e:
            h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, **bad)
        assert e.value.status == "RMG_ERR_ARG"
    h.close()


def test_gs_graph_replay_matches_eager(hip_device):
    """CG half-iterations captured as HIP graphs with the symmetric Gauss-Seidel V-cycle inside:
    every replay gives the eager result bit for bit, with eager work between replays."""
    import torch

    w = synth.workload("c2_small")
    b = harness.to_dev(synth.rhs(w))
    he = harness.gpu_problem(w, smoother=4, jacobi_omega=1.0)
    xe = torch.zeros_like(b)
    oe = he.solve(b, xe, rtol=1e-8, maxit=100)
    hg = harness.gpu_problem(w, smoother=4, jacobi_omega=1.0, use_graph=1)
    for rep in range(3):
        xg = torch.zeros_like(b)
        og = hg.solve(b, xg, rtol=1e-8, maxit=100)
        assert og["iterations"] == oe["iterations"] and og["history"] == oe["history"], rep
        assert torch.equal(xg, xe), rep
        z = torch.empty_like(b)
        hg.apply_vcycle(b, z)
        torch.cuda.synchronize()
        assert torch.isfinite(z).all()
    he.close()
    hg.close()
