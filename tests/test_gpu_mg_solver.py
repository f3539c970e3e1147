"""Multigrid as a solver and the damped Jacobi smoother on the GPU.

The structure of the paper's Table 1: with damped Jacobi (omega 0.6, one sweep) and MG as a
solver on a 2D mesh of 730^2 nodes in 3x3 regions, the regional method's residual history is the
composite method's (the oracle's plain composite multigrid), cycle by cycle.  The table's own
numbers are not reproducible (its right-hand side and initial guess are not given).
"""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu


def test_table1_structure_jacobi_histories(hip_device):
    import torch

    from oracle import assembly, composite, regional
    from oracle.regions import Layout

    o, e = synth.tensor_layout([[244] * 3, [244] * 3])
    w = synth.Workload("table1", 2, 1, o, e, 15, 4, 1, "fd5", seed=0)
    lay = Layout(2, o, e, 15)
    opt = regional.Options(nlevels=4, degree=1, smoother="jacobi", jacobi_omega=0.6)
    clv = composite.setup(lay, assembly.composite_fd5(lay), opt)
    b = synth.rhs(w)
    h = harness.gpu_problem(w, nlevels=4, cheb_degree=1, smoother=1, jacobi_omega=0.6)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-12, maxit=300, method="mg")
    assert out["converged"]
    n = out["iterations"]
    xc, hc = composite.stationary(clv, b.reshape(-1), np.zeros(b.size), opt, n)
    hc = np.asarray(hc)
    hg = np.asarray(out["history"][: n + 1])
    np.testing.assert_allclose(hg[:30], hc[:30], rtol=1e-9)  # cycle by cycle
    big = hc > 1e-9
    np.testing.assert_allclose(hg[big], hc[big], rtol=1e-6)
    assert hc[-1] <= 1e-12 and (n == 1 or hc[-2] > 1e-12)  # same stopping cycle
    harness.assert_close(x.cpu().numpy(), xc, 1e-10)
    print(f"[table1] {n} cycles to 1e-12, asymptotic factor {(hc[-1] / hc[-11]) ** 0.1:.3f}", flush=True)
    h.close()


@pytest.mark.parametrize("name", ["c2_small", "c5_small", "c1_small"])
def test_chebyshev_mg_as_solver(hip_device, name):
    import torch

    from oracle import regional

    w = synth.workload(name)
    lay, levels, opt = harness.oracle_problem(w)
    b = synth.rhs(w)
    h = harness.gpu_problem(w)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8, maxit=100, method="mg")
    n = out["iterations"]
    xr, hr = regional.stationary(levels, lay.to_regional(b), lay.zeros_regional(), opt, n)
    np.testing.assert_allclose(out["history"][: n + 1], hr, rtol=1e-8)
    assert out["converged"] and hr[-1] <= 1e-8 < hr[-2]
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(xr).reshape(-1), 1e-10)
    h.close()


def test_jacobi_smoothed_pcg(hip_device):
    import torch

    from oracle import regional

    w = synth.workload("c2_small")
    lay, levels, opt = harness.oracle_problem(w, smoother="jacobi", jacobi_omega=0.6)
    b = synth.rhs(w)
    ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-8, maxit=200)
    h = harness.gpu_problem(w, smoother=1, jacobi_omega=0.6)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8, maxit=200)
    assert out["iterations"] == ref.iterations
    np.testing.assert_allclose(out["history"], ref.history, rtol=1e-8)
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(ref.x).reshape(-1), 1e-10)
    h.close()


def test_mg_solver_reports_maxit(hip_device):
    import torch

    w = synth.workload("c2_small")
    h = harness.gpu_problem(w)
    b = harness.to_dev(synth.rhs(w))
    x = torch.zeros_like(b)
    out = h.solve(b, x, rtol=1e-14, maxit=2, method="mg", raise_on_fail=False)
    assert out["status"] == "RMG_ERR_NOT_CONVERGED" and out["iterations"] == 2 and len(out["history"]) == 3
    h.close()


@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
def test_table1_rectangular_histories(hip_device, smoother):
    """Table 1(b): 700 x 720 nodes in 3x3 regions (extents 234 and 241/240, not 3^k + 1), 4 levels,
    one smoothing step before and after the coarse correction, MG as a solver to 1e-12.  The GPU's
    regional history is the oracle's regional history cycle by cycle.  Serial structured MG on the
    whole mesh coarsens by the same rule on a different lattice (every third node of 700/720
    instead of the union of the regions' points), so its history is close, not identical, and it
    stops at the same cycle."""
    import torch

    from oracle import assembly, composite, regional
    from oracle.regions import Layout

    w = synth.workload("table1_rect")
    jac = smoother == "jacobi"
    lay, levels, opt = harness.oracle_problem(w, **(dict(smoother="jacobi", jacobi_omega=0.6) if jac else {}))
    b = synth.rhs(w)
    print(f"[table1-rect] {smoother}: GPU solve", flush=True)
    h = harness.gpu_problem(w, **(dict(smoother=1, jacobi_omega=0.6) if jac else {}))
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-12, maxit=300, method="mg")
    assert out["converged"]
    n = out["iterations"]
    xr, hr = regional.stationary(levels, lay.to_regional(b), lay.zeros_regional(), opt, n)
    hr = np.asarray(hr)
    hg = np.asarray(out["history"][: n + 1])
    np.testing.assert_allclose(hg[:30], hr[:30], rtol=1e-9)
    big = hr > 1e-9
    np.testing.assert_allclose(hg[big], hr[big], rtol=1e-6)
    assert hr[-1] <= 1e-12 and hr[-2] > 1e-12  # same stopping cycle
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(xr).reshape(-1), 1e-10)
    h.close()
    one = Layout(2, [[0, 0]], [list(w.composite_shape_xyz)], w.dirichlet_mask)
    sl = composite.setup(one, assembly.composite_fd5(one), opt)
    hs = np.asarray(composite.stationary(sl, b.reshape(-1), np.zeros(b.size), opt, n + 2)[1])
    ns = int(np.argmax(hs <= 1e-12))
    d = np.abs(hr[1:] - hs[1:n + 1]) / hs[1:n + 1]
    print(f"[table1-rect] {smoother}: {n} cycles regional, {ns} structured, histories within {d.max():.3%}",
          flush=True)
    assert abs(ns - n) <= 1 and 1e-6 < d.max() < 0.25


def test_per_level_solve_times(hip_device):
    """rmg_solve_info.level_ms: with profiling on, each region level's share of the preconditioner
    (smoothing, residual, transfers; the coarse solve on the last level) is positive and the shares
    add up to less than the solve; zero with profiling off and beyond the hierarchy."""
    import torch

    w = synth.workload("c2_mid")
    h = harness.gpu_problem(w)
    b = harness.to_dev(synth.rhs(w))
    x = torch.zeros_like(b)
    out = h.solve(b, x)
    assert len(out["level_ms"]) == 12 and all(v == 0.0 for v in out["level_ms"])
    h.profile(True)
    for method in ("pcg", "mg"):
        x.zero_()
        out = h.solve(b, x, method=method)
        lm = out["level_ms"]
        print(f"[level-ms] {method}: {[round(v, 3) for v in lm[:w.nlevels]]} of {out['solve_ms']:.2f} ms", flush=True)
        assert all(v > 0.0 for v in lm[:w.nlevels]) and all(v == 0.0 for v in lm[w.nlevels:])
        assert sum(lm) < out["solve_ms"]
    h.profile(False)
    x.zero_()
    assert all(v == 0.0 for v in h.solve(b, x)["level_ms"])
    h.close()
