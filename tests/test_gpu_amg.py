"""AMG coarse solver below the region hierarchy (Section 3.5, second coarse-level option) on the
GPU against the oracle: every AMG level's matrix and smoothed prolongator (scalar problems, and 3D
elasticity with the rigid-body near-null space on node aggregates), one region V-cycle, PCG
histories, the FP32 V-cycle, graph replay, option errors, and the full-size 3D Laplacian with
three region levels, whose coarsest composite operator (37^3 = 50,653 dofs) is too large for the
dense inverse.
"""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu

# (workload, region levels, rows of the directly solved AMG level)
CASES = [("c2_mid", 2, 200), ("c1", 2, 100), ("uneven3d_small", 2, 30), ("uneven_c4_small", 3, 40),
         ("c2_small", 2, 20), ("c3_small", 2, 200), ("c3_small", 2, 60)]
IDS = [f"{c[0]}-{c[2]}" for c in CASES]


@pytest.fixture(scope="module")
def problems(hip_device):
    cache = {}

    def get(case):
        if case not in cache:
            name, nl, cs = case
            w = synth.workload(name)
            print(f"[gpu-amg] set up {name} with {nl} region levels, AMG down to {cs} rows", flush=True)
            h = harness.gpu_problem(w, nlevels=nl, coarse_amg=1, amg_coarse_size=cs)
            o = harness.oracle_problem(w, nlevels=nl, coarse_amg=True, amg_coarse_size=cs)
            cache[case] = (w, h, o)
        return cache[case]

    yield get
    for w, h, o in cache.values():
        h.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_amg_levels(problems, case):
    """Aggregates, smoothed prolongators and Galerkin products of every AMG level."""
    w, h, (lay, levels, opt) = problems(case)
    ref = levels[-1].amg
    assert h.amg_levels() == len(ref) >= 2
    for l, L in enumerate(ref):
        A = h.amg_matrix(l, 0).toarray()
        harness.assert_close(A, L.A.toarray(), 1e-12, what=repr(l))
        if L.P is not None:
            P = h.amg_matrix(l, 1).toarray()
            assert P.shape == L.P.shape
            harness.assert_close(P, L.P.toarray(), 1e-13, what=repr(l))


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_vcycle_with_amg_coarse_solve(problems, case):
    import torch

    from oracle import regional

    w, h, (lay, levels, opt) = problems(case)
    b = synth.rhs(w)
    z = torch.empty(lay.n_composite, dtype=torch.float64, device="cuda:0")
    h.apply_vcycle(harness.to_dev(b), z)
    ref = lay.to_composite_owner(regional.vcycle(levels, lay.to_regional(b), opt)).reshape(-1)
    harness.assert_close(z.cpu().numpy(), ref, 1e-12)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_pcg_with_amg_coarse_solve(problems, case):
    import torch

    from oracle import regional

    w, h, (lay, levels, opt) = problems(case)
    b = synth.rhs(w)
    ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-8)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8)
    assert out["iterations"] == ref.iterations and ref.converged
    np.testing.assert_allclose(out["history"], ref.history, rtol=1e-8)
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(ref.x).reshape(-1), 1e-10)


def test_fp32_vcycle_and_graph_replay(hip_device):
    """The FP32 V-cycle gathers into and scatters from the FP64 AMG; graph replays of the CG
    iterations equal the eager solve."""
    import torch

    w = synth.workload("c2_mid")
    b = harness.to_dev(synth.rhs(w))
    outs = []
    for kw in (dict(precision=1), dict(use_graph=1), dict()):
        h = harness.gpu_problem(w, nlevels=2, coarse_amg=1, amg_coarse_size=200, **kw)
        x = torch.zeros_like(b)
        out = h.solve(b, x, rtol=1e-8)
        if kw.get("use_graph"):
            x2 = torch.zeros_like(b)
            out2 = h.solve(b, x2, rtol=1e-8)  # replay of the recorded graphs
            assert torch.equal(x, x2) and out2["iterations"] == out["iterations"]
        assert out["converged"] and out["true_relres"] <= 1e-8
        outs.append((out, x))
        h.close()
    (o32, x32), (og, xg), (oe, xe) = outs
    assert torch.equal(xg, xe) and og["iterations"] == oe["iterations"]
    harness.assert_close(x32.cpu().numpy(), xe.cpu().numpy(), 1e-6, floor=1.0)  # FP32 V-cycle: absolute rounding


def test_amg_option_errors(hip_device):
    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    h = harness.gpu_problem(w, setup=False)
    for kw in (dict(amg_coarse_size=0), dict(amg_coarse_size=20001), dict(hybrid=1, smoother=4)):
        with pytest.raises(regmg.RmgError) as e:
            h.setup_hierarchy(nlevels=2, cheb_degree=2, coarse_amg=1, **kw)
        assert e.value.status == "RMG_ERR_ARG"
    h.setup_hierarchy(nlevels=2, cheb_degree=2, coarse_amg=1, amg_coarse_size=20)
    with pytest.raises(regmg.RmgError) as e:
        h.coarse_matrix(7 ** 3)
    assert e.value.status == "RMG_ERR_NOT_SETUP"
    h.setup_hierarchy(nlevels=2, cheb_degree=2)  # back to the direct solver
    assert h.amg_levels() == 0
    h.close()


def test_full_size_three_region_levels(hip_device):
    """3D Q1 Laplacian, 4x4x4 regions of 82^3 (325^3 composite), three region levels: the coarsest
    composite operator has 37^3 = 50,653 dofs, beyond the dense solver; with the AMG coarse solver
    PCG reaches 1e-8 (true residual) in about as many iterations as four region levels with the
    direct solve."""
    import torch

    w = synth.workload("c2")
    b = harness.to_dev(synth.rhs(w))
    h = harness.gpu_problem(w, nlevels=3, coarse_amg=1)
    print(f"[gpu-amg] c2 with 3 region levels: AMG levels {[h.amg_level_info(l)['n'] for l in range(h.amg_levels())]}",
          flush=True)
    assert h.amg_level_info(0)["n"] == 37 ** 3
    x = torch.zeros_like(b)
    out = h.solve(b, x, rtol=1e-8)
    print(f"[gpu-amg] {out['iterations']} PCG iterations, {out['solve_ms']:.1f} ms, true relres "
          f"{out['true_relres']:.2e}", flush=True)
    assert out["converged"] and out["true_relres"] <= 1e-8 and out["iterations"] <= 12
    h.close()
