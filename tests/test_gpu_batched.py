"""Batched uneven regions: persistent tile launches, autotuned launch shapes and HIP-graph
replay of the CG iteration, each checked against the eager FP64 path and the oracle."""
import os

import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu


def solve(h, b, n, **kw):
    import torch

    x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8, maxit=100, **kw)
    return x.cpu().numpy(), out


@pytest.mark.parametrize("name,precision", [("c4_small", 0), ("c4_small", 1), ("c2_mid", 0), ("c1", 0)])
def test_graph_replay_matches_eager(hip_device, name, precision):
    """Graph-replayed CG iterations give the eager result bit for bit; replays are interleaved
    with the program's own eager work and synchronisations, and every replay is checked."""
    import torch

    w = synth.workload(name)
    b = synth.rhs(w)
    n = int(np.prod(b.shape))
    he = harness.gpu_problem(w, precision=precision)
    xe, oe = solve(he, b, n)
    hg = harness.gpu_problem(w, precision=precision, use_graph=1)
    for rep in range(3):
        xg, og = solve(hg, b, n)
        assert og["iterations"] == oe["iterations"], rep
        assert np.array_equal(xg, xe), (rep, harness.max_rel_err(xg, xe))
        assert og["history"] == oe["history"]
        # eager work between replays: a V-cycle and a torch reduction, synchronised
        z = torch.empty(n, dtype=torch.float64, device="cuda:0")
        hg.apply_vcycle(harness.to_dev(b), z)
        torch.cuda.synchronize()
        assert torch.isfinite(z).all()
    he.close()
    hg.close()


def test_autotuned_solve_and_cache(hip_device, tmp_path):
    """Autotuned launch shapes leave the FP64 solution at oracle parity; the second setup reads
    every choice back from the cache file."""
    from oracle import regional

    w = synth.workload("c4_small")
    lay, levels, opt = harness.oracle_problem(w)
    b = synth.rhs(w)
    ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-8, maxit=100)
    xref = lay.to_composite_owner(ref.x).reshape(-1)
    cache = str(tmp_path / "tune.txt")
    h = harness.gpu_problem(w, autotune=1, autotune_cache=cache)
    report = h.tune_report()
    assert report.count("level") == w.nlevels - 1 and "cached" not in report
    x, out = solve(h, b, lay.n_composite)
    assert out["iterations"] == ref.iterations
    harness.assert_close(x, xref, 1e-10)
    h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, autotune=1, autotune_cache=cache)
    assert h.tune_report().count("cached") == w.nlevels - 1
    x2, out2 = solve(h, b, lay.n_composite)
    assert np.array_equal(x2, x)
    assert os.path.getsize(cache) > 0
    h.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_region_by_region_matches_batched(hip_device, precision):
    """The unbatched baseline (one node-parallel launch per region) computes exactly what one
    batched node-parallel launch computes, and stays at oracle parity in FP64."""
    from oracle import regional

    w = synth.workload("c4_small")
    b = synth.rhs(w)
    n = int(np.prod(b.shape))
    hb = harness.gpu_problem(w, precision=precision, stencil_kernel=1)
    hr = harness.gpu_problem(w, precision=precision, batched=0)
    xb, ob = solve(hb, b, n)
    xr, orr = solve(hr, b, n)
    assert orr["iterations"] == ob["iterations"] and np.array_equal(xr, xb)
    if precision == 0:
        lay, levels, opt = harness.oracle_problem(w)
        ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-8, maxit=100)
        assert orr["iterations"] == ref.iterations
        harness.assert_close(xr, lay.to_composite_owner(ref.x).reshape(-1), 1e-10)
    else:
        assert orr["converged"] and orr["true_relres"] <= 1e-8
    hb.close()
    hr.close()
