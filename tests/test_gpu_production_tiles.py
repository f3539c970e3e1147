"""Parity at the benchmark's launch shape.

The 4x4x4-region benchmark runs its finest level on 2.5D tiles of 768 threads (82 x 8 or 9
x-rows) marching 41 planes, with the region table serving the couplings of every node two or more
nodes inside its region, and b and the old direction read a plane ahead.  The automatic choice
keeps those tiles only on levels with at least 1024 of them, which no oracle-sized problem has, so
here `tile_planes = 41` forces the same shape on 2x2x2 of the benchmark's regions (82^3 each,
composite 163^3, the benchmark's mesh width and 4 levels).  Every stencil operation of the cycle
(first and later Chebyshev steps, the scaled residual before restriction, the CG product) then
runs at that shape and is compared element by element with the oracle (operators, smoother and
V-cycle 1e-12, PCG iterate 1e-10 with the same iteration count and history), and with every
coupling streamed (region_table = 0).
"""
import copy

import numpy as np
import pytest

import synth
from tests import harness

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

OPTS = dict(stencil_kernel=2, tile_planes=41)


@pytest.fixture(scope="module")
def octant(hip_device):
    from oracle import regional

    w = synth.workload("c2_octant")
    print("[gpu-production-tiles] oracle set-up of c2_octant", flush=True)
    lay, levels, opt = harness.oracle_problem(w)
    b = synth.rhs(w)
    br = lay.to_regional(b)
    ref_v = lay.to_composite_owner(regional.vcycle(levels, br, opt)).reshape(-1)
    ref_s = lay.flatten(regional.chebyshev(levels[0], lay.zeros_regional(), br, br, opt))
    ref_pcg = regional.pcg(levels, br, opt, rtol=1e-8, maxit=100)
    return dict(w=w, lay=lay, b=b, br=br, levels=levels, opt=opt, ref_v=ref_v, ref_s=ref_s, ref_pcg=ref_pcg)


def run(o, **kw):
    import torch

    w, lay, levels = o["w"], o["lay"], o["levels"]
    h = harness.gpu_problem(w, **OPTS, **kw)
    res = dict(shape=h.level_tiles(0), served=h.level_table_regions(0))
    res["lams"] = [h.level_info(l)["lambda"] for l in range(w.nlevels - 1)]
    res["coefs"] = [[h.level_stencil(l, k, 27, harness.stencil_soa(L.coefs[k], 3).shape[1])
                     for k in range(L.lay.nreg)] for l, L in enumerate(levels)]
    res["Abar"] = h.coarse_matrix(levels[-1].Abar.shape[0])
    u = torch.empty(lay.n_regional, dtype=torch.float64, device="cuda:0")
    h.smooth(0, harness.to_dev(lay.flatten(o["br"])), u)
    z = torch.empty(lay.n_composite, dtype=torch.float64, device="cuda:0")
    h.apply_vcycle(harness.to_dev(o["b"]), z)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    res["out"] = h.solve(harness.to_dev(o["b"]), x, rtol=1e-8, maxit=100)
    h.close()
    res.update(u=u.cpu().numpy(), z=z.cpu().numpy(), x=x.cpu().numpy())
    return res


@pytest.fixture(scope="module")
def runs(octant):
    print("[gpu-production-tiles] region table on / off", flush=True)
    return {t: run(octant, region_table=t) for t in (1, 0)}


def test_launch_shape(octant, runs):
    """Level 0 runs 768-thread, 41-plane tiles (two per 82-plane region column) with the table
    serving all 8 regions; without the table nothing is served."""
    on, off = runs[1], runs[0]
    assert on["shape"] == {"ntiles": 8 * 2 * 10, "threads": 768, "planes": 41}, on["shape"]
    assert on["served"] == len(octant["w"].extents)
    assert off["served"] == 0 and off["shape"] == on["shape"]


def test_operators_at_benchmark_shape(octant, runs):
    """Every level's region stencils (device assembly, then Galerkin products) and the coarsest
    composite matrix, entry by entry; the eigenvalue estimates to 1e-12."""
    levels = octant["levels"]
    on = runs[1]
    for l, L in enumerate(levels):
        for k in range(L.lay.nreg):
            harness.assert_close(on["coefs"][l][k], harness.stencil_soa(L.coefs[k], 3), 1e-12,
                                 what=f"level {l} region {k}")
    harness.assert_close(on["Abar"], levels[-1].Abar, 1e-12, what="coarsest composite matrix")
    for l, lam in enumerate(on["lams"]):
        assert abs(lam - levels[l].lam) <= 1e-12 * levels[l].lam, (l, lam, levels[l].lam)


def test_smoother_at_benchmark_shape(octant, runs):
    harness.assert_close(runs[1]["u"], octant["ref_s"], 1e-12, what="smoother, table")


def test_vcycle_at_benchmark_shape(octant, runs):
    """One V-cycle.  At this size the cycle's output moves by about 500 times the rounding of its
    coarse operators: the device's Galerkin products differ from the oracle's by at most 9e-16 of
    their largest entry (test_operators_at_benchmark_shape) and the two cycles by 4e-13 of the
    largest output entry, while the oracle's regional and composite cycles, whose coarse operators
    round alike, agree to 2e-15.  So the cycle is compared with the oracle's cycle run on the
    device's coarse operators and eigenvalue estimates, which isolates the cycle's own arithmetic
    (smoothing, residual, transfers, coarse solve) at 1e-12."""
    from oracle import regional

    lay, levels, opt = octant["lay"], octant["levels"], octant["opt"]
    on = runs[1]
    dev = [copy.copy(L) for L in levels]
    for l in range(1, len(levels)):
        L = dev[l]
        L.coefs = [on["coefs"][l][k].reshape(levels[l].coefs[k].shape) for k in range(L.lay.nreg)]
        L.extra = {}
        if l < len(levels) - 1:
            L.dinv = [1.0 / d for d in regional.composite_diagonal(L.lay, L.coefs)]
    dev[-1].Abar = on["Abar"]
    for l, lam in enumerate(on["lams"]):
        dev[l].lam = lam
    ref = lay.to_composite_owner(regional.vcycle(dev, octant["br"], opt)).reshape(-1)
    print(f"[gpu-production-tiles] V-cycle max|err|/max|ref|: oracle operators "
          f"{harness.max_rel_err(on['z'], octant['ref_v']):.2e}, device operators "
          f"{harness.max_rel_err(on['z'], ref):.2e}", flush=True)
    harness.assert_close(on["z"], ref, 1e-12, what="V-cycle, table")


def test_pcg_at_benchmark_shape(octant, runs):
    lay, ref = octant["lay"], octant["ref_pcg"]
    out = runs[1]["out"]
    assert out["converged"] and ref.converged
    assert out["iterations"] == ref.iterations, (out["iterations"], ref.iterations)
    np.testing.assert_allclose(out["history"], ref.history, rtol=1e-10, atol=0)
    harness.assert_close(runs[1]["x"], lay.to_composite_owner(ref.x).reshape(-1), 1e-10, what="PCG x")
    assert out["true_relres"] <= 1e-8


def test_table_equals_streaming_at_benchmark_shape(runs):
    """Every stencil output is bit for bit that of streaming every coupling; the PCG iterate only
    up to the grouping of the CG product's fused inner product, whose partial sums follow the
    launch decomposition (deep tiles and shell blocks with the table, whole tiles without)."""
    on, off = runs[1], runs[0]
    assert np.array_equal(on["u"], off["u"])
    assert np.array_equal(on["z"], off["z"])
    assert on["out"]["iterations"] == off["out"]["iterations"]
    np.testing.assert_allclose(on["out"]["history"], off["out"]["history"], rtol=1e-12, atol=0)
    harness.assert_close(on["x"], off["x"], 1e-13, what="PCG x, table vs streaming")
