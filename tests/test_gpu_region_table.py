"""Region class tables of the symmetric FP64 levels: where every node of a region has, bit for bit,
the 27 couplings (3 x 3 blocks for elasticity) of its class (per axis the two low layers, the
inside, the two high layers), the region takes its couplings from its 125-class table: whole-row
class-table tiles on tiled levels, each node's class row on node-block levels.  Each case solves
twice, with the tables (default) and with every coupling streamed (region_table = 0): the V-cycle
output must agree bit for bit, the PCG iterate and residual history to the rounding of the CG
inner product.  The regions served follow the coefficients: every region with at least 5 nodes a
side of a constant-coefficient Laplacian or per-region elasticity, none under per-element random
coefficients or on regions too thin; the FP32 V-cycle builds no table.
"""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu

# (workload, setup options, regions expected on the table at level 0: "thick" = every region with
# at least 5 nodes a side)
CASES = [
    ("c2_small", dict(stencil_kernel=2), "thick"),
    ("c2_mid", dict(stencil_kernel=2), "thick"),
    ("c2_mid", dict(stencil_kernel=3), "thick"),
    ("c2_mid", dict(stencil_kernel=2, precision=1), 0),
    ("uneven3d_small", dict(stencil_kernel=2), "thick"),
    ("uneven_c4_small", dict(stencil_kernel=2), "thick"),
    ("c4_small", dict(stencil_kernel=2), "thick"),
    ("c5_small", dict(stencil_kernel=2), 0),
    ("c3_small", dict(), "thick"),  # elasticity: node blocks read 3 x 3 blocks from the class tables
    ("uneven_tiny3d", dict(stencil_kernel=2), 0),
]
IDS = [f"{n}-" + "-".join(f"{k}{v}" for k, v in kw.items()) for n, kw, _ in CASES]


def run(w, b, **kw):
    import torch

    h = harness.gpu_problem(w, **kw)
    z = torch.empty_like(b)
    h.apply_vcycle(b, z)
    x = torch.zeros_like(b)
    out = h.solve(b, x, rtol=1e-8)
    served = h.level_table_regions(0)
    served1 = h.level_table_regions(1) if w.nlevels > 2 else 0  # node-block level below
    h.close()
    return z, x, out, served, served1


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_table_equals_streamed_couplings(hip_device, case):
    import torch

    name, kw, expect = case
    w = synth.workload(name)
    b = harness.to_dev(synth.rhs(w))
    print(f"[gpu-table] {name} {kw}", flush=True)
    z1, x1, o1, n1, m1 = run(w, b, **kw)
    z0, x0, o0, n0, m0 = run(w, b, region_table=0, **kw)
    thick = int(sum(min(int(v) for v in e) >= 5 for e in np.asarray(w.extents)))
    want = thick if expect == "thick" else expect
    assert n0 == 0 and n1 == want
    # the Galerkin level below a constant-coefficient layout of 28^3 regions (10^3 there) is served
    # too; none without tables or in the FP32 V-cycle
    assert m0 == 0
    if kw.get("precision", 0) != 0:
        assert m1 == 0
    elif name == "c2_mid":
        assert m1 == len(w.extents)
    assert torch.equal(z1, z0)  # every stencil operation of the cycle, bit for bit
    # CG: the product's fused inner-product partial sums follow the launch decomposition (deep
    # tiles and shell blocks with the table, whole tiles without), so only their rounding differs
    assert o1["iterations"] == o0["iterations"] and o1["converged"]
    np.testing.assert_allclose(o1["history"], o0["history"], rtol=1e-12, atol=0)
    harness.assert_close(x1.cpu().numpy(), x0.cpu().numpy(), 1e-13, what="PCG x, table vs streaming")


def test_table_option_error(hip_device):
    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    h = harness.gpu_problem(w, setup=False)
    with pytest.raises(regmg.RmgError) as e:
        h.setup_hierarchy(nlevels=2, cheb_degree=2, region_table=2)
    assert e.value.status == "RMG_ERR_ARG"
    h.close()
