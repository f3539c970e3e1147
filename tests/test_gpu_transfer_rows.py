"""Geometric transfers by rows and planes (rmg_options.transfer_rows = 1, the default) against one
thread per node (transfer_rows = 0), Section 3.3: on every level pair of 2D and 3D, scalar and
elasticity, even and uneven layouts (shortened last coarse intervals), the restriction of a random
regional vector and the prolongation of a random coarse vector (nonzero on Dirichlet coarse nodes,
which a free fine node must not take) agree bit for bit, and so does one V-cycle in FP64 and FP32.
The node-parallel kernels are checked against the oracle by test_gpu_parity."""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu

CASES = [
    ("c2_small", {}),
    ("c2_mid", {}),
    ("uneven3d_small", {}),
    ("uneven3e_small", {}),
    ("uneven_tiny3d", {}),
    ("c1_small", {}),
    ("uneven2d_small", {}),
    ("c3_small", {}),
    ("c2_mid", dict(precision=1)),
    ("c3_small", dict(precision=1)),
]
IDS = [n + "".join(f"-{k}{v}" for k, v in kw.items()) for n, kw in CASES]


def bits(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name,opts", CASES, ids=IDS)
def test_rows_equal_nodes(hip_device, name, opts):
    import torch

    w = synth.workload(name)
    hr = harness.gpu_problem(w, transfer_rows=1, **opts)
    hn = harness.gpu_problem(w, transfer_rows=0, **opts)
    rng = np.random.default_rng(11)
    try:
        nlev = w.nlevels
        for l in range(nlev - 1):
            tr, tn = hr.level_transfer_tiles(l), hn.level_transfer_tiles(l)
            assert tr["restriction"] > 0 and tr["prolongation"] > 0, (l, tr)
            assert tn == {"restriction": 0, "prolongation": 0}
            nf = hr.level_info(l)["n_regional"]
            nc = hr.level_info(l + 1)["n_regional"]
            r = torch.from_numpy(rng.uniform(-1, 1, nf)).to("cuda:0")
            wr = torch.full((nc,), np.nan, dtype=torch.float64, device="cuda:0")
            wn = torch.full((nc,), np.nan, dtype=torch.float64, device="cuda:0")
            hr.restrict(l, r, wr)
            hn.restrict(l, r, wn)
            assert np.array_equal(bits(wr), bits(wn)), f"restriction level {l}"
            ub = torch.from_numpy(rng.uniform(-1, 1, nc)).to("cuda:0")
            u0 = rng.uniform(-1, 1, nf)
            ur = torch.from_numpy(u0.copy()).to("cuda:0")
            un = torch.from_numpy(u0.copy()).to("cuda:0")
            hr.prolongate_add(l, ub, ur)
            hn.prolongate_add(l, ub, un)
            assert np.array_equal(bits(ur), bits(un)), f"prolongation level {l}"
        assert hr.level_transfer_tiles(nlev - 1) == {"restriction": 0, "prolongation": 0}
        b = harness.to_dev(synth.rhs(w))
        zr, zn = torch.empty_like(b), torch.empty_like(b)
        hr.apply_vcycle(b, zr)
        hn.apply_vcycle(b, zn)
        assert np.array_equal(bits(zr), bits(zn)), "V-cycle"
    finally:
        hr.close()
        hn.close()


def test_option_checked(hip_device):
    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    h = harness.gpu_problem(w, setup=False)
    try:
        with pytest.raises(regmg.RmgError):
            h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, transfer_rows=2)
    finally:
        h.close()
