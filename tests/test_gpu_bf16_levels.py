"""BF16 chosen per level by measured convergence factor (precision RMG_PREC_FP32_BF16_AUTO).

Setup measures the factor of bf16_cycles stationary V-cycles with every level's V-cycle copy in
FP32, then, finest level first, switches one level at a time to BF16 off-diagonals (FP32 centre
blocks, row sums kept) and keeps it where the factor stays within (1 + bf16_tolerance) of the
FP32 one.  Checked: the reported factors and choices obey that rule on every level, the FP32
reference equals what rmg_convergence_factor measures on an all-FP32 hierarchy bit for bit, the
flexible FP64 CG still reaches a true residual of 1e-8 at the FP64 oracle's solution (element-wise,
the mixed-precision bound of test_gpu_parity), an unbounded tolerance puts every smoothed level in
BF16, and the option's bounds are enforced.
"""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu

CASES = ["c2_mid", "c3_small"]


@pytest.mark.parametrize("name", CASES)
def test_bf16_levels_follow_measured_factor(hip_device, name):
    import torch

    from oracle import regional
    from paper_2103_11962_amd import regmg

    w = synth.workload(name)
    tol, cycles = 0.05, 10
    h = harness.gpu_problem(w, precision=regmg.PREC_FP32_BF16_AUTO, bf16_tolerance=tol, bf16_cycles=cycles)
    infos = [h.level_precision(l) for l in range(w.nlevels)]
    print(f"[gpu-bf16] {name}: {infos}", flush=True)
    ref32 = infos[0]["rho_fp32"]
    assert 0.0 < ref32 < 1.0
    for l, inf in enumerate(infos[:-1]):
        assert inf["rho_fp32"] == ref32 and inf["rho_bf16"] > 0.0, (l, inf)
        assert inf["coef_type"] == (2 if inf["rho_bf16"] <= ref32 * (1.0 + tol) else 1), (l, inf)
    assert infos[-1] == {"coef_type": 0, "rho_fp32": -1.0, "rho_bf16": -1.0}
    # the reference is the all-FP32 hierarchy's factor
    h32 = harness.gpu_problem(w, precision=regmg.PREC_FP32)
    assert h32.convergence_factor(cycles) == ref32
    assert all(h32.level_precision(l)["coef_type"] == 1 for l in range(w.nlevels - 1))
    h32.close()
    # the solve with the chosen levels
    lay, levels, opt = harness.oracle_problem(w)
    b = synth.rhs(w)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8, maxit=100)
    h.close()
    ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-12, maxit=200)
    assert out["converged"] and out["true_relres"] <= 1e-8, out
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(ref.x).reshape(-1), 1e-6, floor=1.0)


def test_bf16_unbounded_tolerance_takes_every_level(hip_device):
    import torch

    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_mid")
    h = harness.gpu_problem(w, precision=regmg.PREC_FP32_BF16_AUTO, bf16_tolerance=1e9, bf16_cycles=3)
    assert [h.level_precision(l)["coef_type"] for l in range(w.nlevels)] == [2] * (w.nlevels - 1) + [0]
    b = harness.to_dev(synth.rhs(w))
    x = torch.zeros_like(b)
    out = h.solve(b, x, rtol=1e-8, maxit=100)
    h.close()
    assert out["converged"] and out["true_relres"] <= 1e-8, out


def test_fixed_precisions_report_their_storage(hip_device):
    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    for prec, want0, want1 in ((regmg.PREC_FP64, 0, 0), (regmg.PREC_FP32, 1, 1), (regmg.PREC_FP32_BF16, 2, 1)):
        h = harness.gpu_problem(w, precision=prec)
        got = [h.level_precision(l) for l in range(w.nlevels)]
        h.close()
        assert [g["coef_type"] for g in got[:2]] == [want0, want1], (prec, got)
        assert all(g["rho_fp32"] == -1.0 and g["rho_bf16"] == -1.0 for g in got)


@pytest.mark.parametrize("kw", [dict(bf16_tolerance=-0.1), dict(bf16_tolerance=float("nan")), dict(bf16_cycles=0)])
def test_bf16_option_bounds(hip_device, kw):
    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    h = harness.gpu_problem(w, setup=False)
    with pytest.raises(regmg.RmgError) as e:
        h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, precision=regmg.PREC_FP32_BF16_AUTO, **kw)
    assert e.value.status == "RMG_ERR_ARG"
    h.close()
