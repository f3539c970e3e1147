"""Parity at the full workload sizes, in the launch configurations the benchmark times.

The oracle cannot assemble these operators (35M to 113M regional rows), so it evaluates sampled
rows of A x one by one from the element definition (`oracle.assembly.q1_rows`): random nodes
plus nodes on interface faces, edges and corners and on the domain boundary.  Checked:
the finest-level regional product Psi [[A]] Psi^T x = A x at those rows (FP64, 1e-12 relative),
and after PCG to 1e-8 the residual b - A x at those rows against the library's own product.
"""
import numpy as np
import pytest

import synth
from tests import harness

pytestmark = pytest.mark.gpu


def sample_nodes(w, n=300, seed=0):
    """Random composite nodes, plus nodes on every kind of interface and on the boundary."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = w.composite_shape_xyz
    nodes = [tuple(int(v) for v in rng.integers(0, [nx, ny, nz])) for _ in range(n)]
    cuts = [sorted({int(o) for o in w.origins[:, d]} - {0}) for d in range(3)]
    for _ in range(40):
        c = [int(rng.choice(cuts[d])) if cuts[d] else int(rng.integers(0, s))
             for d, s in enumerate((nx, ny, nz))]
        r = [int(rng.integers(0, s)) for s in (nx, ny, nz)]
        nodes += [(c[0], r[1], r[2]), (c[0], c[1], r[2]), (c[0], c[1], c[2])]  # face, edge, corner
        nodes += [(0, r[1], r[2]), (r[0], ny - 1, r[2]), (1, r[1], nz - 2)]  # boundary and next to it
    return nodes


def element_coefficients(w):
    if w.pde == "diffusion":
        return synth.jump_coefficients(w)
    if w.pde == "elasticity":  # Young's modulus per element from the region containing it
        youngs = synth.region_youngs_moduli(w)
        nx, ny, nz = w.composite_shape_xyz
        ce = np.zeros((nz - 1, ny - 1, nx - 1))
        for k in range(w.nreg):
            o, e = w.origins[k], w.extents[k]
            ce[o[2]:o[2] + e[2] - 1, o[1]:o[1] + e[1] - 1, o[0]:o[0] + e[0] - 1] = youngs[k]
        return ce
    return None


def composite_matvec(h, w, xc):
    """A x through the library: Psi^T, regional product with interface sum, owner copies."""
    import torch

    reg = torch.empty(h.level_info(0)["n_regional"], dtype=torch.float64, device="cuda:0")
    h.to_regional(0, xc, reg)
    z = torch.empty_like(reg)
    h.regional_matvec(0, reg, z)
    out = torch.empty_like(xc)
    h.to_composite(0, z, out)
    return out


def at(v, w, nodes):
    nx, ny, nz = w.composite_shape_xyz
    a = v.cpu().numpy().reshape((nz, ny, nx) + ((3,) if w.ndof == 3 else ()))
    return np.array([a[gz, gy, gx] for gx, gy, gz in nodes])


CASES = [
    ("c2", {}),
    ("c5", {}),
    ("c3", {"precision": 2}),
    ("c4", {"precision": 1, "autotune": 1, "use_graph": 1}),
]


@pytest.mark.parametrize("name,opts", CASES, ids=[c[0] for c in CASES])
def test_fullsize_matvec_and_solve(hip_device, tmp_path, name, opts):
    import torch

    from oracle import assembly

    w = synth.workload(name)
    print(f"[fullsize] {name} {opts}", flush=True)
    if opts.get("autotune"):
        opts = dict(opts, autotune_cache=str(tmp_path / "tune.txt"))
    h = harness.gpu_problem(w, **opts)
    nx, ny, nz = w.composite_shape_xyz
    dn = synth.dirichlet_nodes((nx, ny, nz), w.dirichlet_mask)
    ce = element_coefficients(w)
    nodes = sample_nodes(w)
    rng = np.random.default_rng(1)
    shp = (nz, ny, nx) + ((3,) if w.ndof == 3 else ())
    x = rng.uniform(-1, 1, size=shp)
    z = composite_matvec(h, w, harness.to_dev(x))
    ref = assembly.q1_rows((nx, ny, nz), dn, x, nodes, w.pde, h=w.h, elem_coef=ce, nu=w.nu)
    got = at(z, w, nodes)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # PCG to 1e-8; the residual at the sampled rows from the oracle's rows and the library's product
    b = synth.rhs(w)
    bd = harness.to_dev(b)
    xs = torch.zeros_like(bd)
    out = h.solve(bd, xs, rtol=1e-8, maxit=200)
    assert out["converged"] and out["true_relres"] <= 1e-8, out
    res_lib = at(bd - composite_matvec(h, w, xs), w, nodes)
    xsol = xs.cpu().numpy().reshape(shp)
    res_or = np.array([b[gz, gy, gx] for gx, gy, gz in nodes]) - assembly.q1_rows(
        (nx, ny, nz), dn, xsol, nodes, w.pde, h=w.h, elem_coef=ce, nu=w.nu)
    assert np.abs(res_lib - res_or).max() <= 1e-11 * np.abs(b).max()
    h.close()


def test_fullsize_learned_interpolation(hip_device):
    """Learned weights at full size (35M fine nodes, 1.26M cells) are valid, and the judged
    hierarchy solves to 1e-8."""
    import torch

    from paper_2103_11962_amd import regmg

    w = synth.workload("c5")
    h = harness.gpu_problem(w, setup=False)
    h.set_learned_prolongator(synth.mlp_params(seed=3))
    h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree, judge_cycles=3)
    info = h.prolongator_info()
    assert info["flags"] in (0, regmg.PW_JUDGED_WORSE), info
    assert info["rho_learned"] > 0 and info["rho_geometric"] > 0
    b = harness.to_dev(synth.rhs(w))
    x = torch.zeros_like(b)
    out = h.solve(b, x, rtol=1e-8, maxit=200)
    assert out["converged"] and out["true_relres"] <= 1e-8
    h.close()


def test_fullsize_gauss_seidel_pcg(hip_device):
    """Region-local symmetric Gauss-Seidel (64 regions of 82^3, 567 hyperplanes per sweep) as the
    smoother of the PCG preconditioner at full size: converges, and the residual at the sampled
    rows from the oracle's rows agrees with the library's own product."""
    import torch

    from oracle import assembly

    w = synth.workload("c2")
    print("[fullsize] c2 symmetric Gauss-Seidel", flush=True)
    h = harness.gpu_problem(w, smoother=4, jacobi_omega=1.0)
    b = synth.rhs(w)
    bd = harness.to_dev(b)
    xs = torch.zeros_like(bd)
    out = h.solve(bd, xs, rtol=1e-8, maxit=100)
    assert out["converged"] and out["true_relres"] <= 1e-8, out
    nx, ny, nz = w.composite_shape_xyz
    nodes = sample_nodes(w)
    dn = synth.dirichlet_nodes((nx, ny, nz), w.dirichlet_mask)
    res_lib = at(bd - composite_matvec(h, w, xs), w, nodes)
    xsol = xs.cpu().numpy().reshape((nz, ny, nx))
    res_or = np.array([b[gz, gy, gx] for gx, gy, gz in nodes]) - assembly.q1_rows(
        (nx, ny, nz), dn, xsol, nodes, w.pde, h=w.h)
    assert np.abs(res_lib - res_or).max() <= 1e-11 * np.abs(b).max()
    print(f"[fullsize] symmetric GS PCG: {out['iterations']} iterations, {out['solve_ms']:.1f} ms", flush=True)
    h.close()



def test_fullsize_table_equals_streaming(hip_device):
    """At the benchmark's own size and launch shape (4x4x4 regions of 82^3: 1,280 tiles of 768
    threads marching 41 planes), one V-cycle with the region table equals the V-cycle that streams
    every coupling bit for bit; the same shape on 2x2x2 of these regions is compared with the
    oracle element by element in test_gpu_production_tiles."""
    import torch

    w = synth.workload("c2")
    print("[fullsize] c2 region table on / off", flush=True)
    b = harness.to_dev(synth.rhs(w))
    zs = {}
    for t in (1, 0):
        h = harness.gpu_problem(w, region_table=t)
        shape = h.level_tiles(0)
        assert shape == {"ntiles": 1280, "threads": 768, "planes": 41}, shape
        assert h.level_table_regions(0) == (64 if t else 0)
        z = torch.empty_like(b)
        h.apply_vcycle(b, z)
        zs[t] = z
        h.close()
    assert torch.equal(zs[1], zs[0])
