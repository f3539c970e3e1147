"""Shared set-up of one workload on the GPU library and in the oracle.

Used by the tests, the smoke check and the benchmark.  The GPU side receives
only seeded inputs from ``synth`` (layout, right-hand side, coefficient
fields, the assembled composite five-point stencil); every step of the
method runs in the HIP library.
"""
from __future__ import annotations

import numpy as np

import synth


def gpu_problem(w, device=0, setup=True, torch_allocator=False, **opts):
    """Handle with regions, finest operator and (optionally) the hierarchy of workload ``w``."""
    import torch

    from paper_2103_11962_amd import regmg

    h = regmg.Handle(device, torch_allocator=torch_allocator)
    h.build_regions(w.dim, w.ndof, w.extents, w.origins, w.dirichlet_mask)
    if w.pde == "fd5":
        h.set_composite_stencil(5, synth.fd5_composite_stencil(w))
    elif w.pde == "fd7":
        h.set_composite_stencil(27, synth.fd7_composite_stencil(w))
    elif w.pde == "laplace":
        h.assemble_q1(regmg.PDE_LAPLACE, w.h)
    elif w.pde == "elasticity":
        h.assemble_q1(regmg.PDE_ELASTICITY, w.h, youngs=synth.region_youngs_moduli(w), nu=w.nu)
    elif w.pde == "diffusion":
        ec = torch.from_numpy(np.ascontiguousarray(synth.jump_coefficients(w))).to(f"cuda:{device}")
        h.assemble_q1(regmg.PDE_DIFFUSION, w.h, elem_coef=ec.reshape(-1))
        h._keep = ec
    else:
        raise NotImplementedError(w.pde)
    if setup:
        o = dict(nlevels=w.nlevels, cheb_degree=w.cheb_degree)
        o.update(opts)
        h.setup_hierarchy(**o)
    return h


def oracle_problem(w, **opts):
    """(layout, levels, options) of the oracle's regional hierarchy for workload ``w``."""
    from oracle import regional
    from oracle.regions import Layout

    lay = Layout(w.dim, w.origins, w.extents, w.dirichlet_mask, w.ndof)
    youngs = synth.region_youngs_moduli(w) if w.pde == "elasticity" else None
    ec = synth.jump_coefficients(w) if w.pde == "diffusion" else None
    coefs = regional.build_operator(lay, w.pde, h=w.h, elem_coef=ec, youngs=youngs, nu=w.nu)
    kw = dict(nlevels=w.nlevels, degree=w.cheb_degree)
    kw.update(opts)
    opt = regional.Options(**kw)
    levels = regional.setup(lay, coefs, opt)
    return lay, levels, opt


def to_dev(a, device=0):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to(f"cuda:{device}")


def stencil_soa(coef, dim, ndof=1):
    """Oracle region stencil (S, nodes...[, ndof, ndof]) in the library's layout [S*ndof*ndof][nodes]."""
    S = coef.shape[0]
    if ndof == 1:
        return coef.reshape(S, -1)
    c = coef.reshape(S, -1, ndof, ndof)  # (S, nodes, a, b)
    return np.transpose(c, (0, 2, 3, 1)).reshape(S * ndof * ndof, -1)


def vshape(lay):
    """numpy shape of a composite vector of the layout."""
    return lay.shape + ((lay.ndof,) if lay.ndof > 1 else ())


def assert_close(got, ref, tol, floor=0.1, what=""):
    """Element-wise parity: |got_i - ref_i| <= tol * (|ref_i| + floor * max_j |ref_j|) for every i.

    ``tol`` is the relative tolerance of the comparison.  The absolute part admits the rounding of
    entries that are small only through cancellation: every entry of a stencil product, a transfer,
    a smoother or a cycle is a sum of terms as large as the largest entries, so both sides round it
    at that scale, not at its own.  With the default floor 0.1 and the FP64 tolerances used here
    (1e-12, 1e-13) that is 1e-13 (1e-14) of the largest entry, about 450 (45) units in the last
    place of it: the rounding of the few hundred operations such a chain performs (the largest
    deviation seen on MI355X is 4e-14 of the largest entry).  A single entry off by more than that —
    an interface corner, a tile edge — fails, however long the vector; a norm-wise test would let
    one entry deviate by sqrt(n) times as much.
    """
    g = np.asarray(got, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    assert g.shape == r.shape, (what, g.shape, r.shape)
    assert np.all(np.isfinite(g)), (what, "non-finite entries")
    scale = float(np.max(np.abs(r))) if r.size else 0.0
    bound = tol * (np.abs(r) + floor * scale)
    err = np.abs(g - r)
    bad = err > bound
    if np.any(bad):
        i = int(np.argmax(err - bound))
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {g.size} entries outside tol {tol:g} (floor {floor:g}); "
            f"worst index {i}: got {g[i]!r}, ref {r[i]!r}, |err| {err[i]:.3e}, bound {bound[i]:.3e}, "
            f"max|ref| {scale:.3e}, max|err|/max|ref| {float(err.max()) / max(scale, 1e-300):.3e}")


def max_rel_err(got, ref):
    """max_i |got_i - ref_i| / max_i |ref_i| (reported beside element-wise checks)."""
    g = np.asarray(got, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.max(np.abs(g - r)) / max(float(np.max(np.abs(r))), 1e-300)) if r.size else 0.0
