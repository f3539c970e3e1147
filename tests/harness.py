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
