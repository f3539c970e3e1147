"""Seeded workload generators: region layouts, right-hand sides and coefficient fields.

Conventions shared by every consumer:

* Coordinates are (x, y[, z]); composite arrays are C-ordered with x fastest,
  i.e. numpy shape (nz, ny, nx) in 3D and (ny, nx) in 2D.
* A region is an axis-aligned box of grid nodes, ``origin`` .. ``origin+extent-1``
  per axis, in composite node coordinates.  Neighbouring boxes share their
  interface nodes (the region decomposition of the paper's Section 3.1).
* ``dirichlet_mask`` bit 2*d is the low face along axis d, bit 2*d+1 the high face.
* Random numbers come from numpy's PCG64 seeded with the workload seed.

Nothing here computes any part of the multigrid method.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "tensor_layout",
    "workload",
    "WORKLOADS",
    "rhs",
    "uniform_composite",
    "region_youngs_moduli",
    "jump_coefficients",
    "mlp_params",
    "batched_extents",
    "even_slabs",
    "dirichlet_nodes",
    "fd5_composite_stencil",
    "fd7_composite_stencil",
]


@dataclass
class Workload:
    """A region layout plus the solver options a configuration is quoted with."""

    name: str
    dim: int
    ndof: int
    origins: np.ndarray  # (nreg, dim) int64, (x, y[, z])
    extents: np.ndarray  # (nreg, dim) int64
    dirichlet_mask: int
    nlevels: int
    cheb_degree: int
    pde: str  # "fd5" (2D five-point), "fd7" (3D seven-point), "laplace", "diffusion", "elasticity"
    h: float = 1.0
    nu: float = 0.3
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def nreg(self) -> int:
        return int(self.origins.shape[0])

    @property
    def composite_shape_xyz(self) -> tuple:
        return tuple(int(v) for v in (self.origins + self.extents).max(axis=0))

    @property
    def composite_shape(self) -> tuple:
        """numpy shape of a composite node array (x fastest)."""
        return tuple(reversed(self.composite_shape_xyz))

    @property
    def n_composite_nodes(self) -> int:
        return int(np.prod(self.composite_shape_xyz))

    @property
    def n_regional_nodes(self) -> int:
        return int(np.prod(self.extents, axis=1).sum())


def tensor_layout(slab_extents):
    """Regions of a tensor-product layout.

    ``slab_extents[d]`` lists the node extents of the slabs along axis d.
    Neighbouring slabs share one node plane.  Regions are numbered with the
    x slab index fastest.  Returns (origins, extents) as (nreg, dim) arrays.
    """
    dim = len(slab_extents)
    starts = []
    for ext in slab_extents:
        s = [0]
        for e in ext[:-1]:
            s.append(s[-1] + int(e) - 1)
        starts.append(s)
    counts = [len(e) for e in slab_extents]
    origins, extents = [], []
    for idx in np.ndindex(*reversed(counts)):
        idx = tuple(reversed(idx))  # (ix, iy[, iz]) with ix fastest
        origins.append([starts[d][idx[d]] for d in range(dim)])
        extents.append([int(slab_extents[d][idx[d]]) for d in range(dim)])
    return np.asarray(origins, dtype=np.int64), np.asarray(extents, dtype=np.int64)


def _uniform_layout(dim, nper, ext):
    return tensor_layout([[ext] * nper] * dim)


def batched_extents(seed: int = 0, counts=(8, 8, 4), choices=(28, 55, 82, 109)):
    """Slab extents per axis drawn i.i.d. from ``choices`` (batched uneven-region mesh)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [list(rng.choice(np.asarray(choices), size=c)) for c in counts]


def even_slabs(n: int, parts: int):
    """Extents of ``parts`` slabs sharing end nodes that cover n nodes as evenly as possible
    (the first slabs take the extra cells)."""
    cells = n - 1
    base = cells // parts
    ext = [base + 1] * parts
    for i in range(cells - base * parts):
        ext[i] += 1
    return ext


def workload(name: str, seed: int = 0) -> Workload:
    """Named configurations.

    ``c1``  2D five-point Poisson, 2x2 regions of 82^2 nodes, 3 levels, Chebyshev degree 2.
    ``c2``  3D Q1 Laplacian, 4x4x4 regions of 82^3, 4 levels, degree 3.
    ``c2_octant``  2x2x2 of c2's regions (82^3 each, composite 163^3) with c2's mesh width and levels.
    ``c3``  3D Q1 elasticity, 3x3x3 regions of 55^3, E per region lognormal, nu = 0.3.
    ``c4``  3D Q1 Laplacian on 8x8x4 regions with slab extents from {28,55,82,109}.
    ``c5``  3D Q1 diffusion with jump coefficients, 4x4x4 regions of 82^3.
    Small variants (``*_small``) keep the structure at sizes a pure NumPy code
    finishes in seconds.
    ``table1_rect``  2D five-point, 700 x 720 nodes in 3x3 regions (extents 234 and 241/240, not
    3^k + 1), 4 levels, one smoothing step.
    ``uneven*``  region extents that are not 3^k + 1 (2D five-point, 3D Q1 Laplace, elasticity,
    an 8-region mesh with slab extents drawn from 11..31, and 2D/3D meshes of extents 2 to 5).
    """
    full = lambda dim: (1 << (2 * dim)) - 1  # noqa: E731  all faces Dirichlet
    if name == "c1":
        o, e = _uniform_layout(2, 2, 82)
        return Workload(name, 2, 1, o, e, full(2), 3, 2, "fd5", seed=seed)
    if name == "c1_small":
        o, e = _uniform_layout(2, 2, 10)
        return Workload(name, 2, 1, o, e, full(2), 3, 2, "fd5", seed=seed)
    if name == "c2":
        o, e = _uniform_layout(3, 4, 82)
        return Workload(name, 3, 1, o, e, full(3), 4, 3, "laplace", h=1.0 / 324, seed=seed)
    if name == "c2_octant":  # 2x2x2 of c2's 64 regions (composite 163^3), c2's mesh width and levels
        o, e = _uniform_layout(3, 2, 82)
        return Workload(name, 3, 1, o, e, full(3), 4, 3, "laplace", h=1.0 / 324, seed=seed)
    if name == "c2_small":
        o, e = _uniform_layout(3, 2, 10)
        return Workload(name, 3, 1, o, e, full(3), 3, 3, "laplace", h=1.0 / 18, seed=seed)
    if name == "c2_mid":
        o, e = _uniform_layout(3, 2, 28)
        return Workload(name, 3, 1, o, e, full(3), 3, 3, "laplace", h=1.0 / 54, seed=seed)
    if name == "c3":
        o, e = _uniform_layout(3, 3, 55)
        return Workload(name, 3, 3, o, e, full(3), 4, 3, "elasticity", h=1.0 / 162, seed=seed)
    if name == "c3_small":
        o, e = _uniform_layout(3, 2, 10)
        return Workload(name, 3, 3, o, e, full(3), 3, 3, "elasticity", h=1.0 / 18, seed=seed)
    if name == "c4":
        o, e = tensor_layout(batched_extents(seed))
        return Workload(name, 3, 1, o, e, full(3), 4, 3, "laplace", seed=seed)
    if name == "c4_small":
        o, e = tensor_layout(batched_extents(seed, counts=(3, 2, 2), choices=(10, 19, 28)))
        return Workload(name, 3, 1, o, e, full(3), 3, 3, "laplace", seed=seed)
    if name == "c5":
        o, e = _uniform_layout(3, 4, 82)
        return Workload(name, 3, 1, o, e, full(3), 4, 3, "diffusion", h=1.0 / 324, seed=seed)
    if name == "c5_small":
        o, e = _uniform_layout(3, 2, 28)
        return Workload(name, 3, 1, o, e, full(3), 3, 3, "diffusion", h=1.0 / 54, seed=seed)
    if name == "table1_rect":
        o, e = tensor_layout([even_slabs(700, 3), even_slabs(720, 3)])
        return Workload(name, 2, 1, o, e, full(2), 4, 1, "fd5", seed=seed)
    if name == "uneven2d_small":
        o, e = tensor_layout([[12, 17, 10], [16, 11]])
        return Workload(name, 2, 1, o, e, full(2), 3, 2, "fd5", seed=seed)
    if name == "uneven3d_small":
        o, e = tensor_layout([[12, 8], [11, 7], [9, 13]])
        return Workload(name, 3, 1, o, e, full(3), 3, 3, "laplace", h=1.0 / 18, seed=seed)
    if name == "uneven3e_small":
        o, e = tensor_layout([[8, 6], [7, 6], [6, 8]])
        return Workload(name, 3, 3, o, e, full(3), 3, 3, "elasticity", h=1.0 / 12, seed=seed)
    if name == "uneven_tiny3d":  # extents 2 to 5: single-cell and two-cell coarse intervals, levels
        o, e = tensor_layout([[2, 5, 3], [3, 4], [4, 2]])  # that stop shrinking at 2 nodes per axis
        return Workload(name, 3, 1, o, e, full(3), 3, 2, "laplace", h=0.25, seed=seed)
    if name == "uneven_tiny2d":
        o, e = tensor_layout([[2, 3, 4], [5, 2]])
        return Workload(name, 2, 1, o, e, full(2), 4, 2, "fd5", seed=seed)
    if name == "uneven_c4_small":
        o, e = tensor_layout(batched_extents(seed, counts=(2, 2, 2), choices=tuple(range(11, 32))))
        return Workload(name, 3, 1, o, e, full(3), 4, 3, "laplace", seed=seed)
    raise KeyError(name)


WORKLOADS = ("c1", "c1_small", "c2", "c2_octant", "c2_small", "c2_mid", "c3", "c3_small",
             "c4", "c4_small", "c5", "c5_small", "table1_rect", "uneven2d_small", "uneven3d_small",
             "uneven3e_small", "uneven_c4_small", "uneven_tiny3d", "uneven_tiny2d")


def dirichlet_nodes(shape_xyz, mask: int) -> np.ndarray:
    """Boolean composite array (x fastest) of nodes on the masked domain faces."""
    dim = len(shape_xyz)
    out = np.zeros(tuple(reversed(shape_xyz)), dtype=bool)
    for d in range(dim):
        ax = dim - 1 - d  # numpy axis of coordinate d
        n = shape_xyz[d]
        if mask & (1 << (2 * d)):
            sl = [slice(None)] * dim
            sl[ax] = 0
            out[tuple(sl)] = True
        if mask & (1 << (2 * d + 1)):
            sl = [slice(None)] * dim
            sl[ax] = n - 1
            out[tuple(sl)] = True
    return out


def uniform_composite(shape_xyz, ndof: int, seed: int, stream: int = 0) -> np.ndarray:
    """i.i.d. U[-1, 1] values on composite nodes, shape (..nodes.., ndof) if ndof > 1."""
    rng = np.random.Generator(np.random.PCG64([seed, stream]))
    shape = tuple(reversed(shape_xyz)) + ((ndof,) if ndof > 1 else ())
    return rng.uniform(-1.0, 1.0, size=shape)


def rhs(w: Workload, seed: int | None = None) -> np.ndarray:
    """Right-hand side: U[-1, 1] per free dof, zero on Dirichlet nodes (composite layout)."""
    seed = w.seed if seed is None else seed
    b = uniform_composite(w.composite_shape_xyz, w.ndof, seed, stream=1)
    dn = dirichlet_nodes(w.composite_shape_xyz, w.dirichlet_mask)
    b[dn] = 0.0
    return b


def region_youngs_moduli(w: Workload, seed: int | None = None) -> np.ndarray:
    """Young's modulus per region, E = exp(N(0, 1))."""
    seed = w.seed if seed is None else seed
    rng = np.random.Generator(np.random.PCG64([seed, 2]))
    return np.exp(rng.standard_normal(w.nreg))


def jump_coefficients(w: Workload, seed: int | None = None) -> np.ndarray:
    """Per-element diffusion coefficient on the composite element grid (x fastest).

    c_e = 10**s_R * exp(xi_e) with xi_e ~ N(0, 1) per element; s_R ~ U(-4, 4)
    for regions whose tensor index (I+J+K) is even and s_R = 0 otherwise.
    The region of an element is the box that contains it.
    """
    seed = w.seed if seed is None else seed
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    shape_e = tuple(n - 1 for n in reversed(w.composite_shape_xyz))
    xi = rng.standard_normal(shape_e)
    s = rng.uniform(-4.0, 4.0, size=w.nreg)
    # tensor index of each region from its origin rank per axis
    tidx = np.zeros((w.nreg, w.dim), dtype=np.int64)
    for d in range(w.dim):
        uniq = np.unique(w.origins[:, d])
        tidx[:, d] = np.searchsorted(uniq, w.origins[:, d])
    parity_even = (tidx.sum(axis=1) % 2) == 0
    s = np.where(parity_even, s, 0.0)
    c = np.exp(xi)
    for k in range(w.nreg):
        sl = tuple(slice(int(o), int(o + e - 1)) for o, e in zip(reversed(w.origins[k]), reversed(w.extents[k])))
        c[sl] *= 10.0 ** s[k]
    return c


def mlp_params(seed: int = 0, out_scale: float = 0.1) -> np.ndarray:
    """Initial parameters (float32) of a 27 -> 64 -> 64 -> 208 perceptron, flat in the order
    W1 (64x27), b1, W2 (64x64), b2, W3 (208x64), b3: weights U(-a, a) with a = sqrt(6 / fan_in)
    (He-uniform; W3 scaled down by ``out_scale``), biases zero."""
    rng = np.random.Generator(np.random.PCG64([seed, 4]))
    parts = []
    for rows, cols, scale in ((64, 27, 1.0), (64, 64, 1.0), (208, 64, out_scale)):
        a = scale * np.sqrt(6.0 / cols)
        parts.append(rng.uniform(-a, a, size=rows * cols))
        parts.append(np.zeros(rows))
    return np.concatenate(parts).astype(np.float32)


def fd5_composite_stencil(w: Workload) -> np.ndarray:
    """The 2D five-point problem as an assembled composite stencil, shape (5, ny*nx).

    Stencil order (0,-1), (-1,0), (0,0), (1,0), (0,1); values [-1, -1, 4, -1, -1]
    with homogeneous Dirichlet nodes kept as identity rows and every coupling to
    or from them removed.  Couplings leaving the domain are zero.  This is the
    problem statement A u = b handed to the solver, not part of the solver.
    """
    assert w.dim == 2
    nx, ny = w.composite_shape_xyz
    dn = dirichlet_nodes((nx, ny), w.dirichlet_mask)
    offs = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
    vals = [-1.0, -1.0, 4.0, -1.0, -1.0]
    out = np.zeros((5, ny, nx))
    yy, xx = np.indices((ny, nx))
    for s, ((dx, dy), v) in enumerate(zip(offs, vals)):
        jx, jy = xx + dx, yy + dy
        inside = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny)
        nb_dir = np.zeros_like(inside)
        nb_dir[inside] = dn[jy[inside], jx[inside]]
        c = np.where(inside, v, 0.0)
        if (dx, dy) != (0, 0):
            c = np.where(dn | nb_dir, 0.0, c)
        else:
            c = np.where(dn, 1.0, c)
        out[s] = c
    return out.reshape(5, -1)


def fd7_composite_stencil(w: Workload) -> np.ndarray:
    """The 3D seven-point problem as an assembled composite stencil in the 27-point order
    (dx fastest, then dy, dz), shape (27, nz*ny*nx): 6 on the diagonal, -1 to the six face
    neighbours, every other offset zero; homogeneous Dirichlet nodes are identity rows with every
    coupling to or from them removed.  This is the problem statement handed to the solver."""
    assert w.dim == 3
    nx, ny, nz = w.composite_shape_xyz
    dn = dirichlet_nodes((nx, ny, nz), w.dirichlet_mask)
    out = np.zeros((27, nz, ny, nx))
    zz, yy, xx = np.indices((nz, ny, nx))
    for s in range(27):
        dx, dy, dz = s % 3 - 1, (s // 3) % 3 - 1, s // 9 - 1
        if abs(dx) + abs(dy) + abs(dz) > 1:
            continue
        if (dx, dy, dz) == (0, 0, 0):
            out[s] = np.where(dn, 1.0, 6.0)
            continue
        jx, jy, jz = xx + dx, yy + dy, zz + dz
        inside = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny) & (jz >= 0) & (jz < nz)
        nb_dir = np.zeros_like(inside)
        nb_dir[inside] = dn[jz[inside], jy[inside], jx[inside]]
        out[s] = np.where(inside & ~dn & ~nb_dir, -1.0, 0.0)
    return out.reshape(27, -1)
