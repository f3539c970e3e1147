"""Regional operators [[A]] = diag(A^(k)) and the composite operator A
(paper Section 3.1, eq. "extraction sum" and its two restrictions; Section 4,
the splitting rule; region-local element assembly as one admissible split).

Stencil storage (one region): ``coef[s]`` is the coupling of a node to the
neighbour at offset ``offsets(dim)[s]``; shape (S, ez, ey, ex) for scalar
problems and (S, ez, ey, ex, ndof, ndof) for systems ([row comp, col comp]).
S = 9 in 2D, 27 in 3D, s = (dz+1)*9 + (dy+1)*3 + (dx+1).  Couplings to nodes
outside the region box are zero.

Boundary conditions (reading: homogeneous Dirichlet on the masked faces).
Dirichlet nodes stay in the grid as identity rows with all couplings to and
from them removed (symmetric elimination); the identity diagonal is split as
1/mult over the copies of a Dirichlet interface node.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import fem
from .regions import Layout


def offsets(dim):
    rng = (-1, 0, 1)
    if dim == 2:
        return [(dx, dy) for dy in rng for dx in rng]
    return [(dx, dy, dz) for dz in rng for dy in rng for dx in rng]


def center(dim):
    return 4 if dim == 2 else 13


def _shift(x, off, dim):
    """x shifted so that out[i] = x[i + off], zero outside the box (first dim axes only)."""
    pad = [(1, 1)] * dim + [(0, 0)] * (x.ndim - dim)
    xp = np.pad(x, pad)
    sl = []
    for ax in range(dim):
        d = off[dim - 1 - ax]  # numpy axis ax is coordinate dim-1-ax
        n = x.shape[ax]
        sl.append(slice(1 + d, 1 + d + n))
    return xp[tuple(sl)]


def apply_stencil(coef, x, dim, ndof=1):
    """y = A^(k) x for one region (no interface summation)."""
    y = np.zeros_like(x)
    for s, off in enumerate(offsets(dim)):
        xs = _shift(x, off, dim)
        if ndof == 1:
            y += coef[s] * xs
        else:
            y += np.einsum("...ab,...b->...a", coef[s], xs)
    return y


def region_node_index(shape):
    return np.arange(int(np.prod(shape))).reshape(shape)


def stencil_to_csr(coef, dim, ndof=1):
    """Region-local sparse matrix of a stencil (node-major, dof-minor numbering)."""
    shape = coef.shape[1:1 + dim]
    idx = region_node_index(shape)
    n = idx.size
    rows, cols, vals = [], [], []
    for s, off in enumerate(offsets(dim)):
        nb = _shift(idx + 1, off, dim) - 1  # -1 where the neighbour is outside
        ok = nb >= 0
        r = idx[ok]
        c = nb[ok]
        if ndof == 1:
            rows.append(r)
            cols.append(c)
            vals.append(coef[s][ok])
        else:
            blk = coef[s][ok]  # (m, ndof, ndof)
            for a in range(ndof):
                for b in range(ndof):
                    rows.append(r * ndof + a)
                    cols.append(c * ndof + b)
                    vals.append(blk[:, a, b])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * ndof, n * ndof))


def csr_to_stencil(M, shape, dim, ndof=1):
    """Stencil arrays of a region-local sparse matrix; every entry must fit the stencil."""
    M = sp.csr_matrix(M)
    idx = region_node_index(shape)
    S = len(offsets(dim))
    coef = np.zeros((S,) + tuple(shape) + ((ndof, ndof) if ndof > 1 else ()))
    covered = 0.0
    for s, off in enumerate(offsets(dim)):
        nb = _shift(idx + 1, off, dim) - 1
        ok = nb >= 0
        r = idx[ok]
        c = nb[ok]
        if ndof == 1:
            v = np.asarray(M[r, c]).reshape(-1)
            coef[s][ok] = v
            covered += np.abs(v).sum()
        else:
            blk = np.zeros((r.size, ndof, ndof))
            for a in range(ndof):
                for b in range(ndof):
                    blk[:, a, b] = np.asarray(M[r * ndof + a, c * ndof + b]).reshape(-1)
            coef[s][ok] = blk
            covered += np.abs(blk).sum()
    total = np.abs(M.data).sum()
    if not np.isclose(covered, total, rtol=1e-12, atol=1e-300):
        raise ValueError("matrix has entries outside the stencil pattern")
    return coef


# --------------------------------------------------------------- Dirichlet
def eliminate_regional(lay: Layout, k: int, coef):
    """Symmetric Dirichlet elimination of one region's stencil (in place)."""
    dim, ndof = lay.dim, lay.ndof
    dn = lay.dirichlet[lay.box(k)]
    mult = lay.mult[lay.box(k)].astype(np.float64)
    for s, off in enumerate(offsets(dim)):
        nb_d = _shift(dn.astype(np.int8), off, dim).astype(bool)
        coef[s][dn] = 0.0
        coef[s][nb_d] = 0.0
    c = center(dim)
    if ndof == 1:
        coef[c][dn] = 1.0 / mult[dn]
    else:
        coef[c][dn] = np.eye(ndof)[None, :, :] / mult[dn][:, None, None]
    return coef


def eliminate_csr(A, dn_flat):
    """Symmetric Dirichlet elimination of a composite sparse matrix."""
    A = sp.csr_matrix(A)
    keep = sp.diags((~dn_flat).astype(np.float64))
    A = keep @ A @ keep
    A = A + sp.diags(dn_flat.astype(np.float64))
    A.eliminate_zeros()
    return sp.csr_matrix(A)


def dirichlet_dofs(lay: Layout):
    dn = lay.dirichlet.reshape(-1)
    return np.repeat(dn, lay.ndof) if lay.ndof > 1 else dn


# -------------------------------------------------------- composite matrices
def composite_fd5(lay: Layout):
    """Composite five-point operator with eliminated Dirichlet nodes."""
    assert lay.dim == 2 and lay.ndof == 1
    ny, nx = lay.shape
    idx = np.arange(nx * ny).reshape(ny, nx)
    rows, cols, vals = [], [], []
    for (dx, dy), v in fem.fd5_offsets().items():
        ys = slice(max(0, -dy), ny - max(0, dy))
        xs = slice(max(0, -dx), nx - max(0, dx))
        r = idx[ys, xs].reshape(-1)
        c = (idx[ys, xs] + dy * nx + dx).reshape(-1)
        rows.append(r)
        cols.append(c)
        vals.append(np.full(r.size, v))
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nx * ny, nx * ny))
    return eliminate_csr(A, dirichlet_dofs(lay))


def composite_fd7(lay: Layout):
    """Composite seven-point Laplacian (6 on the diagonal, -1 to each face neighbour) with
    eliminated Dirichlet nodes."""
    assert lay.dim == 3 and lay.ndof == 1
    nz, ny, nx = lay.shape
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols, vals = [idx.reshape(-1)], [idx.reshape(-1)], [np.full(n, 6.0)]
    for ax in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[ax] = slice(0, -1)
        b[ax] = slice(1, None)
        lo, hi = idx[tuple(a)].reshape(-1), idx[tuple(b)].reshape(-1)
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [np.full(lo.size, -1.0), np.full(lo.size, -1.0)]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return eliminate_csr(A, dirichlet_dofs(lay))


def composite_q1(lay: Layout, pde, h=1.0, elem_coef=None, youngs=None, nu=0.3):
    """Composite Q1 operator assembled element by element over the whole mesh."""
    assert lay.dim == 3
    nz, ny, nx = lay.shape
    ndof = lay.ndof
    node = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    ez, ey, ex = nz - 1, ny - 1, nx - 1
    rows, cols, vals = [], [], []
    if pde in ("laplace", "diffusion"):
        K = fem.q1_laplace(h)
        c = np.ones((ez, ey, ex)) if elem_coef is None else np.asarray(elem_coef, dtype=np.float64)
        for a, ca in enumerate(fem.CORNERS3):
            ra = node[ca[2]:ca[2] + ez, ca[1]:ca[1] + ey, ca[0]:ca[0] + ex].reshape(-1)
            for b, cb in enumerate(fem.CORNERS3):
                rb = node[cb[2]:cb[2] + ez, cb[1]:cb[1] + ey, cb[0]:cb[0] + ex].reshape(-1)
                rows.append(ra)
                cols.append(rb)
                vals.append(K[a, b] * c.reshape(-1))
    elif pde == "elasticity":
        # Young's modulus per element from the region containing it
        Ee = np.zeros((ez, ey, ex))
        for k in range(lay.nreg):
            o, e = lay.origins[k], lay.extents[k]
            Ee[o[2]:o[2] + e[2] - 1, o[1]:o[1] + e[1] - 1, o[0]:o[0] + e[0] - 1] = youngs[k]
        K1 = fem.q1_elasticity(1.0, nu, h)  # linear in E
        for a, ca in enumerate(fem.CORNERS3):
            ra = node[ca[2]:ca[2] + ez, ca[1]:ca[1] + ey, ca[0]:ca[0] + ex].reshape(-1)
            for b, cb in enumerate(fem.CORNERS3):
                rb = node[cb[2]:cb[2] + ez, cb[1]:cb[1] + ey, cb[0]:cb[0] + ex].reshape(-1)
                for i in range(3):
                    for j in range(3):
                        rows.append(ra * 3 + i)
                        cols.append(rb * 3 + j)
                        vals.append(K1[3 * a + i, 3 * b + j] * Ee.reshape(-1))
    else:
        raise ValueError(pde)
    n = nx * ny * nz * ndof
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return eliminate_csr(A, dirichlet_dofs(lay))


def q1_rows(shape_xyz, dirichlet, x, nodes, pde, h=1.0, elem_coef=None, nu=0.3):
    """Rows of the composite Q1 product A x at selected nodes, evaluated one by one from the
    element definition (for sizes where A itself is too large to assemble here).

    A free node's row sums c_e K_e over the (up to 8) elements containing it, with the columns of
    Dirichlet unknowns removed (symmetric elimination); a Dirichlet node's row is the identity.
    ``elem_coef`` (composite element grid, [z][y][x]) is the diffusion coefficient, or the
    Young's modulus per element for elasticity (K_e is linear in E); x is a composite array
    [z][y][x] (and [dof] for elasticity).  Returns an array (len(nodes),) or (len(nodes), 3).
    """
    nx, ny, nz = shape_xyz
    elastic = pde == "elasticity"
    K = fem.q1_elasticity(1.0, nu, h) if elastic else fem.q1_laplace(h)
    nd = 3 if elastic else 1
    out = np.zeros((len(nodes), nd))
    for r, (gx, gy, gz) in enumerate(nodes):
        if dirichlet[gz, gy, gx]:
            out[r] = x[gz, gy, gx]
            continue
        for ez in (gz - 1, gz):
            for ey in (gy - 1, gy):
                for ex in (gx - 1, gx):
                    if not (0 <= ex < nx - 1 and 0 <= ey < ny - 1 and 0 <= ez < nz - 1):
                        continue
                    c = 1.0 if elem_coef is None else float(elem_coef[ez, ey, ex])
                    a = (gx - ex) + 2 * (gy - ey) + 4 * (gz - ez)
                    for b, cb in enumerate(fem.CORNERS3):
                        bx, by, bz = ex + cb[0], ey + cb[1], ez + cb[2]
                        if dirichlet[bz, by, bx]:
                            continue
                        xb = np.atleast_1d(x[bz, by, bx])
                        out[r] += c * (K[nd * a:nd * a + nd, nd * b:nd * b + nd] @ xb)
    return out[:, 0] if nd == 1 else out


# --------------------------------------------------------- regional matrices
def regional_q1(lay: Layout, pde, h=1.0, elem_coef=None, youngs=None, nu=0.3):
    """Per-region element assembly: A^(k) collects the elements inside region k.

    Each element lies in exactly one region, so sum_k Psi_k A^(k) Psi_k^T = A.
    """
    assert lay.dim == 3
    offs = offsets(3)
    sidx = {o: s for s, o in enumerate(offs)}
    out = []
    if pde in ("laplace", "diffusion"):
        K = fem.q1_laplace(h)
    else:
        K1 = fem.q1_elasticity(1.0, nu, h)
    for k in range(lay.nreg):
        shp = lay.region_shape(k)
        ez, ey, ex = (n - 1 for n in shp)
        o = lay.origins[k]
        if pde in ("laplace", "diffusion"):
            coef = np.zeros((27,) + shp)
            if elem_coef is None:
                ce = np.ones((ez, ey, ex))
            else:
                ce = np.asarray(elem_coef)[o[2]:o[2] + ez, o[1]:o[1] + ey, o[0]:o[0] + ex]
            for a, ca in enumerate(fem.CORNERS3):
                for b, cb in enumerate(fem.CORNERS3):
                    s = sidx[(cb[0] - ca[0], cb[1] - ca[1], cb[2] - ca[2])]
                    coef[s][ca[2]:ca[2] + ez, ca[1]:ca[1] + ey, ca[0]:ca[0] + ex] += K[a, b] * ce
        elif pde == "elasticity":
            coef = np.zeros((27,) + shp + (3, 3))
            Ke = youngs[k] * K1
            for a, ca in enumerate(fem.CORNERS3):
                for b, cb in enumerate(fem.CORNERS3):
                    s = sidx[(cb[0] - ca[0], cb[1] - ca[1], cb[2] - ca[2])]
                    blk = Ke[3 * a:3 * a + 3, 3 * b:3 * b + 3]
                    coef[s][ca[2]:ca[2] + ez, ca[1]:ca[1] + ey, ca[0]:ca[0] + ex] += blk
        else:
            raise ValueError(pde)
        out.append(eliminate_regional(lay, k, coef))
    return out


def split_composite(lay: Layout, A):
    """Non-invasive split of an assembled composite matrix into region matrices (Section 4).

    Off-diagonal A_ij is divided by q, the number of regions containing both
    i and j.  The diagonal of region k's matrix is z_i / mult_i minus the sum
    of its split off-diagonals, with z = A 1, so each region matrix has the
    row sums of A shared out by multiplicity (the edge-based rule with the
    constant nullspace vector; for rows of A with zero sum this is the
    zero-row-sum rule).  Scalar problems only.
    """
    assert lay.ndof == 1
    A = sp.csr_matrix(A)
    dim = lay.dim
    z = np.asarray(A @ np.ones(A.shape[0])).reshape(lay.shape)
    comp_idx = np.arange(A.shape[0]).reshape(lay.shape)
    coords = np.indices(lay.shape)  # numpy axes order
    out = []
    c = center(dim)
    for k in range(lay.nreg):
        sl = lay.box(k)
        shp = lay.region_shape(k)
        coef = np.zeros((len(offsets(dim)),) + shp)
        I = comp_idx[sl]
        for s, off in enumerate(offsets(dim)):
            if s == c:
                continue
            nb = _shift(I + 1, off, dim) - 1
            ok = nb >= 0
            vals = np.asarray(A[I[ok], nb[ok]]).reshape(-1)
            # q = number of regions containing both endpoints
            q = np.zeros(vals.size)
            pi = [coords[ax][sl][ok] for ax in range(dim)]
            pj = [p + off[dim - 1 - ax] for ax, p in enumerate(pi)]
            for m in range(lay.nreg):
                bm = lay.box(m)
                inside_i = np.ones(vals.size, dtype=bool)
                inside_j = np.ones(vals.size, dtype=bool)
                for ax in range(dim):
                    inside_i &= (pi[ax] >= bm[ax].start) & (pi[ax] < bm[ax].stop)
                    inside_j &= (pj[ax] >= bm[ax].start) & (pj[ax] < bm[ax].stop)
                q += inside_i & inside_j
            coef[s][ok] = vals / q
        offsum = coef.sum(axis=0)
        coef[c] = z[sl] / lay.mult[sl] - offsum
        out.append(coef)
    return out


def regional_fd5(lay: Layout):
    """Region matrices of the 2D five-point problem by the splitting rule of Section 4."""
    return split_composite(lay, composite_fd5(lay))


def assemble_from_regions(lay: Layout, coefs):
    """Psi [[A]] Psi^T as a composite sparse matrix (Lemma on the block region matrix)."""
    n = lay.n_composite
    A = sp.csr_matrix((n, n))
    for k in range(lay.nreg):
        Pk = lay.psi_block(k)
        A = A + Pk @ stencil_to_csr(coefs[k], lay.dim, lay.ndof) @ Pk.T
    return sp.csr_matrix(A)


def diagonal(coef, dim, ndof=1):
    """Point diagonal of a region stencil (the scalar diagonal of each dof row)."""
    c = coef[center(dim)]
    if ndof == 1:
        return c.copy()
    return np.einsum("...aa->...a", c).copy()
