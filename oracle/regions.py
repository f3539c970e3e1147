"""Regions, regional vectors and the boolean map Psi (paper Section 3.1; Section 4,
application-supplied region information).

A region is a box of grid nodes.  Neighbouring boxes share interface nodes; a
node's multiplicity is the number of boxes containing it (2/4/8 on faces,
edges and corners of a 3D tensor layout).  A regional vector is a list of
per-region arrays (numpy shape (ez, ey, ex[, ndof]), x fastest).

Psi (composite n x regional n_r) has one nonzero per column.  Its actions
are written as index operations, as the paper's software does:

* Psi^T v        -- copy composite values into every region (``to_regional``)
* Psi [[v]]      -- sum co-located copies (``to_composite_sum``)
* Psi^T Psi [[v]]-- sum co-located copies, write the sum back to every copy
* (Psi Psi^T)^-1 Psi [[v]] -- average of co-located copies

The explicit sparse Psi is built only for small pin tests.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def coarse_positions(e: int):
    """Local positions of a region's coarse nodes along an axis of e nodes: 0, 3, 6, ... below
    e - 1, then e - 1 (Section 3.2: the region's end nodes must be coarse)."""
    return list(range(0, e - 1, 3)) + [e - 1]


class Layout:
    """Region boxes on a composite node lattice."""

    def __init__(self, dim, origins, extents, dirichlet_mask=0, ndof=1, check=True):
        self.dim = int(dim)
        self.ndof = int(ndof)
        self.origins = np.asarray(origins, dtype=np.int64).reshape(-1, dim)
        self.extents = np.asarray(extents, dtype=np.int64).reshape(-1, dim)
        self.nreg = self.origins.shape[0]
        self.dirichlet_mask = int(dirichlet_mask)
        self.shape_xyz = tuple(int(v) for v in (self.origins + self.extents).max(axis=0))
        self.shape = tuple(reversed(self.shape_xyz))  # numpy shape, x fastest
        self.mult = np.zeros(self.shape, dtype=np.int64)
        self.owner = np.full(self.shape, -1, dtype=np.int64)
        for k in range(self.nreg):
            sl = self.box(k)
            self.mult[sl] += 1
            own = self.owner[sl]
            own[own < 0] = k
        if check:
            self._check()
        self.dirichlet = self._dirichlet_nodes()

    # ----------------------------------------------------------------- boxes
    def box(self, k):
        """numpy slice of region k in a composite node array."""
        o, e = self.origins[k], self.extents[k]
        return tuple(slice(int(o[d]), int(o[d] + e[d])) for d in reversed(range(self.dim)))

    def region_shape(self, k):
        return tuple(int(v) for v in reversed(self.extents[k]))

    def _check(self):
        if (self.extents < 2).any():
            raise ValueError("region extents must be >= 2")
        if (self.mult == 0).any():
            raise ValueError("composite nodes not covered by any region")
        # cells (elements) must be covered exactly once: regions overlap only at interfaces
        cells = np.zeros(tuple(n - 1 for n in self.shape), dtype=np.int64)
        for k in range(self.nreg):
            o, e = self.origins[k], self.extents[k]
            cells[tuple(slice(int(o[d]), int(o[d] + e[d] - 1)) for d in reversed(range(self.dim)))] += 1
        if (cells != 1).any():
            raise ValueError("regions must tile the domain, overlapping only at interfaces")

    def _dirichlet_nodes(self):
        out = np.zeros(self.shape, dtype=bool)
        for d in range(self.dim):
            ax = self.dim - 1 - d
            for side in (0, 1):
                if self.dirichlet_mask & (1 << (2 * d + side)):
                    sl = [slice(None)] * self.dim
                    sl[ax] = 0 if side == 0 else self.shape_xyz[d] - 1
                    out[tuple(sl)] = True
        return out

    def coarsen(self):
        """Layout of the next level (coarsening rate 3, Section 3.2 construction rules).

        Along each axis a region keeps every third node counted from its first one, and its last
        node (``coarse_positions``), so its end nodes -- the interface -- are coarse and its last
        coarse interval spans 1, 2 or 3 cells.  The composite coarse lattice along an axis is the
        union of the regions' coarse positions; it must agree with each region's own choice on
        that region's range, so that co-located fine interface nodes see the same coarse nodes from
        every region.  ``fine_positions`` of the result keeps, per axis, the composite fine
        coordinate of each coarse lattice line.  With region extents - 1 and origins divisible by 3
        this is every third node of the composite lattice.
        """
        origins = np.zeros_like(self.origins)
        extents = np.zeros_like(self.extents)
        lines = []
        for d in range(self.dim):
            local = [[int(o) + p for p in coarse_positions(int(e))]
                     for o, e in zip(self.origins[:, d], self.extents[:, d])]
            lattice = sorted({g for pts in local for g in pts})
            index = {g: i for i, g in enumerate(lattice)}
            for k, pts in enumerate(local):
                inside = [g for g in lattice if pts[0] <= g <= pts[-1]]
                if inside != pts:
                    raise ValueError(f"coarse points of region {k} disagree with its neighbours' along axis {d}")
                origins[k, d] = index[pts[0]]
                extents[k, d] = len(pts)
            lines.append(np.asarray(lattice, dtype=np.int64))
        coarse = Layout(self.dim, origins, extents, self.dirichlet_mask, self.ndof)
        coarse.fine_positions = lines
        return coarse

    # ------------------------------------------------------------- vectors
    def _vshape(self, shape):
        return shape + ((self.ndof,) if self.ndof > 1 else ())

    def zeros_regional(self):
        return [np.zeros(self._vshape(self.region_shape(k))) for k in range(self.nreg)]

    def to_regional(self, comp):
        """[[v]] = Psi^T v."""
        return [np.array(comp[self.box(k)], dtype=np.float64, copy=True) for k in range(self.nreg)]

    def to_composite_sum(self, reg):
        """w = Psi [[v]]: sum of co-located copies, accumulated in ascending region order."""
        comp = np.zeros(self._vshape(self.shape))
        for k in range(self.nreg):
            comp[self.box(k)] += reg[k]
        return comp

    def to_composite_owner(self, reg):
        """Composite vector taking the copy of the lowest-numbered region containing each node."""
        comp = np.zeros(self._vshape(self.shape))
        for k in reversed(range(self.nreg)):
            comp[self.box(k)] = reg[k]
        return comp

    def to_composite_avg(self, reg):
        """w = (Psi Psi^T)^-1 Psi [[v]]: average of co-located copies."""
        s = self.to_composite_sum(reg)
        m = self.mult if self.ndof == 1 else self.mult[..., None]
        return s / m

    def interface_sum(self, reg):
        """Psi^T Psi [[v]]: every copy receives the sum of its co-located copies."""
        return self.to_regional(self.to_composite_sum(reg))

    def mult_regional(self):
        return self.to_regional(self.mult.astype(np.float64))

    def dot(self, a, b):
        """Composite inner product of two consistent regional vectors (each dof counted once)."""
        return float(np.sum(self.to_composite_owner(a) * self.to_composite_owner(b)))

    def norm(self, a):
        return float(np.sqrt(self.dot(a, a)))

    def flatten(self, reg):
        """Regional vector in the library's flat layout: region after region, x fastest."""
        return np.concatenate([r.reshape(-1) for r in reg])

    def unflatten(self, flat):
        out, pos = [], 0
        for k in range(self.nreg):
            shp = self._vshape(self.region_shape(k))
            n = int(np.prod(shp))
            out.append(np.asarray(flat[pos:pos + n], dtype=np.float64).reshape(shp))
            pos += n
        return out

    @property
    def n_composite(self):
        return int(np.prod(self.shape)) * self.ndof

    @property
    def n_regional(self):
        return int(sum(np.prod(self.region_shape(k)) for k in range(self.nreg))) * self.ndof

    # ------------------------------------------------- explicit Psi (pins)
    def psi_matrix(self):
        """Explicit boolean Psi (n x n_r), dof-interleaved; for small pin tests only."""
        rows, cols = [], []
        col = 0
        idx = np.arange(self.n_composite).reshape(self._vshape(self.shape))
        for k in range(self.nreg):
            ids = idx[self.box(k)].reshape(-1)
            rows.append(ids)
            cols.append(np.arange(col, col + ids.size))
            col += ids.size
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(self.n_composite, col))

    def psi_block(self, k):
        """Psi_k: the columns of Psi belonging to region k."""
        idx = np.arange(self.n_composite).reshape(self._vshape(self.shape))
        ids = idx[self.box(k)].reshape(-1)
        return sp.csr_matrix((np.ones(ids.size), (ids, np.arange(ids.size))),
                             shape=(self.n_composite, ids.size))
