"""Grid transfers with coarsening rate 3 (paper Section 3.2 construction rules,
eq. "region interp" and "region restriction"; Section 6.1 linear interpolation
with rate 3).

Linear interpolation in 1D: a fine node x between consecutive coarse nodes at
fine positions p0 < p1 takes weight (p1 - x)/(p1 - p0) from the left one and
(x - p0)/(p1 - p0) from the right one; a node at a coarse position takes weight 1
from it.  In 2D/3D the weights are tensor products.  A region's coarse nodes are
every third node from its first one plus its last node (regions.coarse_positions),
so for extents 3^k + 1 the weights are 1, 2/3, 1/3 everywhere, and otherwise the
region's last interval is shorter.  Fine interface nodes interpolate only from
coarse nodes on the same interface and co-located rows match across regions,
because the coarse lattice agrees on every shared interface (Layout.coarsen).

Reading for Dirichlet nodes: a free fine node takes no weight from a
Dirichlet coarse node (interpolation of the interior unknowns with a zero
boundary); a Dirichlet fine node keeps its weights, which all come from
Dirichlet coarse nodes on the same face.  Systems use the scalar weights per
displacement component.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .regions import Layout, coarse_positions


def p1d(nf: int, pos=None) -> sp.csr_matrix:
    """1D linear interpolation onto nf fine nodes from coarse nodes at the increasing fine
    positions ``pos`` (first 0, last nf - 1; default: a region's rate-3 positions)."""
    pos = coarse_positions(nf) if pos is None else [int(p) for p in pos]
    if pos[0] != 0 or pos[-1] != nf - 1 or any(b <= a for a, b in zip(pos, pos[1:])):
        raise ValueError("coarse positions must increase from 0 to nf - 1")
    rows, cols, vals = [], [], []
    for c in range(len(pos) - 1):
        p0, p1 = pos[c], pos[c + 1]
        m = p1 - p0
        for x in range(p0, p1):
            rows.append(x)
            cols.append(c)
            vals.append((p1 - x) / m)
            if x > p0:
                rows.append(x)
                cols.append(c + 1)
                vals.append((x - p0) / m)
    rows.append(nf - 1)
    cols.append(len(pos) - 1)
    vals.append(1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, len(pos)))


def _tensor(shape_np, pos_np=None):
    """Kronecker product of 1D interpolations; numpy shape (x fastest) -> C-order."""
    M = sp.csr_matrix(np.ones((1, 1)))
    for a, n in enumerate(shape_np):  # slowest axis first
        M = sp.kron(M, p1d(n, None if pos_np is None else pos_np[a]), format="csr")
    return M


def _apply_dirichlet(P, dn_fine, dn_coarse):
    P = sp.coo_matrix(P)
    drop = (~dn_fine[P.row]) & dn_coarse[P.col]
    keep = ~drop
    return sp.csr_matrix((P.data[keep], (P.row[keep], P.col[keep])), shape=P.shape)


def region_prolongator(fine: Layout, coarse: Layout, k: int) -> sp.csr_matrix:
    """Psi_k^T P Psi-bar_k: region k's block of the interface-replicated interpolation."""
    P = _tensor(fine.region_shape(k))
    dnf = fine.dirichlet[fine.box(k)].reshape(-1)
    dnc = coarse.dirichlet[coarse.box(k)].reshape(-1)
    P = _apply_dirichlet(P, dnf, dnc)
    if fine.ndof > 1:
        P = sp.kron(P, sp.identity(fine.ndof), format="csr")
    return P


def composite_prolongator(fine: Layout, coarse: Layout) -> sp.csr_matrix:
    """Composite linear interpolation P on the whole lattice (never formed by the regional
    method); ``coarse`` must come from ``fine.coarsen()``, whose lattice lines it interpolates from."""
    P = _tensor(fine.shape, list(reversed(coarse.fine_positions)))
    P = _apply_dirichlet(P, fine.dirichlet.reshape(-1), coarse.dirichlet.reshape(-1))
    if fine.ndof > 1:
        P = sp.kron(P, sp.identity(fine.ndof), format="csr")
    return P


def regional_prolongate(fine: Layout, coarse: Layout, Pk, ubar):
    """[[w]] = P^(r) [[v]]: region-local products, no interface communication."""
    out = []
    for k in range(fine.nreg):
        v = ubar[k].reshape(-1)
        out.append((Pk[k] @ v).reshape(fine.zeros_regional()[k].shape))
    return out


def regional_restrict(fine: Layout, coarse: Layout, Pk, r):
    """[[w]] = Psi-bar^T Psi-bar R^(r) [[Psi Psi^T]]^-1 [[r]] with R^(r) = P^(r)T.

    Region-local scaling by 1/multiplicity, region-local transpose product,
    then the coarse interface sum.
    """
    mult = fine.mult_regional()
    local = []
    for k in range(fine.nreg):
        m = mult[k] if fine.ndof == 1 else mult[k][..., None]
        v = (r[k] / m).reshape(-1)
        local.append((Pk[k].T @ v).reshape(coarse.zeros_regional()[k].shape))
    return coarse.interface_sum(local)
