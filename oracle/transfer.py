"""Grid transfers with coarsening rate 3 (paper Section 3.2 construction rules,
eq. "region interp" and "region restriction"; Section 6.1 linear interpolation
with rate 3).

Linear interpolation in 1D: fine node x = 3c + t (t in {0, 1, 2}) takes
weight 1 - t/3 from coarse node c and t/3 from coarse node c + 1; in 2D/3D
the weights are tensor products.  Coarse nodes are the fine nodes whose
coordinates are multiples of 3, so fine interface nodes interpolate only from
coarse nodes on the same interface and co-located rows match across regions.

Reading for Dirichlet nodes: a free fine node takes no weight from a
Dirichlet coarse node (interpolation of the interior unknowns with a zero
boundary); a Dirichlet fine node keeps its weights, which all come from
Dirichlet coarse nodes on the same face.  Systems use the scalar weights per
displacement component.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .regions import Layout


def p1d(nf: int) -> sp.csr_matrix:
    """1D linear interpolation from (nf-1)/3+1 coarse nodes to nf fine nodes."""
    if (nf - 1) % 3:
        raise ValueError("fine extent - 1 must be divisible by 3")
    nc = (nf - 1) // 3 + 1
    rows, cols, vals = [], [], []
    for x in range(nf):
        c, t = divmod(x, 3)
        rows.append(x)
        cols.append(c)
        vals.append((3 - t) / 3.0)
        if t:
            rows.append(x)
            cols.append(c + 1)
            vals.append(t / 3.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def _tensor(shape_np):
    """Kronecker product of 1D interpolations; numpy shape (x fastest) -> C-order."""
    M = sp.csr_matrix(np.ones((1, 1)))
    for n in shape_np:  # slowest axis first
        M = sp.kron(M, p1d(n), format="csr")
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
    """Composite linear interpolation P on the whole lattice (never formed by the regional method)."""
    P = _tensor(fine.shape)
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
