"""Algebraic multigrid below the region hierarchy (Section 3.5, coarse level solver, second
option): when the coarsest composite operator Abar is too large for a direct solver, the coarse
solve of the region cycle becomes one AMG V-cycle on Abar.  Test infrastructure only: a plain FP64
CPU statement of the method, never called by the library.

Hierarchy (smoothed aggregation, after the SA-AMG the section cites):

* aggregates: the staged plain aggregation of the hybrid section (hybrid.aggregate_region) without
  its interface stage, since one composite matrix has no interfaces: roots, joins, leftovers on the
  graph of couplings |a_ij| > 1e-12 sqrt(a_ii a_jj) between free rows (the rounding residue of a
  Galerkin product, which depends on the order of its sums, is no coupling).  Dirichlet rows are
  not aggregated.  Coarse rows are numbered by the smallest row of their aggregate;
* tentative prolongator T: a 1 in the column of its aggregate for every aggregated row (the
  constant near-null space of a scalar problem);
* systems (the section's "operator and its nullspace"): the rows are grouped into nodes (``nodes``:
  dof offsets), aggregation runs on the node graph in which nodes I and J are coupled when their
  block has ||A_IJ||_F > 1e-12 sqrt(||A_II||_F ||A_JJ||_F), a node is free when all its rows are, and
  the tentative prolongator is built from the near-null space B (rows x k): per aggregate, the rows
  of B of its dofs (ascending) are factored B_a = Q_a R_a (thin QR, diag(R_a) >= 0); Q_a fills the
  aggregate's k columns of T and R_a gives the coarse near-null space, whose nodes are the
  aggregates (k dofs each).  An aggregate with fewer than k dofs is an error;
* smoothed prolongator P = (I - omega D^-1 A) T, omega = 4 / (3 rho), rho = max_i sum_j |a_ij| / a_ii
  (Gershgorin's bound on lambda_max(D^-1 A), so no random start vector is needed);
* coarse operator P^T A P; coarsening stops at the first level with at most ``coarse_size`` rows,
  or when a level no longer shrinks, and that level is solved directly;
* smoother: the region levels' degree-K Chebyshev recurrence (Algorithm 2 as read for the region
  levels) on the interval [rho / eta, rho] of D^-1 A, the Gershgorin bound rho standing in for the
  power method's estimate (it bounds lambda_max from above, so no boost factor);
* cycle: a V-cycle with zero initial guess, the same polynomial before and after the coarse
  correction, so the cycle is a symmetric operator.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .hybrid import HRegion, aggregate_region


@dataclass
class AmgLevel:
    A: sp.csr_matrix
    free: np.ndarray
    agg: np.ndarray = None      # coarse row of every row, -1 if not aggregated
    P: sp.csr_matrix = None     # smoothed prolongator to the next level
    omega: float = 0.0
    rho: float = 0.0            # Gershgorin bound on lambda_max(D^-1 A)
    degree: int = 2             # Chebyshev degree
    eta: float = 20.0           # lambda_max / lambda_min of the smoothing interval
    Adense: np.ndarray = None   # coarsest level


STRENGTH = 1e-12


def aggregates(A: sp.csr_matrix, free: np.ndarray) -> np.ndarray:
    """Coarse row of every row (-1: not aggregated), numbered by each aggregate's smallest row."""
    n = A.shape[0]
    C = sp.coo_matrix(A)
    d = np.abs(A.diagonal())
    keep = (C.row == C.col) | (np.abs(C.data) > STRENGTH * np.sqrt(d[C.row] * d[C.col]))
    G = sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=A.shape)
    R = HRegion(G, np.arange(n), np.full((n, 1), -1), np.asarray(free, dtype=bool))
    lab, _ = aggregate_region(R, True, np.zeros(n, dtype=bool), (n, 1, 1), 0)
    out = np.full(n, -1, dtype=np.int64)
    number = {}
    for i in range(n):
        if lab[i] >= 0:
            if lab[i] not in number:
                number[lab[i]] = len(number)
            out[i] = number[lab[i]]
    return out


def node_graph(A: sp.csr_matrix, nodes: np.ndarray) -> sp.csr_matrix:
    """Nodes coupled by a block of Frobenius norm > STRENGTH sqrt(||A_II||_F ||A_JJ||_F)."""
    nn = nodes.size - 1
    node = np.repeat(np.arange(nn), np.diff(nodes))
    C = sp.coo_matrix(A)
    S = sp.csr_matrix((C.data ** 2, (node[C.row], node[C.col])), shape=(nn, nn))  # duplicates summed
    S.sum_duplicates()
    F = sp.coo_matrix(S)
    F.data = np.sqrt(F.data)
    d = np.zeros(nn)
    on = F.row == F.col
    d[F.row[on]] = F.data[on]
    keep = on | (F.data > STRENGTH * np.sqrt(d[F.row] * d[F.col]))
    return sp.csr_matrix((F.data[keep], (F.row[keep], F.col[keep])), shape=(nn, nn))


def tentative_system(agg: np.ndarray, nodes: np.ndarray, B: np.ndarray):
    """T and the coarse near-null space from per-aggregate thin QR of B (aggregates over nodes)."""
    k = B.shape[1]
    na = int(agg.max()) + 1 if (agg >= 0).any() else 0
    rows, cols, vals = [], [], []
    Bc = np.zeros((na * k, k))
    members = [[] for _ in range(na)]
    for I in range(agg.size):
        if agg[I] >= 0:
            members[agg[I]].extend(range(nodes[I], nodes[I + 1]))
    for a in range(na):
        dofs = np.asarray(sorted(members[a]), dtype=np.int64)
        if dofs.size < k:
            raise ValueError(f"aggregate {a} has {dofs.size} dofs, fewer than the near-null space's {k}")
        Q, R = np.linalg.qr(B[dofs])
        sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
        Q, R = Q * sgn, R * sgn[:, None]
        rows.append(np.repeat(dofs, k))
        cols.append(np.tile(np.arange(a * k, (a + 1) * k), dofs.size))
        vals.append(Q.ravel())
        Bc[a * k:(a + 1) * k] = R
    n = int(nodes[-1])
    if na == 0:
        return sp.csr_matrix((n, 0)), Bc
    T = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, na * k))
    return T, Bc


def rigid_body_modes(coords: np.ndarray) -> np.ndarray:
    """Near-null space of 3D elasticity at nodes (n, 3): three translations, then the rotations
    (-y, x, 0), (0, -z, y), (z, 0, -x); rows node-major, dof fastest."""
    n = coords.shape[0]
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    B = np.zeros((n, 3, 6))
    B[:, 0, 0] = B[:, 1, 1] = B[:, 2, 2] = 1.0
    B[:, 0, 3], B[:, 1, 3] = -y, x
    B[:, 1, 4], B[:, 2, 4] = -z, y
    B[:, 0, 5], B[:, 2, 5] = z, -x
    return B.reshape(3 * n, 6)


def tentative(agg: np.ndarray) -> sp.csr_matrix:
    rows = np.flatnonzero(agg >= 0)
    nc = int(agg.max()) + 1 if rows.size else 0
    return sp.csr_matrix((np.ones(rows.size), (rows, agg[rows])), shape=(agg.size, nc))


def gershgorin(A: sp.csr_matrix) -> float:
    """rho = max_i sum_j |a_ij| / a_ii >= lambda_max(D^-1 A)."""
    d = A.diagonal()
    rowabs = np.asarray(abs(A).sum(axis=1)).ravel()
    return float(np.max(rowabs / d))


def setup(A: sp.csr_matrix, free: np.ndarray, coarse_size: int = 2000, degree: int = 2, eta: float = 20.0,
          max_levels: int = 20, nodes: np.ndarray = None, B: np.ndarray = None):
    """AMG levels of A; the last one is solved directly.  ``nodes`` (dof offsets of the nodes) and
    ``B`` (near-null space, rows x k) select the system form; ``free`` flags rows."""
    levels = []
    A = sp.csr_matrix(A)
    free = np.asarray(free, dtype=bool)
    for _ in range(max_levels - 1):
        L = AmgLevel(A, free, degree=degree, eta=eta)
        levels.append(L)
        if A.shape[0] <= coarse_size:
            break
        if nodes is None:
            agg = aggregates(A, free)
            T = tentative(agg)
        else:
            nfree = np.array([free[nodes[I]:nodes[I + 1]].all() for I in range(nodes.size - 1)])
            agg = aggregates(node_graph(A, nodes), nfree)
            T, Bc = tentative_system(agg, nodes, B)
        if T.shape[1] == 0 or T.shape[1] >= A.shape[0]:
            break
        L.agg = agg
        L.rho = gershgorin(A)
        L.omega = 4.0 / (3.0 * L.rho)
        Dinv = sp.diags(1.0 / A.diagonal())
        L.P = sp.csr_matrix(T - L.omega * (Dinv @ (A @ T)))
        A = sp.csr_matrix(L.P.T @ A @ L.P)
        free = np.ones(A.shape[0], dtype=bool)
        if nodes is not None:
            k = B.shape[1]
            nodes, B = np.arange(0, A.shape[0] + 1, k), Bc
    else:
        levels.append(AmgLevel(A, free, degree=degree, eta=eta))
    last = levels[-1]
    last.agg, last.P = None, None
    last.Adense = last.A.toarray()
    return levels


def chebyshev(L: AmgLevel, u, b, r):
    """Degree-K Chebyshev smoothing on [rho / eta, rho]; r = b - A u on entry."""
    alpha = L.rho / L.eta
    beta = L.rho
    theta = 0.5 * (alpha + beta)
    delta = 2.0 / (beta - alpha)
    rho = 1.0 / (theta * delta)
    dinv = 1.0 / L.A.diagonal()
    d = (1.0 / theta) * (dinv * r)
    u = u + d
    for _ in range(L.degree - 1):
        r = b - L.A @ u
        rho_old = rho
        rho = 1.0 / (2.0 * theta * delta - rho_old)
        d = (rho * rho_old) * d + (2.0 * rho * delta) * (dinv * r)
        u = u + d
    return u


def vcycle(levels, b: np.ndarray, l: int = 0) -> np.ndarray:
    """z = V_l(b) with zero initial guess."""
    L = levels[l]
    if L.P is None:
        return np.linalg.solve(L.Adense, b)
    u = chebyshev(L, np.zeros_like(b), b, b)
    r = b - L.A @ u
    u = u + L.P @ vcycle(levels, L.P.T @ r, l + 1)
    return chebyshev(L, u, b, b - L.A @ u)
