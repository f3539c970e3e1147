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
          max_levels: int = 20):
    """AMG levels of A; the last one is solved directly."""
    levels = []
    A = sp.csr_matrix(A)
    free = np.asarray(free, dtype=bool)
    for _ in range(max_levels - 1):
        L = AmgLevel(A, free, degree=degree, eta=eta)
        levels.append(L)
        if A.shape[0] <= coarse_size:
            break
        agg = aggregates(A, free)
        T = tentative(agg)
        if T.shape[1] == 0 or T.shape[1] >= A.shape[0]:
            break
        L.agg = agg
        L.rho = gershgorin(A)
        L.omega = 4.0 / (3.0 * L.rho)
        Dinv = sp.diags(1.0 / A.diagonal())
        L.P = sp.csr_matrix(T - L.omega * (Dinv @ (A @ T)))
        A = sp.csr_matrix(L.P.T @ A @ L.P)
        free = np.ones(A.shape[0], dtype=bool)
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
