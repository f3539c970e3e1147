"""Regional multigrid with structured and unstructured regions (the paper's structured/unstructured
mesh hybrid section and its Table 5 experiment).  Test infrastructure only: a plain FP64 CPU
statement of the method, never called by the library.

Every region's matrix on every level is a sparse matrix; grid transfers are piecewise constant
(plain aggregation), P^(k) having a single 1 per aggregated row.  Coarsening:

* structured region: a free node joins the aggregate of its nearest rate-3 coarse point (the
  composite coordinates that are multiples of 3), so aggregates are 3x3x3 boxes;
* unstructured region: staged plain aggregation.  Stage I (the interface stage the section adds)
  aggregates the region's interface nodes with the structured rule above, so that every copy of
  an interface node ends in the same coarse node in every region (the Lemma on P); the standard
  stages follow: II roots (a node whose free neighbours are all unaggregated takes them), III
  joins (a leftover joins the neighbouring aggregate it has most couplings to), IV leftovers (a
  node still unaggregated starts an aggregate with its unaggregated neighbours).

Readings of points the paper leaves open (both sides of the library follow them):

* nearest coarse point per axis: c = 3 floor((g + 1) / 3); a coarse point on a Dirichlet face
  moves one coarse step inward (Dirichlet nodes are never aggregated and have no coarse node);
* graph neighbours are the nonzero off-diagonal entries of the region's matrix between free nodes;
* stage III decides from the aggregates as they stand when the stage starts; ties go to the
  aggregate whose smallest member has the smallest local index; stage IV is sequential;
* the coarse nodes of a region are ordered by the smallest local index in their aggregate;
* coarse composite numbering: regions in order, their coarse nodes in order, a new number at the
  first sight of a node (nodes with coordinates are the same node in every region);
* Galerkin product per region, A_c^(k) = P^(k)T A^(k) P^(k) (the Theorem); restriction by the
  regional formula of Section 3.3 (residual divided by multiplicity, P^T, coarse interface sum);
* cycle: ``degree`` smoothing iterations before and after the coarse correction, gamma coarse
  cycles per visit (2: W-cycle), dense direct solve on the coarsest composite matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assembly
from .regions import Layout


@dataclass
class HOptions:
    nlevels: int = 3
    degree: int = 2           # smoothing iterations before and after the coarse correction
    smoother: str = "symgs"   # "jacobi", "gs" (forward), "symgs" (forward then backward)
    omega: float = 1.0
    gamma: int = 2            # 1 V-cycle, 2 W-cycle


@dataclass
class HRegion:
    A: sp.csr_matrix          # region matrix on this level
    comp: np.ndarray          # composite number of each node on this level
    coords: np.ndarray        # (n, dim) composite coordinates on this level, -1 if none
    free: np.ndarray          # False for Dirichlet nodes (finest level only)


@dataclass
class HLevel:
    regions: list
    ncomp: int
    shape: tuple              # composite lattice extent per axis (x, y, z) on this level
    mask: int                 # Dirichlet faces
    dinv: list = None
    agg: list = None          # per region: coarse local index of each node, -1 if none
    Abar: np.ndarray = None   # coarsest level: composite matrix (dense)
    extra: dict = field(default_factory=dict)

    @property
    def nreg(self):
        return len(self.regions)

    # ---------------------------------------------------- regional vectors
    def mult(self):
        m = np.zeros(self.ncomp, dtype=np.int64)
        for R in self.regions:
            np.add.at(m, R.comp, 1)
        return m

    def to_composite_sum(self, v):
        s = np.zeros(self.ncomp)
        for R, vk in zip(self.regions, v):
            np.add.at(s, R.comp, vk)  # ascending region order
        return s

    def to_regional(self, x):
        return [x[R.comp].astype(np.float64) for R in self.regions]

    def interface_sum(self, v):
        return self.to_regional(self.to_composite_sum(v))

    def average(self, v):
        return self.to_regional(self.to_composite_sum(v) / self.mult())

    def to_composite_owner(self, v):
        out = np.zeros(self.ncomp)
        for R, vk in reversed(list(zip(self.regions, v))):
            out[R.comp] = vk
        return out

    def matvec(self, x):
        return self.interface_sum([R.A @ xk for R, xk in zip(self.regions, x)])

    def residual(self, b, u):
        z = self.matvec(u)
        return [bk - zk for bk, zk in zip(b, z)]

    def norm(self, v):
        return float(np.linalg.norm(self.to_composite_owner(v)))

    def composite_matrix(self):
        n = self.ncomp
        A = sp.csr_matrix((n, n))
        for R in self.regions:
            S = sp.csr_matrix((np.ones(R.comp.size), (R.comp, np.arange(R.comp.size))), shape=(n, R.comp.size))
            A = A + S @ R.A @ S.T
        return sp.csr_matrix(A)


# ------------------------------------------------------------------ level 0
def finest_level(lay: Layout, coefs) -> HLevel:
    """Region matrices of the finest level from the per-region stencils (scalar problems)."""
    assert lay.ndof == 1
    regions = []
    shape_xyz = lay.shape_xyz
    strides = np.cumprod((1,) + shape_xyz[:-1])
    for k in range(lay.nreg):
        A = sp.csr_matrix(assembly.stencil_to_csr(coefs[k], lay.dim))
        e, o = lay.extents[k], lay.origins[k]
        loc = np.indices(tuple(int(v) for v in reversed(e))).reshape(lay.dim, -1)[::-1].T  # (n, dim) x first
        g = loc + o
        comp = (g * strides).sum(axis=1)
        free = ~lay.dirichlet.reshape(-1)[comp]
        regions.append(HRegion(A, comp.astype(np.int64), g.astype(np.int64), free))
    return HLevel(regions, lay.n_composite, tuple(shape_xyz), lay.dirichlet_mask)


# -------------------------------------------------------------- aggregation
def coarse_point(g, shape, mask):
    """Nearest rate-3 coarse point of composite coordinates g (array (..., dim)), moved one
    coarse step inward where it would lie on a Dirichlet face."""
    c = 3 * np.floor_divide(g + 1, 3)
    for a in range(g.shape[-1]):
        if mask & (1 << (2 * a)):
            c[..., a] = np.where(c[..., a] == 0, 3, c[..., a])
        if mask & (1 << (2 * a + 1)):
            c[..., a] = np.where(c[..., a] == shape[a] - 1, shape[a] - 4, c[..., a])
    return c


def neighbours(R: HRegion):
    """Graph neighbours: free nodes coupled by a nonzero off-diagonal entry."""
    A = R.A.tocsr()
    out = []
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        nb = [int(j) for j, v in zip(cols, vals) if j != i and v != 0.0 and R.free[j]]
        out.append(sorted(set(nb)))
    return out


def aggregate_region(R: HRegion, unstructured: bool, interface: np.ndarray, shape, mask):
    """Aggregate id (arbitrary labels) of every node, -1 for Dirichlet nodes, and the coarse point
    of each label formed by the structured rule (None for the others)."""
    n = R.comp.size
    agg = np.full(n, -1, dtype=np.int64)
    points = {}   # label -> coarse point (tuple) for structured-rule aggregates
    label_of_point = {}

    def structured(i):
        cp = tuple(int(v) for v in coarse_point(R.coords[i], shape, mask))
        if cp not in label_of_point:
            label_of_point[cp] = len(points)
            points[len(points)] = cp
        agg[i] = label_of_point[cp]

    if not unstructured:  # every free node by the structured rule, labels in order of first sight
        idx = np.flatnonzero(R.free)
        cps = coarse_point(R.coords[idx], shape, mask)
        uniq, first, inv = np.unique(cps, axis=0, return_index=True, return_inverse=True)
        rank = np.empty(len(uniq), dtype=np.int64)
        rank[np.argsort(first)] = np.arange(len(uniq))
        agg[idx] = rank[inv.ravel()]
        for u, rk in zip(uniq, rank):
            points[int(rk)] = tuple(int(v) for v in u)
        return agg, points
    # stage I: interface nodes, structured rule
    for i in range(n):
        if R.free[i] and interface[i]:
            structured(i)
    nb = neighbours(R)
    nlab = len(points)
    # stage II: roots
    for i in range(n):
        if R.free[i] and agg[i] < 0 and all(agg[j] < 0 for j in nb[i]):
            agg[i] = nlab
            for j in nb[i]:
                agg[j] = nlab
            nlab += 1
    # stage III: joins, from the aggregates as they stand now
    snap = agg.copy()
    first = {}
    for i in range(n):
        if snap[i] >= 0 and snap[i] not in first:
            first[snap[i]] = i
    for i in range(n):
        if not R.free[i] or snap[i] >= 0:
            continue
        count = {}
        for j in nb[i]:
            if snap[j] >= 0:
                count[snap[j]] = count.get(snap[j], 0) + 1
        if count:
            best = max(count.values())
            agg[i] = min((first[a], a) for a, c in count.items() if c == best)[1]
    # stage IV: leftovers
    for i in range(n):
        if R.free[i] and agg[i] < 0:
            agg[i] = nlab
            for j in nb[i]:
                if agg[j] < 0:
                    agg[j] = nlab
            nlab += 1
    return agg, points


def coarsen(L: HLevel, kinds) -> tuple:
    """Aggregates of every region (coarse local numbers) and the next level (without operators)."""
    for s in L.shape:
        if (s - 1) % 3 or s < 7:
            raise ValueError("composite extent - 1 must be divisible by 3 and at least 6 on aggregated levels")
    mult = L.mult()
    aggs, cnodes = [], []
    for k, R in enumerate(L.regions):
        interface = mult[R.comp] >= 2
        lab, points = aggregate_region(R, bool(kinds[k]), interface, L.shape, L.mask)
        first = {}
        for i in range(lab.size):
            if lab[i] >= 0 and lab[i] not in first:
                first[lab[i]] = i
        order = sorted(first, key=lambda a: first[a])
        local = {a: c for c, a in enumerate(order)}
        aggs.append(np.array([local[a] if a >= 0 else -1 for a in lab], dtype=np.int64))
        coords = np.full((len(order), R.coords.shape[1]), -1, dtype=np.int64)
        for c, a in enumerate(order):
            if a in points:
                coords[c] = np.asarray(points[a]) // 3
        cnodes.append(coords)
    # coarse composite numbering: first sight, regions in order
    ids = {}
    regions = []
    for k, coords in enumerate(cnodes):
        comp = np.empty(len(coords), dtype=np.int64)
        for c, x in enumerate(coords):
            key = ("x",) + tuple(int(v) for v in x) if x[0] >= 0 else ("p", k, c)
            if key not in ids:
                ids[key] = len(ids)
            comp[c] = ids[key]
        regions.append(HRegion(None, comp, coords, np.ones(len(coords), dtype=bool)))
    shape = tuple((s - 1) // 3 + 1 for s in L.shape)
    return aggs, HLevel(regions, len(ids), shape, L.mask)


def region_prolongator(agg, nc):
    rows = np.flatnonzero(agg >= 0)
    return sp.csr_matrix((np.ones(rows.size), (rows, agg[rows])), shape=(agg.size, nc))


def setup(L0: HLevel, kinds, opt: HOptions):
    """Hierarchy of ``opt.nlevels`` levels below and including L0."""
    levels = [L0]
    L = L0
    for l in range(opt.nlevels):
        if l == opt.nlevels - 1:
            L.Abar = L.composite_matrix().toarray()
            break
        d = L.interface_sum([R.A.diagonal() for R in L.regions])
        L.dinv = [1.0 / dk for dk in d]
        aggs, C = coarsen(L, kinds)
        L.agg = aggs
        for k, R in enumerate(L.regions):
            P = region_prolongator(aggs[k], C.regions[k].comp.size)
            C.regions[k].A = sp.csr_matrix(P.T @ R.A @ P)
        levels.append(C)
        L = C
    return levels


# -------------------------------------------------------------- smoothing
def gs_sweep(L: HLevel, u, r, omega, backward=False):
    """Region-local Gauss-Seidel sweep (Algorithm 1), copies of interface nodes averaged."""
    delta = []
    cache = L.extra.setdefault("tri", {})
    for k, R in enumerate(L.regions):
        key = (k, backward, omega)
        if key not in cache:
            dg = 1.0 / L.dinv[k]
            cache[key] = sp.csr_matrix((sp.triu(R.A, 1) if backward else sp.tril(R.A, -1)) + sp.diags(dg / omega))
        delta.append(spla.spsolve_triangular(cache[key], r[k], lower=not backward))
    avg = L.average(delta)
    return [uk + dk for uk, dk in zip(u, avg)]


def smooth(L: HLevel, u, b, r, opt: HOptions):
    for i in range(opt.degree):
        if i:
            r = L.residual(b, u)
        if opt.smoother == "jacobi":
            u = [uk + opt.omega * dk * rk for uk, dk, rk in zip(u, L.dinv, r)]
        elif opt.smoother == "gs":
            u = gs_sweep(L, u, r, opt.omega)
        elif opt.smoother == "symgs":
            u = gs_sweep(L, u, r, opt.omega)
            u = gs_sweep(L, u, L.residual(b, u), opt.omega, backward=True)
        else:
            raise ValueError(opt.smoother)
    return u


def restrict(L: HLevel, C: HLevel, r):
    """Regional restriction (Section 3.3): divide by multiplicity, P^T per region, coarse
    interface sum."""
    m = L.mult()
    w = []
    for k, R in enumerate(L.regions):
        P = region_prolongator(L.agg[k], C.regions[k].comp.size)
        w.append(P.T @ (r[k] / m[R.comp]))
    return C.interface_sum(w)


def prolongate(L: HLevel, C: HLevel, ubar):
    return [region_prolongator(L.agg[k], C.regions[k].comp.size) @ ubar[k] for k in range(L.nreg)]


def coarse_solve(L: HLevel, w):
    return L.to_regional(np.linalg.solve(L.Abar, L.to_composite_owner(w)))


def cycle(levels, b, opt: HOptions, l=0):
    """V- (gamma 1) or W-cycle (gamma 2) with zero initial guess."""
    L = levels[l]
    if l == len(levels) - 1:
        return coarse_solve(L, b)
    u = smooth(L, [np.zeros_like(bk) for bk in b], b, b, opt)
    r = L.residual(b, u)
    C = levels[l + 1]
    w = restrict(L, C, r)
    ubar = cycle(levels, w, opt, l + 1)
    if opt.gamma == 2 and l + 1 < len(levels) - 1:
        rc = C.residual(w, ubar)
        ubar = [a + c for a, c in zip(ubar, cycle(levels, rc, opt, l + 1))]
    u = [uk + pk for uk, pk in zip(u, prolongate(L, C, ubar))]
    return smooth(L, u, b, L.residual(b, u), opt)


def stationary(levels, b, x0, opt: HOptions, rtol=1e-6, maxit=100):
    """MG as a solver: x <- x + cycle(b - A x) until ||r|| <= rtol ||r0||; returns (x, history)."""
    L = levels[0]
    x = [xk.copy() for xk in x0]
    r = L.residual(b, x)
    r0 = L.norm(r)
    hist = [1.0]
    while hist[-1] > rtol and len(hist) <= maxit:
        x = [xk + ck for xk, ck in zip(x, cycle(levels, r, opt))]
        r = L.residual(b, x)
        hist.append(L.norm(r) / r0)
    return x, hist


def pcg(levels, b, opt: HOptions, rtol=1e-6, maxit=100):
    """CG preconditioned by one cycle, x0 = 0, with the flexible coefficient
    beta = (z_new, r_new - r_old) / (z_old, r_old) (the region-local sweeps average the interface
    copies, so the cycle is not exactly a symmetric operator); composite inner products.
    Returns (x, history of ||r|| / ||b||)."""
    L = levels[0]

    def dot(a, c):
        return float(L.to_composite_owner(a) @ L.to_composite_owner(c))

    x = [np.zeros_like(bk) for bk in b]
    r = [bk.copy() for bk in b]
    bnorm = L.norm(b)
    hist = [1.0]
    z = cycle(levels, r, opt)
    p = [zk.copy() for zk in z]
    rz = dot(r, z)
    while len(hist) <= maxit:
        q = L.matvec(p)
        alpha = rz / dot(p, q)
        x = [xk + alpha * pk for xk, pk in zip(x, p)]
        r_old = r
        r = [rk - alpha * qk for rk, qk in zip(r, q)]
        hist.append(L.norm(r) / bnorm)
        if hist[-1] <= rtol:
            # accepted only if the true residual b - A x agrees; else CG continues from it
            rt = [bk - ak for bk, ak in zip(b, L.matvec(x))]
            if L.norm(rt) / bnorm <= rtol:
                break
            r = rt
        z = cycle(levels, r, opt)
        beta = dot(z, [a - c for a, c in zip(r, r_old)]) / rz
        rz = dot(r, z)
        p = [zk + beta * pk for zk, pk in zip(z, p)]
    return x, hist


# ------------------------------------------------------------ composite form
def composite_prolongator(L: HLevel, C: HLevel):
    """Composite P assembled from the region prolongators (each composite row from any copy;
    the Lemma on P makes the copies agree)."""
    rows, cols = [], []
    for k, R in enumerate(L.regions):
        sel = L.agg[k] >= 0
        rows.append(R.comp[sel])
        cols.append(C.regions[k].comp[L.agg[k][sel]])
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    key = np.unique(np.stack([rows, cols], axis=1), axis=0)
    return sp.csr_matrix((np.ones(len(key)), (key[:, 0], key[:, 1])), shape=(L.ncomp, C.ncomp))
