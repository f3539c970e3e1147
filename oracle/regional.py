"""Regional multigrid hierarchy, V-cycle and preconditioned CG, written out in the
regional form (paper Section 3.2 setup, Section 3.3 cycle, Section 3.4
Chebyshev smoother, Section 3.5 direct coarse solver, Section 3.6 summary
figure of the regional two-level method, applied recursively).

Readings of points the paper leaves open:

* Chebyshev (Algorithm 2): the first correction is d = D~^-1 r / theta (the
  extra delta factor in the printed initialisation is dropped; it is
  inconsistent with rho = 1/(theta delta)); degree K means K corrections and
  K-1 residual updates inside the smoother.
* D~ of a system (Section 3.2 smoother setup speaks of the diagonal): the point
  diagonal by default; with ``block_diag`` the ndof x ndof nodal blocks of
  [[A]]'s centre stencil summed over the copies (Psi^T Psi column by column) and
  inverted per node, used wherever D~^-1 enters (power method, Chebyshev,
  Jacobi).
* Eigenvalue interval [lambda/eta, kappa*lambda] with lambda the largest
  eigenvalue of D~^-1 A, estimated by power iterations from the counter-based
  start vector of ``rng``; eta = 20, kappa = 1.1, 10 iterations by default.
* Coarse composite operator Abar = Psi-bar [[Abar]] Psi-bar^T (the printed
  formula omits the right factor), solved densely.
* Pre- and post-smoothing each apply one degree-K Chebyshev polynomial.
* Region-local Gauss-Seidel (Algorithm 1): after a sweep the copies of an
  interface node carry different corrections (each region saw only its own
  updates); they are replaced by their average, so that u stays the regional
  form of a composite vector.  The "gs" smoother sweeps forward before and after
  the coarse correction; "sgs" sweeps backward (reverse lexicographic order)
  after it; "symgs" (symmetric Gauss-Seidel) does a forward then a backward
  sweep per iteration, before and after.  The damping omega of Algorithm 1 is
  ``jacobi_omega``.
* CG: textbook Hestenes-Stiefel with x0 = 0, preconditioner z = V(r, 0),
  stopping when the recursive residual ||r||/||b|| <= rtol and the true residual
  ||b - A x||/||b|| agrees (else r is replaced by the true residual and CG goes
  on).  Inner products are composite ones: every composite dof counted once.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import amg, assembly, rng, transfer
from .regions import Layout


# ------------------------------------------------------------ vector helpers
def lin(a, x, b=None, y=None):
    """a*x + b*y on regional (list) vectors."""
    if y is None:
        return [a * xi for xi in x]
    return [a * xi + b * yi for xi, yi in zip(x, y)]


def mul(x, y):
    return [xi * yi for xi, yi in zip(x, y)]


@dataclass
class Level:
    lay: Layout
    coefs: list
    dinv: list = None
    lam: float = None
    P: list = None  # region prolongators to the next level
    Abar: np.ndarray = None  # coarsest composite operator (dense)
    amg: list = None  # coarsest level with the AMG coarse solver: its levels (amg.setup)
    dblk: list = None  # block_diag: per region the inverse nodal blocks of D~, shape (..., ndof, ndof)
    extra: dict = field(default_factory=dict)

    def apply_dinv(self, r):
        """D~^-1 r: the point diagonal's reciprocal, or the inverse nodal blocks (block_diag)."""
        if self.dblk is None:
            return mul(self.dinv, r)
        return [np.einsum("...ab,...b->...a", Dk, rk) for Dk, rk in zip(self.dblk, r)]

    def matvec(self, x):
        """Psi^T Psi [[A]] [[x]]: region-local stencil products, then interface sum (RegMatVec)."""
        lay = self.lay
        z = [assembly.apply_stencil(self.coefs[k], x[k], lay.dim, lay.ndof) for k in range(lay.nreg)]
        return lay.interface_sum(z)

    def residual(self, b, u):
        return lin(1.0, b, -1.0, self.matvec(u))


@dataclass
class Options:
    nlevels: int = 3
    degree: int = 2
    eig_ratio: float = 20.0
    boost: float = 1.1
    power_iters: int = 10
    seed: int = 0
    smoother: str = "chebyshev"  # or "jacobi", "gs", "sgs", "symgs"
    gamma: int = 1  # coarse-level cycles per visit: 1 V-cycle, 2 W-cycle
    jacobi_omega: float = 0.6
    block_diag: bool = False  # systems (ndof > 1): D~ of nodal blocks instead of the point diagonal
    coarse_amg: bool = False  # coarse solve: one AMG V-cycle on Abar instead of a direct solve
    amg_coarse_size: int = 2000  # the AMG's directly solved level has at most this many rows


def composite_diagonal(lay: Layout, coefs):
    """D~ = Psi^T Psi diag([[A]]) (Section 3.2 smoother setup)."""
    d = [assembly.diagonal(coefs[k], lay.dim, lay.ndof) for k in range(lay.nreg)]
    return lay.interface_sum(d)


def composite_block_diagonal(lay: Layout, coefs):
    """Nodal-block D~ of a system (ndof > 1): every node's ndof x ndof centre block of [[A]] summed
    over the node's copies (Psi^T Psi applied column by column); shape (..., ndof, ndof) per region."""
    cen = [coefs[k][assembly.center(lay.dim)] for k in range(lay.nreg)]  # (..., a, b)
    cols = [lay.interface_sum([c[..., :, j] for c in cen]) for j in range(lay.ndof)]
    return [np.stack([cols[j][k] for j in range(lay.ndof)], axis=-1) for k in range(lay.nreg)]


def start_vector(lay: Layout, level: int, seed: int):
    """Power-method start vector: counter-based uniform values, zero on Dirichlet dofs."""
    v = rng.uniform_pm1(lay.n_composite, level, seed)
    shp = lay.shape + ((lay.ndof,) if lay.ndof > 1 else ())
    v = v.reshape(shp)
    v[lay.dirichlet] = 0.0
    return lay.to_regional(v)


def power_method(L: Level, x0, iters: int):
    """Largest eigenvalue of D~^-1 Psi^T Psi [[A]] by power iteration with a Rayleigh quotient.

    x <- x0/||x0||; repeat: y = D~^-1 A x, lambda = (x, y), x = y/||y||.
    """
    lay = L.lay
    x = lin(1.0 / lay.norm(x0), x0)
    lam = 0.0
    for _ in range(iters):
        y = L.apply_dinv(L.matvec(x))
        lam = lay.dot(x, y)
        x = lin(1.0 / lay.norm(y), y)
    return lam


def finest_coordinates(levels):
    """Coordinates (n, 3) of the last level's composite nodes (x fastest) on the finest lattice,
    relative to the finest lattice's centre: each coarse lattice line is a line of the level above
    (Layout.fine_positions), followed up to level 0."""
    lay = levels[-1].lay
    axes = []
    for d in range(lay.dim):
        p = np.arange(int(lay.shape_xyz[d]))
        for L in reversed(levels[1:]):
            p = np.asarray(L.lay.fine_positions[d])[p]
        n0 = int(levels[0].lay.shape_xyz[d])
        axes.append(p - 0.5 * (n0 - 1))
    grids = np.meshgrid(*axes[::-1], indexing="ij")  # (z, y, x) order, x fastest
    return np.stack([g.reshape(-1) for g in grids[::-1]], axis=1)


def coarse_composite(lay: Layout, coefs):
    """Abar = Psi-bar [[Abar]] Psi-bar^T as a dense matrix."""
    return assembly.assemble_from_regions(lay, coefs).toarray()


def setup(lay0: Layout, coefs0, opt: Options, P0=None):
    """Regional hierarchy; ``P0`` optionally replaces the finest level's region prolongators."""
    levels = []
    lay, coefs = lay0, coefs0
    for l in range(opt.nlevels):
        L = Level(lay, coefs)
        levels.append(L)
        if l == opt.nlevels - 1:
            if opt.coarse_amg:  # Section 3.5: an AMG V-cycle on Abar replaces the direct solver
                Ab = assembly.assemble_from_regions(lay, coefs)
                free = ~lay.dirichlet.reshape(-1)
                if lay.ndof == 1:
                    L.amg = amg.setup(Ab, free, opt.amg_coarse_size, opt.degree, opt.eig_ratio)
                elif lay.ndof == 3 and lay.dim == 3:
                    # the near-null space from the region hierarchy: rigid-body modes at the
                    # coarsest nodes' positions on the finest lattice (coarse points are fine nodes)
                    B = amg.rigid_body_modes(finest_coordinates(levels))
                    nn = free.size
                    L.amg = amg.setup(Ab, np.repeat(free, 3), opt.amg_coarse_size, opt.degree, opt.eig_ratio,
                                      nodes=np.arange(0, 3 * nn + 1, 3), B=B)
                else:
                    raise ValueError("the AMG coarse solver handles scalar problems and 3D elasticity")
            else:
                L.Abar = coarse_composite(lay, coefs)
            break
        L.dinv = [1.0 / d for d in composite_diagonal(lay, coefs)]
        if opt.block_diag:
            if lay.ndof == 1 or opt.smoother not in ("chebyshev", "jacobi"):
                raise ValueError("nodal-block D~ needs a system (ndof > 1) and the Chebyshev or Jacobi smoother")
            L.dblk = [np.linalg.inv(B) for B in composite_block_diagonal(lay, coefs)]
        if opt.smoother == "chebyshev":
            L.lam = power_method(L, start_vector(lay, l, opt.seed), opt.power_iters)
        coarse = lay.coarsen()
        if l == 0 and P0 is not None:
            L.P = list(P0)
        else:
            L.P = [transfer.region_prolongator(lay, coarse, k) for k in range(lay.nreg)]
        ccoefs = []
        for k in range(lay.nreg):
            Ak = assembly.stencil_to_csr(coefs[k], lay.dim, lay.ndof)
            Ac = L.P[k].T @ Ak @ L.P[k]  # regional Galerkin product, per region
            ccoefs.append(assembly.csr_to_stencil(Ac, coarse.region_shape(k), lay.dim, lay.ndof))
        lay, coefs = coarse, ccoefs
    return levels


def chebyshev(L: Level, u, b, r, opt: Options):
    """Degree-K Chebyshev smoothing (Algorithm 2, reading above); r = b - A u on entry."""
    alpha = L.lam / opt.eig_ratio
    beta = opt.boost * L.lam
    theta = 0.5 * (alpha + beta)
    delta = 2.0 / (beta - alpha)
    rho = 1.0 / (theta * delta)
    d = lin(1.0 / theta, L.apply_dinv(r))
    u = lin(1.0, u, 1.0, d)
    for _ in range(opt.degree - 1):
        r = L.residual(b, u)
        rho_old = rho
        rho = 1.0 / (2.0 * theta * delta - rho_old)
        d = lin(rho * rho_old, d, 2.0 * rho * delta, L.apply_dinv(r))
        u = lin(1.0, u, 1.0, d)
    return u


def jacobi(L: Level, u, b, r, opt: Options):
    """Damped Jacobi sweeps u += omega D~^-1 r (Section 3.4), ``degree`` sweeps."""
    for i in range(opt.degree):
        if i:
            r = L.residual(b, u)
        u = lin(1.0, u, opt.jacobi_omega, L.apply_dinv(r))
    return u


def region_matrix(L: Level, k: int):
    """Region k's matrix [[A]]_k in region-local lexicographic order (x fastest, dof fastest)."""
    cache = L.extra.setdefault("csr", {})
    if k not in cache:
        cache[k] = sp.csr_matrix(assembly.stencil_to_csr(L.coefs[k], L.lay.dim, L.lay.ndof))
    return cache[k]


def gs_sweep(L: Level, u, r, omega, backward=False):
    """One region-local Gauss-Seidel sweep (Algorithm 1) from the composite residual r = b - A u.

    In every region k, visiting its dofs in lexicographic order, r_i -= sum_j A^(k)_ij delta_j over
    the dofs already visited and delta_i = omega r_i / d~_i.  Unrolled, that is the triangular solve
    (D~_k / omega + L_k) delta_k = r_k with L_k the strictly lower triangle of [[A]]_k (upper
    triangle, ``backward``).  The copies' corrections are averaged (reading in the module header).
    """
    lay = L.lay
    delta = []
    for k in range(lay.nreg):
        A = region_matrix(L, k)
        dg = 1.0 / L.dinv[k].reshape(-1)
        T = (sp.triu(A, 1) if backward else sp.tril(A, -1)) + sp.diags(dg / omega)
        dk = spla.spsolve_triangular(sp.csr_matrix(T), r[k].reshape(-1), lower=not backward)
        delta.append(dk.reshape(r[k].shape))
    return lin(1.0, u, 1.0, lay.to_regional(lay.to_composite_avg(delta)))


def gauss_seidel(L: Level, u, b, r, opt: Options, backward=False):
    """``degree`` region-local Gauss-Seidel sweeps; r = b - A u on entry; the composite residual
    is recomputed before every further sweep (its interface sum is the sweep's only
    communication)."""
    for i in range(opt.degree):
        if i:
            r = L.residual(b, u)
        u = gs_sweep(L, u, r, opt.jacobi_omega, backward)
    return u


def symmetric_gauss_seidel(L: Level, u, b, r, opt: Options):
    """``degree`` symmetric Gauss-Seidel iterations: each a forward sweep then a backward sweep,
    each sweep from a fresh composite residual."""
    for i in range(opt.degree):
        if i:
            r = L.residual(b, u)
        u = gs_sweep(L, u, r, opt.jacobi_omega, backward=False)
        u = gs_sweep(L, u, L.residual(b, u), opt.jacobi_omega, backward=True)
    return u


def smooth(L, u, b, r, opt, post=False):
    if opt.smoother == "chebyshev":
        return chebyshev(L, u, b, r, opt)
    if opt.smoother == "jacobi":
        return jacobi(L, u, b, r, opt)
    if opt.smoother in ("gs", "sgs"):
        return gauss_seidel(L, u, b, r, opt, backward=post and opt.smoother == "sgs")
    if opt.smoother == "symgs":
        return symmetric_gauss_seidel(L, u, b, r, opt)
    raise ValueError(f"unknown smoother {opt.smoother!r}")


def coarse_solve(L: Level, w):
    lay = L.lay
    wbar = lay.to_composite_owner(w).reshape(-1)
    ubar = amg.vcycle(L.amg, wbar) if L.amg is not None else np.linalg.solve(L.Abar, wbar)
    shp = lay.shape + ((lay.ndof,) if lay.ndof > 1 else ())
    return lay.to_regional(ubar.reshape(shp))


def vcycle(levels, b, opt: Options, l: int = 0):
    """z = V_l(b) with zero initial guess (Section 3.6 figure, recursive); with gamma = 2 every
    level above the coarsest is visited twice per visit of the level above (W-cycle)."""
    L = levels[l]
    if l == len(levels) - 1:
        return coarse_solve(L, b)
    u0 = L.lay.zeros_regional()
    u = smooth(L, u0, b, b, opt)  # u0 = 0: residual is b
    r = L.residual(b, u)
    C = levels[l + 1]
    w = transfer.regional_restrict(L.lay, C.lay, L.P, r)
    ubar = vcycle(levels, w, opt, l + 1)
    if opt.gamma == 2 and l + 1 < len(levels) - 1:  # W-cycle: a second coarse cycle on its residual
        ubar = lin(1.0, ubar, 1.0, vcycle(levels, C.residual(w, ubar), opt, l + 1))
    u = lin(1.0, u, 1.0, transfer.regional_prolongate(L.lay, C.lay, L.P, ubar))
    r = L.residual(b, u)
    return smooth(L, u, b, r, opt, post=True)


@dataclass
class SolveResult:
    x: list
    iterations: int
    history: list
    true_relres: float
    converged: bool


def pcg(levels, b, opt: Options, rtol=1e-8, maxit=200, precondition=True):
    """Preconditioned CG on the regional system (textbook form, reading above)."""
    L = levels[0]
    lay = L.lay
    x = lay.zeros_regional()
    r = [bi.copy() for bi in b]
    bnorm = lay.norm(b)
    hist = [1.0]
    if bnorm == 0.0:
        return SolveResult(x, 0, hist, 0.0, True)
    z = vcycle(levels, r, opt) if precondition else [ri.copy() for ri in r]
    p = [zi.copy() for zi in z]
    rz = lay.dot(r, z)
    it = 0
    converged = False
    while it < maxit:
        q = L.matvec(p)
        alpha = rz / lay.dot(p, q)
        x = lin(1.0, x, alpha, p)
        r = lin(1.0, r, -alpha, q)
        it += 1
        rel = lay.norm(r) / bnorm
        hist.append(rel)
        if rel <= rtol:
            # the tolerance is on the relative residual of the system, so the recursively
            # updated residual is checked against b - A x before the solve ends; where rounding
            # has separated them, CG goes on from the true residual (residual replacement)
            rt = L.residual(b, x)
            if lay.norm(rt) / bnorm <= rtol:
                converged = True
                break
            r = rt
        z = vcycle(levels, r, opt) if precondition else [ri.copy() for ri in r]
        rz_new = lay.dot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = lin(1.0, z, beta, p)
    true = lay.norm(L.residual(b, x)) / bnorm
    return SolveResult(x, it, hist, true, converged)


def stationary(levels, b, x0, opt: Options, cycles: int):
    """MG as a solver: x <- x + V(b - A x); returns iterates' relative residuals."""
    L = levels[0]
    lay = L.lay
    x = [xi.copy() for xi in x0]
    r = L.residual(b, x)
    r0 = lay.norm(r)
    hist = [1.0]
    for _ in range(cycles):
        x = lin(1.0, x, 1.0, vcycle(levels, r, opt))
        r = L.residual(b, x)
        hist.append(lay.norm(r) / r0)
    return x, hist


def build_operator(lay: Layout, pde, h=1.0, elem_coef=None, youngs=None, nu=0.3):
    """Finest-level region matrices for the model problems."""
    if pde == "fd5":
        return assembly.regional_fd5(lay)
    if pde == "fd7":
        return assembly.split_composite(lay, assembly.composite_fd7(lay))
    return assembly.regional_q1(lay, pde, h=h, elem_coef=elem_coef, youngs=youngs, nu=nu)


def composite_operator(lay: Layout, pde, h=1.0, elem_coef=None, youngs=None, nu=0.3):
    if pde == "fd5":
        return assembly.composite_fd5(lay)
    if pde == "fd7":
        return assembly.composite_fd7(lay)
    return assembly.composite_q1(lay, pde, h=h, elem_coef=elem_coef, youngs=youngs, nu=nu)
