"""Plain composite multigrid (the standard two-level method of the paper's
Section 3 figure, applied recursively): sparse A, linear P, R = P^T,
Abar = R A P, Chebyshev or damped Jacobi smoothing with the composite
diagonal, or true lexicographic Gauss-Seidel, dense coarse solve, and preconditioned CG.

This is the textbook method the regional form must reproduce up to rounding
(Lemmas and Theorem of Section 3.1, Table 1 equivalence).  It uses the same
readings as ``regional`` (Chebyshev initialisation, eigenvalue interval,
counter-based power-method start vector, Dirichlet treatment).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import amg, assembly, rng, transfer
from .regional import Options
from .regions import Layout


@dataclass
class CLevel:
    lay: Layout
    A: sp.csr_matrix
    dinv: np.ndarray = None
    lam: float = None
    P: sp.csr_matrix = None
    amg: list = None  # coarsest level with the AMG coarse solver


def start_vector(lay: Layout, level: int, seed: int):
    v = rng.uniform_pm1(lay.n_composite, level, seed)
    v[assembly.dirichlet_dofs(lay)] = 0.0
    return v


def power_method(L: CLevel, x0, iters):
    x = x0 / np.linalg.norm(x0)
    lam = 0.0
    for _ in range(iters):
        y = L.dinv * (L.A @ x)
        lam = float(x @ y)
        x = y / np.linalg.norm(y)
    return lam


def setup(lay0: Layout, A0, opt: Options, lams=None):
    """Composite hierarchy; ``lams`` overrides the eigenvalue estimates when given."""
    levels = []
    lay, A = lay0, sp.csr_matrix(A0)
    for l in range(opt.nlevels):
        L = CLevel(lay, A)
        levels.append(L)
        if l == opt.nlevels - 1:
            if opt.coarse_amg:
                L.amg = amg.setup(A, ~lay.dirichlet.reshape(-1), opt.amg_coarse_size, opt.degree, opt.eig_ratio)
            break
        L.dinv = 1.0 / A.diagonal()
        if opt.smoother == "chebyshev":
            L.lam = lams[l] if lams is not None else power_method(L, start_vector(lay, l, opt.seed), opt.power_iters)
        coarse = lay.coarsen()
        L.P = transfer.composite_prolongator(lay, coarse)
        A = sp.csr_matrix(L.P.T @ A @ L.P)
        lay = coarse
    return levels


def chebyshev(L: CLevel, u, b, r, opt: Options):
    alpha = L.lam / opt.eig_ratio
    beta = opt.boost * L.lam
    theta = 0.5 * (alpha + beta)
    delta = 2.0 / (beta - alpha)
    rho = 1.0 / (theta * delta)
    d = L.dinv * r / theta
    u = u + d
    for _ in range(opt.degree - 1):
        r = b - L.A @ u
        rho_old = rho
        rho = 1.0 / (2.0 * theta * delta - rho_old)
        d = rho * rho_old * d + 2.0 * rho * delta * (L.dinv * r)
        u = u + d
    return u


def jacobi(L: CLevel, u, b, r, opt: Options):
    for i in range(opt.degree):
        if i:
            r = b - L.A @ u
        u = u + opt.jacobi_omega * L.dinv * r
    return u


def gauss_seidel(L: CLevel, u, b, r, opt: Options, backward=False):
    """True Gauss-Seidel on the composite matrix, ``degree`` sweeps in lexicographic order
    (reverse order when ``backward``): u += (D / omega + L)^-1 (b - A u), L the strictly lower
    triangle of A (upper, ``backward``)."""
    T = (sp.triu(L.A, 1) if backward else sp.tril(L.A, -1)) + sp.diags(L.A.diagonal() / opt.jacobi_omega)
    T = sp.csr_matrix(T)
    for i in range(opt.degree):
        if i:
            r = b - L.A @ u
        u = u + spla.spsolve_triangular(T, r, lower=not backward)
    return u


def smooth(L: CLevel, u, b, r, opt: Options, post=False):
    if opt.smoother == "chebyshev":
        return chebyshev(L, u, b, r, opt)
    if opt.smoother == "jacobi":
        return jacobi(L, u, b, r, opt)
    if opt.smoother in ("gs", "sgs"):
        return gauss_seidel(L, u, b, r, opt, backward=post and opt.smoother == "sgs")
    if opt.smoother == "symgs":
        for i in range(opt.degree):
            if i:
                r = b - L.A @ u
            u = gauss_seidel(L, u, b, r, Options(degree=1, jacobi_omega=opt.jacobi_omega))
            u = gauss_seidel(L, u, b, b - L.A @ u, Options(degree=1, jacobi_omega=opt.jacobi_omega), backward=True)
        return u
    raise ValueError(f"unknown smoother {opt.smoother!r}")


def vcycle(levels, b, opt: Options, l=0):
    L = levels[l]
    if l == len(levels) - 1:
        if L.amg is not None:
            return amg.vcycle(L.amg, b)
        return np.linalg.solve(L.A.toarray(), b)
    u = smooth(L, np.zeros_like(b), b, b, opt)
    r = b - L.A @ u
    bc = L.P.T @ r
    ubar = vcycle(levels, bc, opt, l + 1)
    if opt.gamma == 2 and l + 1 < len(levels) - 1:
        ubar = ubar + vcycle(levels, bc - levels[l + 1].A @ ubar, opt, l + 1)
    u = u + L.P @ ubar
    r = b - L.A @ u
    return smooth(L, u, b, r, opt, post=True)


def pcg(levels, b, opt: Options, rtol=1e-8, maxit=200):
    A = levels[0].A
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    z = vcycle(levels, r, opt)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= rtol:
            rt = b - A @ x  # accepted only if the true residual agrees (residual replacement)
            if np.linalg.norm(rt) / bnorm <= rtol:
                break
            r = rt
        z = vcycle(levels, r, opt)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, hist


def stationary(levels, b, x0, opt: Options, cycles: int):
    A = levels[0].A
    x = x0.copy()
    r = b - A @ x
    r0 = np.linalg.norm(r)
    hist = [1.0]
    for _ in range(cycles):
        x = x + vcycle(levels, r, opt)
        r = b - A @ x
        hist.append(np.linalg.norm(r) / r0)
    return x, hist
