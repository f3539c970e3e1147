"""Oracle pins of the nodal-block D~ of a system (block_diag; Section 3.2 smoother setup).

* The blocks are the ndof x ndof diagonal blocks of the composite matrix assembled independently
  (composite Q1 elasticity), which pins the copy sums at interfaces, edges and corners.
* Their diagonals are the point diagonal D~.
* On a block-diagonal operator (random SPD nodal blocks split unevenly over the copies of shared
  nodes) one Jacobi sweep with omega = 1 is the exact solve, compared with a dense solve.
* The power method with blocks gives exactly the Rayleigh quotient of the 10th iterate, evaluated
  from an eigendecomposition of L^-1 A L^-T (D = L L^T per node): the spectral closed form.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import assembly, regional, rng
from oracle.regions import Layout


def elasticity():
    """2x2x2 regions of 5^3 nodes (9^3 composite), Dirichlet on the x-, y-, z- faces, Young's
    moduli jumping by 10 between regions."""
    o, e = synth.tensor_layout([[5, 5]] * 3)
    lay = Layout(3, o, e, 0b010101, 3)
    youngs = [10.0 ** (k % 3) for k in range(lay.nreg)]
    coefs = regional.build_operator(lay, "elasticity", h=0.125, youngs=youngs, nu=0.3)
    A = regional.composite_operator(lay, "elasticity", h=0.125, youngs=youngs, nu=0.3)
    return lay, coefs, (A.toarray() if hasattr(A, "toarray") else np.asarray(A))


def composite_blocks(lay, blocks):
    """Composite (owner copy) form of consistent regional nodal blocks: (nodes, ndof, ndof)."""
    cols = [lay.to_composite_owner([b[..., :, j] for b in blocks]).reshape(-1, lay.ndof) for j in range(lay.ndof)]
    return np.stack(cols, axis=-1)


def test_blocks_are_the_composite_matrix_diagonal_blocks():
    lay, coefs, A = elasticity()
    D = composite_blocks(lay, regional.composite_block_diagonal(lay, coefs))
    nd = lay.ndof
    ref = np.stack([A[i * nd:(i + 1) * nd, i * nd:(i + 1) * nd] for i in range(D.shape[0])])
    free = ~lay.dirichlet.reshape(-1)
    assert free.sum() > 0 and (~free).sum() > 0
    np.testing.assert_allclose(D[free], ref[free], rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    # and their diagonals are the point diagonal
    pd = lay.to_composite_owner(regional.composite_diagonal(lay, coefs)).reshape(-1, nd)
    np.testing.assert_array_equal(np.einsum("naa->na", D), pd)


def test_block_jacobi_solves_a_block_diagonal_operator():
    w = synth.workload("c3_small")
    lay = Layout(w.dim, w.origins, w.extents, 0, 3)  # no Dirichlet nodes
    g = np.random.default_rng(5)
    ncomp = lay.n_composite // 3
    M = g.standard_normal((ncomp, 3, 3))
    Bc = M @ np.transpose(M, (0, 2, 1)) + 3.0 * np.eye(3)  # SPD composite blocks
    # split every node's block over its copies with uneven weights that sum to one
    share = lay.to_regional(np.zeros(lay.shape + (3,)))
    wts = [g.uniform(0.2, 1.0, s.shape[:-1]) for s in share]
    tot = lay.to_composite_sum([wk[..., None] * np.ones(3) for wk in wts]).reshape(-1, 3)[:, 0]
    coefs = []
    for k in range(lay.nreg):
        c = np.zeros((27,) + lay.region_shape(k) + (3, 3))
        comp = lay.to_regional(np.arange(ncomp, dtype=np.float64).reshape(lay.shape)[..., None] * np.ones(3))[k]
        idx = comp[..., 0].astype(np.int64)
        c[assembly.center(3)] = Bc[idx] * (wts[k] / tot[idx])[..., None, None]
        coefs.append(c)
    L = regional.Level(lay, coefs)
    L.dblk = [np.linalg.inv(B) for B in regional.composite_block_diagonal(lay, coefs)]
    b = g.standard_normal(lay.shape + (3,))
    br = lay.to_regional(b)
    opt = regional.Options(degree=1, jacobi_omega=1.0, smoother="jacobi")
    u = regional.jacobi(L, lay.zeros_regional(), br, br, opt)
    want = np.linalg.solve(Bc, b.reshape(-1, 3)[..., None])[..., 0]
    np.testing.assert_allclose(lay.to_composite_owner(u).reshape(-1, 3), want, rtol=1e-12, atol=1e-12)


def test_block_power_method_equals_spectral_rayleigh_quotient():
    lay, coefs, A = elasticity()
    opt = regional.Options(nlevels=2, power_iters=10, block_diag=True)
    lv = regional.setup(lay, coefs, opt)
    nd = lay.ndof
    free = np.repeat(~lay.dirichlet.reshape(-1), nd)  # Dirichlet nodes fix all their dofs
    Af = A[np.ix_(free, free)]
    # block-diagonal D of the free dofs
    D = np.zeros_like(Af)
    node = np.repeat(np.arange(A.shape[0] // nd), nd)[free]
    same = node[:, None] == node[None, :]
    D[same] = Af[same]
    Lc = np.linalg.cholesky(D)
    S = sla.solve_triangular(Lc, sla.solve_triangular(Lc, Af, lower=True).T, lower=True).T
    mu, V = np.linalg.eigh(0.5 * (S + S.T))
    x0 = rng.uniform_pm1(lay.n_composite, 0, opt.seed)[free]
    # M = D^-1 A = L^-T S L^T, so M^9 x0 = L^-T V mu^9 V^T L^T x0
    c = V.T @ (Lc.T @ x0)
    x9 = sla.solve_triangular(Lc.T, V @ (mu ** 9 * c), lower=False)
    x9 /= np.linalg.norm(x9)
    Mx = sla.solve_triangular(Lc.T, V @ (mu * (V.T @ (Lc.T @ x9))), lower=False)
    lam = float(x9 @ Mx)
    assert abs(lv[0].lam - lam) <= 1e-11 * lam, (lv[0].lam, lam)


def test_block_diag_needs_a_system_and_a_point_smoother():
    w = synth.workload("c2_small")
    lay = Layout(w.dim, w.origins, w.extents, w.dirichlet_mask, 1)
    coefs = regional.build_operator(lay, "laplace", h=w.h)
    with pytest.raises(ValueError):
        regional.setup(lay, coefs, regional.Options(nlevels=2, block_diag=True))
