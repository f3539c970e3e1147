"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Every check here uses something other than the oracle itself: explicit boolean
matrices, an independent composite assembly, closed-form stencils, textbook
polynomial identities, dense eigen-solves and dense direct solves.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import assembly, composite, fem, regional, rng, transfer
from oracle.regions import Layout


def layout_of(name, mask=None, ndof=None):
    w = synth.workload(name)
    return w, Layout(w.dim, w.origins, w.extents, w.dirichlet_mask if mask is None else mask,
                     w.ndof if ndof is None else ndof)


def tiny_layouts():
    # 2x2 regions of 4^2 and 7^2 nodes, 2x2x2 regions of 4^3, and an uneven 3x2 tensor layout
    out = []
    for dim, slabs in ((2, [[4, 4], [4, 4]]), (2, [[7, 7], [7, 7]]), (3, [[4, 4]] * 3),
                       (2, [[4, 7, 4], [7, 4]])):
        o, e = synth.tensor_layout(slabs)
        out.append(Layout(dim, o, e, (1 << 2 * dim) - 1))
    return out


# --------------------------------------------------------------------- Psi
@pytest.mark.parametrize("lay", tiny_layouts())
def test_psi_identities(lay):
    """Properties of Psi listed in Section 3.1, checked against the explicit boolean matrix."""
    Psi = lay.psi_matrix()
    assert Psi.shape == (lay.n_composite, lay.n_regional)
    assert np.all(np.asarray(Psi.sum(axis=0)).ravel() == 1)  # one nonzero per column
    PPt = (Psi @ Psi.T).toarray()
    assert np.array_equal(PPt, np.diag(lay.mult.reshape(-1).astype(float)))  # exact integers
    rng_ = np.random.default_rng(1)
    v = rng_.standard_normal(lay.n_regional)
    reg = lay.unflatten(v)
    np.testing.assert_allclose(lay.to_composite_sum(reg).reshape(-1), Psi @ v, rtol=0, atol=1e-14)
    np.testing.assert_allclose(lay.flatten(lay.interface_sum(reg)), Psi.T @ (Psi @ v), rtol=0, atol=1e-14)
    avg = sp.diags(1.0 / PPt.diagonal()) @ (Psi @ v)
    np.testing.assert_allclose(lay.to_composite_avg(reg).reshape(-1), avg, rtol=0, atol=1e-14)
    u = rng_.standard_normal(lay.n_composite)
    np.testing.assert_array_equal(lay.flatten(lay.to_regional(u.reshape(lay.shape))), Psi.T @ u)
    # partition Psi = [Psi_1 ... Psi_m]
    blocks = sp.hstack([lay.psi_block(k) for k in range(lay.nreg)]).tocsr()
    assert (blocks != Psi).nnz == 0
    # Psi_k^T S Psi_k extracts region k's submatrix; Psi_k Psi_k^T filters region k's dofs
    k = lay.nreg - 1
    Pk = lay.psi_block(k)
    filt = (Pk @ Pk.T).toarray()
    inbox = np.zeros(lay.shape, dtype=bool)
    inbox[lay.box(k)] = True
    assert np.array_equal(filt, np.diag(inbox.reshape(-1).astype(float)))


@pytest.mark.parametrize("lay", tiny_layouts())
def test_multiplicities_and_owner(lay):
    # 3D tensor layouts: faces 2, edges 4, corners 8 (Section 4)
    m = lay.mult
    assert set(np.unique(m)) <= {1, 2, 4, 8}
    assert np.all(lay.owner >= 0)
    for k in range(lay.nreg):
        own = lay.owner[lay.box(k)]
        assert np.all(own <= k)


def test_dot_counts_each_composite_dof_once():
    lay = tiny_layouts()[2]
    rng_ = np.random.default_rng(3)
    a = rng_.standard_normal(lay.shape)
    b = rng_.standard_normal(lay.shape)
    assert abs(lay.dot(lay.to_regional(a), lay.to_regional(b)) - float((a * b).sum())) < 1e-12


def test_layout_rejects_overlap_and_gaps():
    with pytest.raises(ValueError):
        Layout(2, [[0, 0], [2, 0]], [[4, 4], [4, 4]])  # overlapping cells
    with pytest.raises(ValueError):
        Layout(2, [[0, 0], [4, 0]], [[4, 4], [4, 4]])  # gap between boxes


# ------------------------------------------------------- element matrices
def test_q1_laplace_closed_form():
    """Trilinear stiffness = h * sum_d K1(d) (x) M1 (x) M1 with the 1D stiffness and mass matrices."""
    h = 0.37
    K = fem.q1_laplace(h)
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    m1 = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    ref = np.zeros((8, 8))
    for a, ca in enumerate(fem.CORNERS3):
        for b, cb in enumerate(fem.CORNERS3):
            ref[a, b] = h * sum(
                k1[ca[d], cb[d]] * np.prod([m1[ca[e], cb[e]] for e in range(3) if e != d]) for d in range(3))
    np.testing.assert_allclose(K, ref, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-14)


def test_q1_interior_stencil():
    """Assembled interior Q1 Laplacian stencil: h*(8/3 center, 0 face, -1/6 edge, -1/12 corner)."""
    w, lay = layout_of("c2_small")
    coefs = assembly.regional_q1(lay, "laplace", h=w.h)
    A = assembly.assemble_from_regions(lay, coefs)
    node = np.arange(lay.n_composite).reshape(lay.shape)
    i = node[4, 5, 6]
    for s, off in enumerate(assembly.offsets(3)):
        nz = sum(abs(o) for o in off)
        expect = {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[nz] * w.h
        j = node[4 + off[2], 5 + off[1], 6 + off[0]]
        assert abs(A[i, j] - expect) < 1e-15


def test_elasticity_rigid_body_modes_and_patch():
    E, nu, h = 2.3, 0.3, 0.5
    K = fem.q1_elasticity(E, nu, h)
    np.testing.assert_allclose(K, K.T, atol=1e-12)
    X = np.array(fem.CORNERS3, dtype=float) * h
    modes = []
    for i in range(3):
        t = np.zeros((8, 3))
        t[:, i] = 1.0
        modes.append(t.reshape(-1))
    for (i, j) in ((0, 1), (1, 2), (0, 2)):
        r = np.zeros((8, 3))
        r[:, i] = -X[:, j]
        r[:, j] = X[:, i]
        modes.append(r.reshape(-1))
    for m in modes:
        assert np.abs(K @ m).max() < 1e-12
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-10) == 6 and ev.min() > -1e-12
    # patch test: a uniform strain field stores energy volume * (lam tr(e)^2 + 2 mu e:e) / 2
    eps = np.array([[0.3, 0.1, -0.2], [0.1, -0.5, 0.05], [-0.2, 0.05, 0.7]])
    u = (X @ eps.T).reshape(-1)
    lam, mu = fem.lame(E, nu)
    energy = 0.5 * h ** 3 * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    assert abs(0.5 * u @ K @ u - energy) < 1e-12 * max(1.0, energy)


def test_region_elasticity_nullspace():
    """Each region's pure-Neumann elasticity matrix annihilates the six rigid-body modes."""
    w, lay = layout_of("c3_small", mask=0)
    youngs = synth.region_youngs_moduli(w)
    coefs = assembly.regional_q1(lay, "elasticity", h=w.h, youngs=youngs, nu=w.nu)
    k = 0
    shp = lay.region_shape(k)
    zz, yy, xx = np.meshgrid(*[np.arange(n) * w.h for n in shp], indexing="ij")
    X = [xx, yy, zz]
    for mode in range(6):
        v = np.zeros(shp + (3,))
        if mode < 3:
            v[..., mode] = 1.0
        else:
            i, j = ((0, 1), (1, 2), (0, 2))[mode - 3]
            v[..., i] = -X[j]
            v[..., j] = X[i]
        y = assembly.apply_stencil(coefs[k], v, 3, 3)
        assert np.abs(y).max() < 1e-10


# ---------------------------------------------------------------- splitting
@pytest.mark.parametrize("name", ["c1_small", "c2_small", "c3_small", "c5_small", "c4_small"])
def test_split_sums_to_composite(name):
    """eq. (extraction sum) and both restrictions, against an independent composite assembly."""
    w, lay = layout_of(name)
    youngs = synth.region_youngs_moduli(w) if w.pde == "elasticity" else None
    ec = synth.jump_coefficients(w) if w.pde == "diffusion" else None
    coefs = regional.build_operator(lay, w.pde, h=w.h, elem_coef=ec, youngs=youngs, nu=w.nu)
    A = regional.composite_operator(lay, w.pde, h=w.h, elem_coef=ec, youngs=youngs, nu=w.nu)
    Ar = assembly.assemble_from_regions(lay, coefs)
    scale = abs(A).max()
    assert abs(Ar - A).max() <= 1e-14 * scale
    pattern = (abs(A) > 0).astype(int)
    for k in range(lay.nreg):
        Pk = lay.psi_block(k)
        Ak = Pk @ assembly.stencil_to_csr(coefs[k], lay.dim, lay.ndof) @ Pk.T
        # A^(k)_ij != 0 => A_ij != 0 (entries of rounding size, from cancelling element sums, ignored)
        nz = (abs(Ak) > 1e-12 * scale).astype(int)
        assert (nz - nz.multiply(pattern)).nnz == 0


def test_fd5_split_rule():
    """Section 4 split: off-diagonals over q regions; diagonals give region row sums z_i/mult_i."""
    w, lay = layout_of("c1_small")
    A = assembly.composite_fd5(lay)
    coefs = assembly.regional_fd5(lay)
    z = (A @ np.ones(A.shape[0])).reshape(lay.shape)
    for k in range(lay.nreg):
        rowsum = coefs[k].sum(axis=0)
        np.testing.assert_allclose(rowsum, z[lay.box(k)] / lay.mult[lay.box(k)], atol=1e-15)
    # an interface edge shared by two regions carries -1/2 in each
    o = lay.origins[1]
    c0 = coefs[0]
    # node on the shared vertical interface of regions 0 and 1, coupling along the interface (dy = +1)
    x_if = int(lay.extents[0][0] - 1)
    assert c0[7][3, x_if] == -0.5
    assert c0[5][3, x_if - 1] == -1.0  # interior edge unchanged
    assert o[0] == x_if


# ------------------------------------------------------------ transfers
@pytest.mark.parametrize("name", ["c1_small", "c2_small", "c3_small", "c4_small"])
def test_transfer_lemmas(name):
    """Lemma P: P^(r) Psibar^T = Psi^T P.  Lemma R: Psibar R^(r) = R Psi (Section 3.1)."""
    w, lay = layout_of(name)
    coarse = lay.coarsen()
    P = transfer.composite_prolongator(lay, coarse)
    Pr = sp.block_diag([transfer.region_prolongator(lay, coarse, k) for k in range(lay.nreg)]).tocsr()
    Psi, Psib = lay.psi_matrix(), coarse.psi_matrix()
    assert abs(Pr @ Psib.T - Psi.T @ P).max() == 0.0
    assert abs(Psib @ Pr.T - P.T @ Psi).max() == 0.0


def test_prolongation_reproduces_linear_functions():
    """Linear interpolation is exact for (multi)linear functions (no Dirichlet rows)."""
    o, e = synth.tensor_layout([[10, 19], [10, 10], [19]])
    lay = Layout(3, o, e, 0)
    coarse = lay.coarsen()
    P = transfer.composite_prolongator(lay, coarse)
    zf, yf, xf = np.indices(lay.shape).astype(float)
    zc, yc, xc = np.indices(coarse.shape).astype(float) * 3.0
    f = lambda x, y, z: 0.3 + 1.5 * x - 0.7 * y + 2.1 * z + 0.05 * x * y * z  # noqa: E731
    np.testing.assert_allclose(P @ f(xc, yc, zc).reshape(-1), f(xf, yf, zf).reshape(-1), rtol=1e-13, atol=1e-12)


def test_regional_restriction_formula():
    """Psibar^T Psibar R^(r) [[Psi Psi^T]]^-1 Psi^T r = Psibar^T R r (Section 3.3)."""
    w, lay = layout_of("c2_small")
    coarse = lay.coarsen()
    P = transfer.composite_prolongator(lay, coarse)
    Pk = [transfer.region_prolongator(lay, coarse, k) for k in range(lay.nreg)]
    r = np.random.default_rng(5).standard_normal(lay.shape)
    w_reg = transfer.regional_restrict(lay, coarse, Pk, lay.to_regional(r))
    w_comp = (P.T @ r.reshape(-1)).reshape(coarse.shape)
    np.testing.assert_allclose(coarse.flatten(w_reg), coarse.flatten(coarse.to_regional(w_comp)), atol=1e-13)


# ------------------------------------------------------------------- RAP
@pytest.mark.parametrize("name", ["c1_small", "c2_small", "c3_small", "c5_small"])
def test_rap_theorem(name):
    """Theorem: Psibar R^(r) [[A]] P^(r) Psibar^T = R A P, at every level."""
    w, lay = layout_of(name)
    youngs = synth.region_youngs_moduli(w) if w.pde == "elasticity" else None
    ec = synth.jump_coefficients(w) if w.pde == "diffusion" else None
    coefs = regional.build_operator(lay, w.pde, h=w.h, elem_coef=ec, youngs=youngs, nu=w.nu)
    A = regional.composite_operator(lay, w.pde, h=w.h, elem_coef=ec, youngs=youngs, nu=w.nu)
    levels = regional.setup(lay, coefs, regional.Options(nlevels=w.nlevels, degree=w.cheb_degree))
    for l in range(1, w.nlevels):
        P = transfer.composite_prolongator(levels[l - 1].lay, levels[l].lay)
        A = P.T @ A @ P
        Ar = assembly.assemble_from_regions(levels[l].lay, levels[l].coefs)
        assert abs(Ar - A).max() <= 1e-13 * abs(A).max()


def test_rap_closed_form_2d():
    """Galerkin coarse stencil of the 5-point operator with rate-3 bilinear P:
    (1/3)[-1 2 -1] (x) M + M (x) (1/3)[-1 2 -1], M = [4/9 19/9 4/9], i.e.
    76/27 center, -11/27 edge, -8/27 corner (derived from the 1D products)."""
    o, e = synth.tensor_layout([[28, 28], [28, 28]])
    lay = Layout(2, o, e, 0xF)
    lv = regional.setup(lay, assembly.regional_fd5(lay), regional.Options(nlevels=2))
    Ac = assembly.assemble_from_regions(lv[1].lay, lv[1].coefs)
    node = np.arange(lv[1].lay.n_composite).reshape(lv[1].lay.shape)
    i = node[9, 9]  # interior coarse node on the region interface (x = y = 9)
    expect = {0: 76 / 27, 1: -11 / 27, 2: -8 / 27}
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            assert abs(Ac[i, node[9 + dy, 9 + dx]] - expect[abs(dx) + abs(dy)]) < 1e-14


def test_rap_q1_nested_spaces():
    """Q1 spaces are nested under rate-3 linear interpolation, so the interior Galerkin
    stencil equals the Q1 stencil of the coarse mesh (side 3h): 3x the fine stencil."""
    w, lay = layout_of("c2_mid")
    coefs = assembly.regional_q1(lay, "laplace", h=w.h)
    lv = regional.setup(lay, coefs, regional.Options(nlevels=3, degree=1))
    fine = coefs[0][:, 5, 5, 5]
    for l in (1, 2):
        c = lv[l].coefs[0][:, 2, 2, 2] if l == 2 else lv[l].coefs[0][:, 5, 5, 5]
        np.testing.assert_allclose(c, 3.0 ** l * fine, rtol=1e-12, atol=1e-13 * np.abs(c).max())


# -------------------------------------------------------------- smoothers
def test_chebyshev_is_the_chebyshev_polynomial():
    """With b = 0 the smoother maps e0 to p_K(D^-1 A) e0, p_K(t) = T_K((theta-t)/h)/T_K(theta/h)."""
    w, lay = layout_of("c1_small")
    coefs = assembly.regional_fd5(lay)
    for K in (1, 2, 3, 5):
        opt = regional.Options(nlevels=2, degree=K)
        lv = regional.setup(lay, coefs, opt)
        L = lv[0]
        A = assembly.composite_fd5(lay).toarray()
        dinv = 1.0 / np.diag(A)
        e0 = np.random.default_rng(K).standard_normal(lay.shape)
        e0[lay.dirichlet] = 0.0
        zero = lay.zeros_regional()
        u0 = lay.to_regional(e0)
        r0 = L.residual(zero, u0)
        uK = lay.to_composite_owner(regional.chebyshev(L, u0, zero, r0, opt)).reshape(-1)
        a, b = L.lam / opt.eig_ratio, opt.boost * L.lam
        theta, hw = 0.5 * (a + b), 0.5 * (b - a)
        # D^-1 A is similar to the symmetric D^-1/2 A D^-1/2
        S = np.sqrt(dinv)[:, None] * A * np.sqrt(dinv)[None, :]
        ev, V = np.linalg.eigh(S)
        T = np.polynomial.chebyshev.Chebyshev.basis(K)
        pk = T((theta - ev) / hw) / T(theta / hw)
        dm, dp = np.sqrt(dinv), 1.0 / np.sqrt(dinv)  # D^-1/2, D^1/2
        expect = dm * (V @ (pk * (V.T @ (dp * e0.reshape(-1)))))
        np.testing.assert_allclose(uK, expect, rtol=0, atol=1e-12 * np.abs(e0).max())


def test_power_method_bounds():
    w, lay = layout_of("c1_small")
    coefs = assembly.regional_fd5(lay)
    lv = regional.setup(lay, coefs, regional.Options(nlevels=2, power_iters=10))
    A = assembly.composite_fd5(lay).toarray()
    free = ~lay.dirichlet.reshape(-1)
    Af = A[np.ix_(free, free)]
    d = np.diag(Af)
    lmax = np.linalg.eigvalsh(Af / np.sqrt(np.outer(d, d))).max()
    assert lv[0].lam <= lmax * (1 + 1e-12)
    # sanity: 10 iterations land within 6% here (0.948 of lambda_max at this size and at C1's
    # 163^2); the boost 1.1 covers the rest
    assert lv[0].lam >= 0.94 * lmax


@pytest.mark.parametrize("name", ["c1_small", "c2_small"])
def test_power_method_equals_spectral_rayleigh_quotient(name):
    """The estimate is exactly the Rayleigh quotient (x, D^-1 A x) of the unit 10th iterate
    x ~ (D^-1 A)^9 x0, evaluated here from an eigendecomposition of the composite operator
    (D^-1 A = D^-1/2 V diag(mu) V^T D^1/2 with S = D^-1/2 A D^-1/2 = V diag(mu) V^T): a wrong
    iteration count, quotient, diagonal or interface sum in the regional iteration changes it."""
    w, lay = layout_of(name)
    coefs = regional.build_operator(lay, w.pde, h=w.h)
    opt = regional.Options(nlevels=2, power_iters=10)
    lv = regional.setup(lay, coefs, opt)
    A = regional.composite_operator(lay, w.pde, h=w.h)
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    free = ~lay.dirichlet.reshape(-1)
    Af = A[np.ix_(free, free)]
    d = np.diag(Af)
    mu, V = np.linalg.eigh(Af / np.sqrt(np.outer(d, d)))
    x0 = rng.uniform_pm1(lay.n_composite, 0, opt.seed)[free]
    c = V.T @ (np.sqrt(d) * x0)
    x9 = (V @ (mu ** 9 * c)) / np.sqrt(d)  # D^-1/2 V mu^9 V^T D^1/2 x0
    x9 /= np.linalg.norm(x9)
    Mx = (V @ (mu * (V.T @ (np.sqrt(d) * x9)))) / np.sqrt(d)
    lam = float(x9 @ Mx)
    assert abs(lv[0].lam - lam) <= 1e-12 * lam, (lv[0].lam, lam)


def test_counter_rng_reference_values():
    """SplitMix64 of state 0 gives 0xE220A8397B1DCDAF, the published first output for seed 0."""
    z = rng.splitmix64(np.array([0], dtype=np.uint64))
    assert int(z[0]) == 0xE220A8397B1DCDAF
    u = rng.uniform_pm1(1000, 2, 7)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.1


# -------------------------------------------------------- cycle and solve
@pytest.mark.parametrize("name,smoother", [("c1_small", "chebyshev"), ("c1_small", "jacobi"),
                                           ("c2_small", "chebyshev"), ("c3_small", "chebyshev"),
                                           ("c4_small", "chebyshev")])
def test_vcycle_regional_equals_composite(name, smoother):
    """Regional V-cycle = composite V-cycle on Psi^T r when the eigenvalue estimates are shared
    (the Table 1 equivalence, Section 6.1)."""
    w, lay = layout_of(name)
    youngs = synth.region_youngs_moduli(w) if w.pde == "elasticity" else None
    coefs = regional.build_operator(lay, w.pde, h=w.h, youngs=youngs, nu=w.nu)
    A = regional.composite_operator(lay, w.pde, h=w.h, youngs=youngs, nu=w.nu)
    opt = regional.Options(nlevels=w.nlevels, degree=w.cheb_degree, smoother=smoother)
    lv = regional.setup(lay, coefs, opt)
    clv = composite.setup(lay, A, opt, lams=[L.lam for L in lv[:-1]])
    b = synth.rhs(w)
    z = lay.to_composite_owner(regional.vcycle(lv, lay.to_regional(b), opt))
    zc = composite.vcycle(clv, b.reshape(-1), opt)
    np.testing.assert_allclose(z.reshape(-1), zc, rtol=0, atol=1e-13 * np.abs(zc).max())
    # copies of every interface dof agree (consistent regional vector)
    zr = regional.vcycle(lv, lay.to_regional(b), opt)
    np.testing.assert_allclose(lay.flatten(zr), lay.flatten(lay.to_regional(lay.to_composite_avg(zr))),
                               rtol=0, atol=1e-14 * np.abs(zc).max())


def test_jacobi_histories_coincide():
    """MG as a solver with damped Jacobi: regional and composite residual histories coincide."""
    w, lay = layout_of("c1_small")
    coefs = assembly.regional_fd5(lay)
    A = assembly.composite_fd5(lay)
    opt = regional.Options(nlevels=3, degree=1, smoother="jacobi", jacobi_omega=0.6)
    lv = regional.setup(lay, coefs, opt)
    clv = composite.setup(lay, A, opt)
    b = synth.rhs(w)
    _, h = regional.stationary(lv, lay.to_regional(b), lay.zeros_regional(), opt, 12)
    _, hc = composite.stationary(clv, b.reshape(-1), np.zeros(b.size), opt, 12)
    np.testing.assert_allclose(h, hc, rtol=1e-10)


def test_pcg_against_dense_solve():
    w, lay = layout_of("c1_small")
    coefs = assembly.regional_fd5(lay)
    A = assembly.composite_fd5(lay).toarray()
    opt = regional.Options(nlevels=3, degree=2)
    lv = regional.setup(lay, coefs, opt)
    b = synth.rhs(w)
    res = regional.pcg(lv, lay.to_regional(b), opt, rtol=1e-8)
    x = lay.to_composite_owner(res.x).reshape(-1)
    xs = np.linalg.solve(A, b.reshape(-1))
    kappa = np.linalg.cond(A)
    assert res.converged
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-8
    assert res.true_relres <= 1e-8


def test_pcg_manufactured_solution_3d():
    """b = A u* for u* = sin(pi x) sin(pi y) sin(pi z); solve to 1e-12 and recover u*."""
    w, lay = layout_of("c2_small")
    coefs = assembly.regional_q1(lay, "laplace", h=w.h)
    A = assembly.composite_q1(lay, "laplace", h=w.h)
    z, y, x = (np.indices(lay.shape) * w.h)
    ustar = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    ustar[lay.dirichlet] = 0.0
    b = (A @ ustar.reshape(-1)).reshape(lay.shape)
    opt = regional.Options(nlevels=3, degree=3)
    lv = regional.setup(lay, coefs, opt)
    res = regional.pcg(lv, lay.to_regional(b), opt, rtol=1e-12)
    u = lay.to_composite_owner(res.x)
    Ad = A.toarray()
    kappa = np.linalg.cond(Ad[np.ix_(~lay.dirichlet.reshape(-1), ~lay.dirichlet.reshape(-1))])
    assert np.linalg.norm(u - ustar) / np.linalg.norm(ustar) <= kappa * 1e-12


def test_discretization_error_second_order():
    """-Lap u = f on the unit square, five-point FD: max error falls as O(h^2) (textbook)."""
    errs = []
    for n in (10, 19, 37):  # regions 2x2 of n nodes; composite 2n-1
        o, e = synth.tensor_layout([[n, n], [n, n]])
        lay = Layout(2, o, e, 0xF)
        N = 2 * n - 1
        h = 1.0 / (N - 1)
        yy, xx = np.indices(lay.shape) * h
        uex = np.sin(np.pi * xx) * np.sin(np.pi * yy)
        f = 2 * np.pi ** 2 * uex * h * h  # five-point operator without 1/h^2
        f[lay.dirichlet] = 0.0
        nl = 2 if n == 10 else 3
        opt = regional.Options(nlevels=nl, degree=2)
        lv = regional.setup(lay, assembly.regional_fd5(lay), opt)
        res = regional.pcg(lv, lay.to_regional(f), opt, rtol=1e-12)
        u = lay.to_composite_owner(res.x)
        errs.append(np.abs(u - uex).max())
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(2.0) for i in range(2)]
    assert all(1.8 < r < 2.2 for r in rates), rates


def test_iterations_roughly_mesh_independent():
    its = []
    for n, nl in ((10, 3), (28, 3), (82, 3)):
        o, e = synth.tensor_layout([[n, n], [n, n]])
        lay = Layout(2, o, e, 0xF)
        wl = synth.Workload("x", 2, 1, o, e, 0xF, nl, 2, "fd5")
        opt = regional.Options(nlevels=nl, degree=2)
        lv = regional.setup(lay, assembly.regional_fd5(lay), opt)
        res = regional.pcg(lv, lay.to_regional(synth.rhs(wl)), opt)
        its.append(res.iterations)
    assert max(its) - min(its) <= 4, its


@pytest.mark.parametrize("name", ["c2_small", "c5_small", "c3_small"])
def test_q1_rows_match_assembled_operator(name):
    """Row-by-row evaluation of A x (used at sizes too large to assemble) equals the rows of the
    assembled composite operator, at every kind of node (interior, interface, boundary)."""
    from oracle import assembly
    from oracle.regions import Layout

    w = synth.workload(name)
    lay = Layout(w.dim, w.origins, w.extents, w.dirichlet_mask, w.ndof)
    ec = synth.jump_coefficients(w) if w.pde == "diffusion" else None
    youngs = synth.region_youngs_moduli(w) if w.pde == "elasticity" else None
    A = assembly.composite_q1(lay, w.pde, h=w.h, elem_coef=ec, youngs=youngs, nu=w.nu)
    rng = np.random.default_rng(3)
    shp = lay.shape + ((3,) if w.ndof == 3 else ())
    x = rng.uniform(-1, 1, size=shp)
    ref = (A @ x.reshape(-1)).reshape(shp)
    nz, ny, nx = lay.shape
    nodes = [tuple(int(v) for v in rng.integers(0, [nx, ny, nz])) for _ in range(60)]
    nodes += [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 2, ny // 2, nz // 2), (1, 1, 1)]
    coef = ec
    if w.pde == "elasticity":  # Young's modulus per element from the region containing it
        coef = np.zeros((nz - 1, ny - 1, nx - 1))
        for k in range(lay.nreg):
            o, e = lay.origins[k], lay.extents[k]
            coef[o[2]:o[2] + e[2] - 1, o[1]:o[1] + e[1] - 1, o[0]:o[0] + e[0] - 1] = youngs[k]
    got = assembly.q1_rows((nx, ny, nz), lay.dirichlet, x, nodes, w.pde, h=w.h, elem_coef=coef, nu=w.nu)
    want = np.array([ref[gz, gy, gx] for gx, gy, gz in nodes])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


# ------------------------------------------------- region-local Gauss-Seidel
def brute_force_region_gs(lay, coefs, dg, u, b, omega, sweeps, backward=False):
    """Algorithm 1 node by node on dense region matrices: per sweep the composite residual, then
    each region's dofs in (reverse) lexicographic order, r_i -= sum_j A_ij delta_j,
    delta_i = omega r_i / d~_i, u_i += delta_i; finally the copies of u are averaged."""
    Ad = [assembly.stencil_to_csr(c, lay.dim, lay.ndof).toarray() for c in coefs]
    for _ in range(sweeps):
        z = lay.interface_sum([(Ad[k] @ u[k].reshape(-1)).reshape(u[k].shape) for k in range(lay.nreg)])
        r = [b[k] - z[k] for k in range(lay.nreg)]
        new = []
        for k in range(lay.nreg):
            rk, uk, dk = r[k].reshape(-1).copy(), u[k].reshape(-1).copy(), dg[k].reshape(-1)
            delta = np.zeros_like(rk)
            order = range(rk.size - 1, -1, -1) if backward else range(rk.size)
            for i in order:
                rk[i] = rk[i] - sum(Ad[k][i, j] * delta[j] for j in np.nonzero(Ad[k][i])[0])
                delta[i] = omega * rk[i] / dk[i]
                uk[i] += delta[i]
            new.append(uk.reshape(u[k].shape))
        u = lay.to_regional(lay.to_composite_avg(new))
    return u


@pytest.mark.parametrize("case", ["2d", "3d", "elasticity", "uneven"])
@pytest.mark.parametrize("backward", [False, True])
def test_region_gs_against_brute_force(case, backward):
    rg = np.random.default_rng(7)
    if case == "elasticity":
        o, e = synth.tensor_layout([[4, 4], [4], [4]])
        lay = Layout(3, o, e, 1, 3)
        coefs = assembly.regional_q1(lay, "elasticity", youngs=np.array([1.0, 3.0]), nu=0.3)
    else:
        dim, slabs = {"2d": (2, [[4, 5], [4, 4]]), "3d": (3, [[4, 4], [4, 4], [4]]),
                      "uneven": (2, [[4, 7, 4], [7, 4]])}[case]
        o, e = synth.tensor_layout(slabs)
        lay = Layout(dim, o, e, 1)
        if dim == 2:
            coefs = assembly.regional_fd5(lay)
        else:
            coefs = assembly.regional_q1(lay, "diffusion",
                                         elem_coef=np.exp(rg.normal(size=tuple(s - 1 for s in lay.shape))))
    shp = lay.shape + ((lay.ndof,) if lay.ndof > 1 else ())
    x0 = rg.uniform(-1, 1, size=shp)
    x0[lay.dirichlet] = 0.0
    b = rg.uniform(-1, 1, size=shp)
    b[lay.dirichlet] = 0.0
    u0, br = lay.to_regional(x0), lay.to_regional(b)
    opt = regional.Options(nlevels=2, degree=2, smoother="gs", jacobi_omega=0.8)
    L = regional.Level(lay, coefs)
    dg = regional.composite_diagonal(lay, coefs)
    L.dinv = [1.0 / d for d in dg]
    got = regional.gauss_seidel(L, u0, br, L.residual(br, u0), opt, backward=backward)
    ref = brute_force_region_gs(lay, coefs, dg, u0, br, 0.8, 2, backward=backward)
    np.testing.assert_allclose(lay.flatten(got), lay.flatten(ref), rtol=0, atol=1e-13)


def test_one_region_gs_is_textbook_gs():
    """Without interfaces the region sweep is classical Gauss-Seidel on A: one sweep is
    u + (D/omega + L)^-1 (b - A u) with dense matrices; many sweeps reach A^-1 b."""
    o, e = synth.tensor_layout([[6], [5]])
    lay = Layout(2, o, e, 15)
    coefs = assembly.regional_fd5(lay)
    A = assembly.composite_fd5(lay).toarray()
    rg = np.random.default_rng(3)
    b = rg.uniform(-1, 1, size=lay.shape)
    b[lay.dirichlet] = 0.0
    u = rg.uniform(-1, 1, size=lay.shape)
    u[lay.dirichlet] = 0.0
    for backward in (False, True):
        opt = regional.Options(nlevels=1, degree=1, smoother="gs", jacobi_omega=0.7)
        L = regional.Level(lay, coefs)
        L.dinv = [1.0 / d for d in regional.composite_diagonal(lay, coefs)]
        got = regional.gauss_seidel(L, [u.copy()], [b], L.residual([b], [u.copy()]), opt, backward=backward)[0]
        T = (np.triu(A, 1) if backward else np.tril(A, -1)) + np.diag(np.diag(A)) / 0.7
        ref = u.reshape(-1) + np.linalg.solve(T, b.reshape(-1) - A @ u.reshape(-1))
        np.testing.assert_allclose(got.reshape(-1), ref, rtol=0, atol=1e-14)
    opt = regional.Options(nlevels=1, degree=400, smoother="gs", jacobi_omega=1.0)
    got = regional.gauss_seidel(L, [np.zeros_like(b)], [b], [b], opt)[0]
    np.testing.assert_allclose(got.reshape(-1), np.linalg.solve(A, b.reshape(-1)), rtol=0, atol=1e-12)


@pytest.mark.parametrize("smoother", ["gs", "sgs"])
def test_one_region_gs_vcycle_equals_composite(smoother):
    o, e = synth.tensor_layout([[19], [19]])
    lay = Layout(2, o, e, 15)
    opt = regional.Options(nlevels=3, degree=1, smoother=smoother, jacobi_omega=1.0)
    lv = regional.setup(lay, assembly.regional_fd5(lay), opt)
    clv = composite.setup(lay, assembly.composite_fd5(lay), opt)
    b = np.random.default_rng(5).uniform(-1, 1, size=lay.shape)
    b[lay.dirichlet] = 0.0
    z = regional.vcycle(lv, [b], opt)[0]
    zc = composite.vcycle(clv, b.reshape(-1), opt)
    np.testing.assert_allclose(z.reshape(-1), zc, rtol=0, atol=1e-13 * np.abs(zc).max())


def test_symmetric_gs_vcycle_is_symmetric():
    """Forward pre-sweeps and backward post-sweeps make the composite V-cycle a symmetric operator
    (a transposed sweep direction breaks it); forward sweeps on both sides do not."""
    w, lay = layout_of("c1_small")
    A = assembly.composite_fd5(lay)
    free = np.flatnonzero(~lay.dirichlet.reshape(-1))
    rg = np.random.default_rng(11)
    a, c = np.zeros(A.shape[0]), np.zeros(A.shape[0])
    a[free], c[free] = rg.uniform(-1, 1, free.size), rg.uniform(-1, 1, free.size)
    asym = {}
    for sm in ("sgs", "gs"):
        opt = regional.Options(nlevels=3, degree=1, smoother=sm, jacobi_omega=1.0)
        clv = composite.setup(lay, A, opt)
        va, vc = composite.vcycle(clv, a, opt), composite.vcycle(clv, c, opt)
        asym[sm] = abs(c @ va - a @ vc) / (np.linalg.norm(a) * np.linalg.norm(vc))
    assert asym["sgs"] < 1e-13 and asym["gs"] > 1e-4


def test_region_gs_histories_close_to_composite():
    """MG as a solver with Gauss-Seidel (Table 1 setting): the region-local smoother differs from
    true Gauss-Seidel only through the interface updates, so the histories stay close."""
    w, lay = layout_of("c1_small")
    opt = regional.Options(nlevels=3, degree=1, smoother="gs", jacobi_omega=1.0)
    lv = regional.setup(lay, assembly.regional_fd5(lay), opt)
    clv = composite.setup(lay, assembly.composite_fd5(lay), opt)
    b = synth.rhs(w)
    _, h = regional.stationary(lv, lay.to_regional(b), lay.zeros_regional(), opt, 12)
    _, hc = composite.stationary(clv, b.reshape(-1), np.zeros(b.size), opt, 12)
    h, hc = np.asarray(h), np.asarray(hc)
    ratio = h[1:] / hc[1:]
    print("regional/composite GS residual ratios", np.round(ratio, 3))
    assert np.all(ratio > 0.5) and np.all(ratio < 2.0)
    assert not np.allclose(h, hc, rtol=1e-6)  # not the same smoother
    assert h[-1] < 1e-6 and hc[-1] < 1e-6
