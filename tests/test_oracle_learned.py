"""Pins of the learned-prolongator part of the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import assembly, learned, regional, transfer
from oracle.regions import Layout


def small_problem():
    w = synth.workload("c5_small")
    lay = Layout(w.dim, w.origins, w.extents, w.dirichlet_mask)
    ec = synth.jump_coefficients(w)
    return w, lay, ec


def random_theta(seed=0, scale=0.3):
    return np.random.default_rng(seed).standard_normal(learned.NPARAM) * scale


def test_cell_node_table():
    # 24 edge nodes x 2 corners + 24 face nodes x 4 + 8 interior x 8 = 208 logits
    counts = [len(n[3]) for n in learned.NODES]
    assert counts.count(2) == 24 and counts.count(4) == 24 and counts.count(8) == 8
    assert learned.NPARAM == 19472


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((5, 27))
    E = rng.standard_normal((5, 4, 4, 4))
    theta = random_theta(1)
    L, g = learned.loss_and_grad(theta, X, E)
    h = 1e-6
    idx = rng.choice(learned.NPARAM, size=40, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (learned.loss_and_grad(tp, X, E)[0] - learned.loss_and_grad(tm, X, E)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_forward_hand_computed_network():
    """A network worked by hand: sparse weights, non-zero biases on every layer and negative
    pre-activations in both hidden layers, so each ReLU, each bias, the layer order and the
    orientation of every weight matrix change the logits if done wrong.  The flat parameter
    vector is laid out here from the documented order (W1 64x27 row-major, b1, W2 64x64, b2,
    W3 208x64, b3), not through the oracle's own unpacking."""
    nin, nh, nout = 27, 64, 208
    theta = np.zeros(nh * nin + nh + nh * nh + nh + nout * nh + nout)
    oW1, ob1 = 0, nh * nin
    oW2, ob2 = ob1 + nh, ob1 + nh + nh * nh
    oW3, ob3 = ob2 + nh, ob2 + nh + nout * nh
    # layer 1: a1_0 = x0 + x1 + 0.5 = -0.5 (ReLU -> 0); a1_1 = 2 x0 + 0.25 = 2.25;
    #          a1_2 = -x1 - 3 = -1 (ReLU -> 0)
    theta[oW1 + 0 * nin + 0] = 1.0
    theta[oW1 + 0 * nin + 1] = 1.0
    theta[ob1 + 0] = 0.5
    theta[oW1 + 1 * nin + 0] = 2.0
    theta[ob1 + 1] = 0.25
    theta[oW1 + 2 * nin + 1] = -1.0
    theta[ob1 + 2] = -3.0
    # layer 2: a2_0 = 100 h1_0 + 2 h1_1 - 7 h1_2 - 1 = 3.5; a2_1 = -h1_1 + 0.5 = -1.75 (ReLU -> 0);
    #          W2[1, 0] = 5 would move h1_0 into a2_1 if W2 were applied transposed: it is 0 there
    theta[oW2 + 0 * nh + 0] = 100.0
    theta[oW2 + 0 * nh + 1] = 2.0
    theta[oW2 + 0 * nh + 2] = -7.0
    theta[ob2 + 0] = -1.0
    theta[oW2 + 1 * nh + 1] = -1.0
    theta[ob2 + 1] = 0.5
    theta[oW2 + 1 * nh + 0] = 5.0
    # layer 3: z_0 = h2_0 + 10 h2_1 + 0.125 = 3.625; z_5 = -2 h2_0 + b3_5 = -7 + 0.05;
    #          every other z_k = b3_k = 0.01 k
    theta[oW3 + 0 * nh + 0] = 1.0
    theta[oW3 + 0 * nh + 1] = 10.0
    theta[oW3 + 5 * nh + 0] = -2.0
    theta[ob3:ob3 + nout] = 0.01 * np.arange(nout)
    theta[ob3 + 0] = 0.125
    X = np.zeros((2, nin))
    X[0, 0], X[0, 1] = 1.0, -2.0  # sample 0 as above
    # sample 1: x0 = -1: a1_0 = -0.5 -> 0, a1_1 = -1.75 -> 0, a1_2 = -3 -> 0; a2_0 = -1 -> 0,
    # a2_1 = 0.5; z_0 = 10 * 0.5 + 0.125 = 5.125, z_5 = 0.05
    X[1, 0] = -1.0
    z, _ = learned.forward(theta, X)
    expect = np.tile(0.01 * np.arange(nout), (2, 1))
    expect[0, 0], expect[0, 5] = 3.625, -7.0 + 0.05
    expect[1, 0], expect[1, 5] = 5.125, 0.05
    np.testing.assert_allclose(z, expect, rtol=0, atol=1e-14)


def test_softmax_weights_partition_of_unity():
    X = np.random.default_rng(4).standard_normal((7, 27))
    z, _ = learned.forward(random_theta(2), X)
    for w in learned.weights_from_logits(z):
        np.testing.assert_allclose(w.sum(axis=1), 1.0, atol=1e-15)
        assert (w >= 0).all()


def test_geometric_stored_weights_reproduce_linear_interpolation():
    _, lay, _ = small_problem()
    coarse = lay.coarsen()
    W = learned.geometric_weights(lay, coarse)
    for k in range(lay.nreg):
        A = learned.stored_prolongator(lay, coarse, k, W[k])
        B = transfer.region_prolongator(lay, coarse, k)
        assert abs(A - B).max() < 1e-15


def test_learned_weights_consistent_and_rap_theorem():
    """Averaged learned weights: co-located rows match across regions (Lemma P holds), free rows
    away from the boundary sum to 1, corners inject, and the Galerkin theorem holds with them."""
    w, lay, ec = small_problem()
    coarse = lay.coarsen()
    W = learned.node_weights(lay, coarse, random_theta(5), ec)
    Pk = [learned.stored_prolongator(lay, coarse, k, W[k]) for k in range(lay.nreg)]
    Pr = sp.block_diag(Pk).tocsr()
    Psi, Psib = lay.psi_matrix(), coarse.psi_matrix()
    # Lemma P: P^(r) Psibar^T = Psi^T P for the composite P assembled from region 0.. rows
    M = Pr @ Psib.T  # rows of every regional copy
    P = sp.csr_matrix((Psi @ M).multiply(1.0 / lay.mult.reshape(-1)[:, None]))  # average of copies
    assert abs(M - Psi.T @ P).max() < 1e-14  # copies agree
    rows = np.asarray(P.sum(axis=1)).ravel().reshape(lay.shape)
    inner = (slice(3, -3),) * 3
    np.testing.assert_allclose(rows[inner], 1.0, atol=1e-13)
    coefs = assembly.regional_q1(lay, "diffusion", h=w.h, elem_coef=ec)
    A = assembly.composite_q1(lay, "diffusion", h=w.h, elem_coef=ec)
    lv = regional.setup(lay, coefs, regional.Options(nlevels=2, degree=2), P0=Pk)
    Ar = assembly.assemble_from_regions(lv[1].lay, lv[1].coefs)
    RAP = P.T @ A @ P
    assert abs(Ar - RAP).max() <= 1e-12 * abs(RAP).max()


def test_adam_first_step():
    theta = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    t1, m, v = learned.adam_step(theta, g, np.zeros(4), np.zeros(4), 1, 0.1)
    # bias-corrected first step moves every nonzero coordinate by lr against the gradient's sign
    np.testing.assert_allclose(t1[:3], -0.1 * np.sign(g[:3]), rtol=1e-6)
    assert t1[3] == 0.0


def test_training_reduces_loss():
    w, lay, ec = small_problem()
    coefs = assembly.regional_q1(lay, "diffusion", h=w.h, elem_coef=ec)
    opt = regional.Options(nlevels=2, degree=3)
    lv = regional.setup(lay, coefs, opt)
    X, E = learned.training_set(lay, lv, opt, ec, nsamples=2, seed=1)
    theta = random_theta(6, 0.1)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0, _ = learned.loss_and_grad(theta, X, E)
    for t in range(1, 61):
        L, g = learned.loss_and_grad(theta, X, E)
        theta, m, v = learned.adam_step(theta, g, m, v, t, 3e-3)
    L1, _ = learned.loss_and_grad(theta, X, E)
    assert L1 < 0.7 * L0, (L0, L1)


def test_energy_gradient_matches_central_differences():
    rng = np.random.default_rng(13)
    X = rng.standard_normal((4, 27))
    E = rng.standard_normal((4, 4, 4, 4))
    theta = random_theta(7)
    L, g = learned.loss_and_grad(theta, X, E, kind="energy")
    h = 1e-6
    for i in rng.choice(learned.NPARAM, size=40, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (learned.loss_and_grad(tp, X, E, kind="energy")[0] - learned.loss_and_grad(tm, X, E, kind="energy")[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_cell_matrix_is_the_assembled_cube_operator():
    """With unit coefficients the cell operator is the Q1 Laplacian assembled on one 4^3-node
    box without boundary conditions; it is symmetric and annihilates constants for any c."""
    lay = Layout(3, np.array([[0, 0, 0]]), np.array([[4, 4, 4]]), 0)
    A1 = assembly.composite_q1(lay, "laplace", h=1.0).toarray()
    np.testing.assert_allclose(learned.cell_matrix(np.zeros((1, 27)))[0], A1, atol=1e-14)
    X = np.random.default_rng(2).standard_normal((3, 27))
    A = learned.cell_matrix(X)
    np.testing.assert_allclose(A, np.transpose(A, (0, 2, 1)), atol=1e-14)
    np.testing.assert_allclose(A @ np.ones(64), 0.0, atol=1e-12)


def test_energy_loss_vanishes_for_trilinear_errors():
    """Trilinear weights (zero hidden-to-output weights, output biases log w) reproduce any
    affine error exactly, so both losses vanish."""
    theta = np.zeros(learned.NPARAM)
    b3 = theta[-learned.NOUT:]
    for n, (i, j, k, corners) in enumerate(learned.NODES):
        for c, slot in enumerate(corners):
            w = 1.0
            for d, p in enumerate((i, j, k)):
                w *= p / 3.0 if (slot >> d) & 1 else (3 - p) / 3.0
            b3[learned.LOGIT_OFFSET[n] + c] = np.log(w)
    g = np.arange(4.0)
    a = np.random.default_rng(1).standard_normal((3, 4))
    E = np.stack([a[s, 0] + a[s, 1] * g[None, None, :] + a[s, 2] * g[None, :, None] + a[s, 3] * g[:, None, None]
                  for s in range(3)])
    X = np.random.default_rng(5).standard_normal((3, 27))
    for kind in ("l2", "energy"):
        L, _ = learned.loss_and_grad(theta, X, E, kind=kind)
        assert L < 1e-28, (kind, L)
