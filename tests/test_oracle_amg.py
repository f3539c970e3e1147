"""Pins of the oracle's AMG coarse solver (Section 3.5, second option: one AMG V-cycle on the
coarsest composite operator instead of a direct solve; smoothed aggregation after the SA-AMG it
cites).

Pinned by a hand-worked 1D example (aggregates, smoothing weight, smoothed prolongator and coarse
operator written out as fractions), the constant preserved by P on rows where A 1 = 0 (closed
form of the smoothing step), aggregates partitioning the free rows, the two-level cycle against
its error propagator composed from dense matrices and the closed-form Chebyshev polynomial,
symmetry of the multilevel cycle, the direct solve it reduces to, and the Theorem: the region cycle with the AMG coarse solver equals the
composite cycle with the same coarse solver.
"""
from fractions import Fraction as F

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amg, assembly, composite, regional
from oracle.regions import Layout
from tests import harness


def laplace_1d_7():
    """1D Laplacian [-1 2 -1] on 7 nodes, end nodes Dirichlet (identity rows, eliminated)."""
    n = 7
    A = np.zeros((n, n))
    A[0, 0] = A[6, 6] = 1.0
    for i in range(1, 6):
        A[i, i] = 2.0
        if i > 1:
            A[i, i - 1] = -1.0
        if i < 5:
            A[i, i + 1] = -1.0
    return sp.csr_matrix(A), np.array([0, 1, 1, 1, 1, 1, 0], dtype=bool)


def test_hand_worked_1d():
    """Stage II makes row 1 a root with row 2, row 3 is left, row 4 a root with rows 3 and 5:
    aggregates {1, 2}, {3, 4, 5}.  rho = max (2 + 1 + 1) / 2 = 2, omega = 4 / 6 = 2/3; the columns
    of P = T - omega D^-1 A T and P^T A P worked out by hand."""
    A, free = laplace_1d_7()
    lv = amg.setup(A, free, coarse_size=2)
    assert len(lv) == 2
    np.testing.assert_array_equal(lv[0].agg, [-1, 0, 0, 1, 1, 1, -1])
    assert lv[0].omega == 2.0 / 3.0
    t = F(1, 3)
    P = [[0, 0], [2 * t, 0], [2 * t, t], [t, 2 * t], [0, 1], [0, 2 * t], [0, 0]]
    np.testing.assert_allclose(lv[0].P.toarray(), np.array(P, dtype=float), atol=1e-16)
    Ac = [[F(2, 3), F(-2, 9)], [F(-2, 9), F(8, 9)]]
    np.testing.assert_allclose(lv[1].Adense, np.array(Ac, dtype=float), atol=1e-15)


def lattice_laplace(n=24):
    o, e = synth.tensor_layout([[n], [n]])
    lay = Layout(2, o, e, 15)
    return lay, sp.csr_matrix(assembly.composite_fd5(lay)), ~lay.dirichlet.reshape(-1)


def test_aggregates_partition_the_free_rows():
    lay, A, free = lattice_laplace()
    agg = amg.aggregates(A, free)
    assert np.all(agg[~free] == -1) and np.all(agg[free] >= 0)
    firsts = [int(np.flatnonzero(agg == a)[0]) for a in range(agg.max() + 1)]
    assert firsts == sorted(firsts)  # numbered by smallest row
    # each aggregate is connected in the matrix graph
    G = sp.csr_matrix((A != 0).astype(int))
    for a in range(agg.max() + 1):
        rows = np.flatnonzero(agg == a)
        sub = G[rows][:, rows]
        ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
        assert ncomp == 1


def test_smoothed_prolongator_keeps_constants():
    """P 1 = (I - omega D^-1 A) T 1 = 1 - omega D^-1 A 1 = 1 on every aggregated row with A 1 = 0."""
    lay, A, free = lattice_laplace()
    lv = amg.setup(A, free, coarse_size=10)
    P = lv[0].P
    ones = np.ones(P.shape[1])
    rows = np.flatnonzero(np.isclose(A @ np.ones(A.shape[0]), 0.0, atol=1e-14) & free)
    assert rows.size > 100
    np.testing.assert_allclose((P @ ones)[rows], 1.0, atol=1e-14)


def chebyshev_matrix(Ad, K, rho, eta):
    """p_K(D^-1 A) = T_K((theta I - D^-1 A) / h) / T_K(theta / h), theta, h the centre and half
    width of [rho / eta, rho], T_K by its three-term recurrence (the polynomial the smoother's
    error follows)."""
    n = Ad.shape[0]
    alpha, beta = rho / eta, rho
    theta, h = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    X = (theta * np.eye(n) - Ad / np.diag(Ad)[:, None]) / h
    Tm, T = np.eye(n), X
    tm, t = 1.0, theta / h
    for _ in range(K - 1):
        Tm, T = T, 2.0 * X @ T - Tm
        tm, t = t, 2.0 * (theta / h) * t - tm
    return (np.eye(n) if K == 0 else T) / (1.0 if K == 0 else t)


@pytest.mark.parametrize("K", [1, 2, 3])
def test_two_level_cycle_is_its_error_propagator(K):
    """With an exact coarse solve, V(b) = (I - E) A^-1 b with E = S (I - P Ac^-1 P^T A) S and
    S = p_K(D^-1 A) the Chebyshev polynomial, composed here from dense matrices."""
    lay, A, free = lattice_laplace(13)
    lv = amg.setup(A, free, coarse_size=60, degree=K)
    assert len(lv) == 2
    Ad = A.toarray()
    n = Ad.shape[0]
    I = np.eye(n)
    P = lv[0].P.toarray()
    Ac = P.T @ Ad @ P
    S = chebyshev_matrix(Ad, K, amg.gershgorin(A), 20.0)
    E = S @ (I - P @ np.linalg.solve(Ac, P.T @ Ad)) @ S
    B = np.random.default_rng(1).standard_normal((n, 3))
    for j in range(3):
        expect = (I - E) @ np.linalg.solve(Ad, B[:, j])
        np.testing.assert_allclose(amg.vcycle(lv, B[:, j]), expect, rtol=1e-10, atol=1e-12)


def test_multilevel_cycle_is_symmetric_and_reduces_to_direct():
    lay, A, free = lattice_laplace(40)
    lv = amg.setup(A, free, coarse_size=20)
    assert len(lv) >= 3
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    a, b = amg.vcycle(lv, x) @ y, x @ amg.vcycle(lv, y)
    assert abs(a - b) <= 1e-12 * abs(a)
    direct = amg.setup(A, free, coarse_size=A.shape[0])
    assert len(direct) == 1
    np.testing.assert_allclose(amg.vcycle(direct, x), np.linalg.solve(A.toarray(), x), rtol=1e-12)


@pytest.mark.parametrize("name", ["c2_small", "uneven2d_small"])
def test_region_cycle_with_amg_coarse_solve(name):
    """Theorem: the region hierarchy's coarsest composite operator is the composite one, so the
    region PCG with the AMG coarse solver has the composite PCG history with the same AMG; it
    needs no more than two iterations beyond the direct coarse solve."""
    w = synth.workload(name)
    b = synth.rhs(w)
    lay, lv, opt = harness.oracle_problem(w, nlevels=2, coarse_amg=True, amg_coarse_size=30)
    assert len(lv[-1].amg) >= 2
    ref = regional.pcg(lv, lay.to_regional(b), opt, rtol=1e-8)
    A = regional.composite_operator(lay, w.pde, h=w.h)
    clv = composite.setup(lay, A, opt, lams=[L.lam for L in lv[:-1]])
    _, its, hist = composite.pcg(clv, b.reshape(-1), opt, rtol=1e-8)
    assert its == ref.iterations
    np.testing.assert_allclose(hist, ref.history, rtol=1e-9)
    _, lvd, optd = harness.oracle_problem(w, nlevels=2)
    direct = regional.pcg(lvd, lay.to_regional(b), optd, rtol=1e-8)
    assert ref.converged and ref.iterations <= direct.iterations + 2
