"""Pins of the hybrid structured/unstructured oracle (the paper's structured/unstructured mesh
hybrid section, Table 5): aggregation invariants, the Lemma on P for aggregation transfers,
closed-form aggregate sizes, the Theorem (regional Galerkin levels and regional Jacobi cycles equal
the composite ones), symmetry of the symmetric Gauss-Seidel W-cycle, the W-cycle's two-level
formula, and Table 5's structure (unstructured regions change the iteration count only a little).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import assembly, composite, hybrid, regional
from oracle.regions import Layout

KINDS = {
    "structured": [],
    "unstructured": list(range(27)),
    "centre": [13],
    "left_face": [k for k in range(27) if k % 3 == 0],
    "corners": [0, 2, 6, 8, 18, 20, 24, 26],
}


def layout(ext=10, mask=63):
    o, e = synth.tensor_layout([[ext] * 3] * 3)
    return Layout(3, o, e, mask)


def finest(lay):
    return hybrid.finest_level(lay, assembly.split_composite(lay, assembly.composite_fd7(lay)))


def kinds_of(name, n=27):
    k = np.zeros(n, dtype=int)
    k[KINDS[name]] = 1
    return k


@pytest.mark.parametrize("name", list(KINDS))
def test_aggregation_invariants(name):
    lay = layout()
    L = finest(lay)
    kinds = kinds_of(name)
    for _ in range(2):  # levels 0 and 1
        aggs, C = hybrid.coarsen(L, kinds)
        # every free node in exactly one aggregate, Dirichlet nodes in none, coarse numbers dense
        for k, R in enumerate(L.regions):
            assert np.array_equal(aggs[k] >= 0, R.free)
            nc = C.regions[k].comp.size
            assert np.array_equal(np.unique(aggs[k][aggs[k] >= 0]), np.arange(nc))
        # Lemma on P: every copy of a composite node ends in the same coarse composite node
        target = {}
        for k, R in enumerate(L.regions):
            for i in np.flatnonzero(aggs[k] >= 0):
                t = int(C.regions[k].comp[aggs[k][i]])
                assert target.setdefault(int(R.comp[i]), t) == t
        # structured aggregates are the boxes of one coarse point; unstructured ones are connected
        for k, R in enumerate(L.regions):
            for a in range(C.regions[k].comp.size):
                members = np.flatnonzero(aggs[k] == a)
                if not kinds[k]:
                    cps = hybrid.coarse_point(R.coords[members], L.shape, L.mask)
                    assert (cps == cps[0]).all()
                else:
                    sub = R.A[members][:, members]
                    ncomp, _ = sp.csgraph.connected_components(sub != 0, directed=False)
                    assert ncomp == 1
        # the coarse level's regions: co-located nodes carry equal coordinates
        for R in C.regions:
            shared = R.coords[:, 0] >= 0
            assert (R.coords[shared] >= 0).all()
        for k, R in enumerate(L.regions):
            P = hybrid.region_prolongator(aggs[k], C.regions[k].comp.size)
            C.regions[k].A = sp.csr_matrix(P.T @ R.A @ P)
        L = C


def test_structured_aggregate_sizes_closed_form():
    """All regions structured: composite aggregates are products of per-axis runs.  On 28 nodes
    per axis with Dirichlet ends the free nodes 1..26 group as {1,2,3,4}, {5,6,7}, ...,
    {23,24,25,26} around the coarse points 3, 6, ..., 24."""
    lay = layout()
    L = finest(lay)
    aggs, C = hybrid.coarsen(L, kinds_of("structured"))
    L.agg = aggs
    P = hybrid.composite_prolongator(L, C)
    sizes = np.asarray(P.sum(axis=0)).ravel()
    run = np.array([4] + [3] * 6 + [4])
    expect = np.sort((run[:, None, None] * run[None, :, None] * run[None, None, :]).ravel())
    assert C.ncomp == 8 ** 3
    np.testing.assert_array_equal(np.sort(sizes), expect)


@pytest.mark.parametrize("name", ["structured", "centre", "left_face", "unstructured"])
@pytest.mark.parametrize("gamma", [1, 2])
def test_theorem_regional_equals_composite(name, gamma):
    """Regional Galerkin levels equal P^T A P of the composite operator, and the regional cycle
    with Jacobi smoothing equals the composite cycle (Theorem, Lemmas on P and R)."""
    lay = layout()
    opt = hybrid.HOptions(nlevels=3, degree=2, smoother="jacobi", omega=0.7, gamma=gamma)
    lv = hybrid.setup(finest(lay), kinds_of(name), opt)
    A = lv[0].composite_matrix()
    assert abs(A - assembly.composite_fd7(lay)).max() <= 1e-14
    cl = []
    for l, L in enumerate(lv):
        C = composite.CLevel(None, A)
        if l < len(lv) - 1:
            C.dinv = 1.0 / A.diagonal()
            C.P = hybrid.composite_prolongator(L, lv[l + 1])
            Ac = sp.csr_matrix(C.P.T @ A @ C.P)
            assert abs(lv[l + 1].composite_matrix() - Ac).max() <= 1e-12 * abs(Ac).max()
            A = Ac
        cl.append(C)
    copt = regional.Options(nlevels=3, degree=2, smoother="jacobi", jacobi_omega=0.7, gamma=gamma)
    b = synth.rhs(synth.Workload("h", 3, 1, lay.origins, lay.extents, 63, 3, 2, "fd7", seed=0))
    z = lv[0].to_composite_owner(hybrid.cycle(lv, lv[0].to_regional(b.reshape(-1)), opt))
    zc = composite.vcycle(cl, b.reshape(-1), copt)
    np.testing.assert_allclose(z, zc, rtol=0, atol=1e-12 * np.abs(zc).max())


def test_wcycle_two_level_formula():
    """With three levels, the W-cycle replaces the level-1 solve by two level-1 cycles: its coarse
    correction is (I - E_1^2) A_1^-1 with E_1 the level-1 cycle's error propagation, checked with
    dense matrices on the composite form."""
    lay = layout()
    opt = hybrid.HOptions(nlevels=3, degree=1, smoother="jacobi", omega=0.6, gamma=2)
    lv = hybrid.setup(finest(lay), kinds_of("centre"), opt)
    P0 = hybrid.composite_prolongator(lv[0], lv[1]).toarray()
    A0 = lv[0].composite_matrix().toarray()
    A1 = lv[1].composite_matrix().toarray()
    n1 = A1.shape[0]
    # level-1 cycle as a dense operator B1 (cycle on level 1 from b1)
    B1 = np.column_stack([lv[1].to_composite_owner(hybrid.cycle(lv, lv[1].to_regional(e), opt, 1))
                          for e in np.eye(n1)])
    E1 = np.eye(n1) - B1 @ A1
    coarse = (np.eye(n1) - E1 @ E1) @ np.linalg.inv(A1)
    D = np.diag(A0)
    free = D != 1.0
    b = np.where(free, np.random.default_rng(2).uniform(-1, 1, A0.shape[0]), 0.0)
    S = lambda u, f: u + 0.6 * (f - A0 @ u) / D  # noqa: E731
    u = S(np.zeros_like(b), b)
    u = u + P0 @ (coarse @ (P0.T @ (b - A0 @ u)))
    u = S(u, b)
    z = lv[0].to_composite_owner(hybrid.cycle(lv, lv[0].to_regional(b), opt))
    np.testing.assert_allclose(z, u, rtol=0, atol=1e-12 * np.abs(u).max())


def test_symmetric_gs_wcycle_is_symmetric():
    """One region (no interface averaging): the W-cycle with symmetric Gauss-Seidel is a
    symmetric operator; forward-only Gauss-Seidel is not."""
    o, e = synth.tensor_layout([[28]] * 3)
    lay = Layout(3, o, e, 63)
    rg = np.random.default_rng(4)
    free = ~lay.dirichlet.reshape(-1)
    a = np.where(free, rg.uniform(-1, 1, free.size), 0.0)
    c = np.where(free, rg.uniform(-1, 1, free.size), 0.0)
    asym = {}
    for sm in ("symgs", "gs"):
        opt = hybrid.HOptions(nlevels=3, degree=2, smoother=sm, omega=1.0, gamma=2)
        lv = hybrid.setup(finest(lay), [1], opt)
        va = lv[0].to_composite_owner(hybrid.cycle(lv, lv[0].to_regional(a), opt))
        vc = lv[0].to_composite_owner(hybrid.cycle(lv, lv[0].to_regional(c), opt))
        asym[sm] = abs(c @ va - a @ vc) / (np.linalg.norm(a) * np.linalg.norm(vc))
    assert asym["symgs"] < 1e-13 and asym["gs"] > 1e-5


def test_table5_structure():
    """W-cycle, two symmetric Gauss-Seidel iterations, piecewise-constant transfers, MG as a solver
    to 1e-6: every layout converges, and unstructured regions change the count only a little."""
    lay = layout()
    b = synth.rhs(synth.Workload("h", 3, 1, lay.origins, lay.extents, 63, 3, 2, "fd7", seed=0)).reshape(-1)
    its = {}
    for name in ("structured", "centre", "unstructured"):
        opt = hybrid.HOptions(nlevels=3, degree=2, smoother="symgs", omega=1.0, gamma=2)
        lv = hybrid.setup(finest(lay), kinds_of(name), opt)
        _, h = hybrid.stationary(lv, lv[0].to_regional(b), [np.zeros(R.comp.size) for R in lv[0].regions], opt)
        assert h[-1] <= 1e-6
        its[name] = len(h) - 1
    print("Table 5 structure, cycles to 1e-6:", its)
    assert max(its.values()) <= 30 and max(its.values()) - min(its.values()) <= 4


def test_staged_aggregation_hand_example():
    """One unstructured 4x3 region of the five-point operator, no interfaces and no Dirichlet
    nodes, rows i = x + 4y.  Worked by hand: stage II makes roots 0 -> {0, 1, 4}, 3 -> {3, 2, 7}
    and 9 -> {9, 8, 10, 5} (2, 5, 6, 8 and 11 each have an aggregated neighbour when visited);
    stage III: node 6 couples twice to {2, 3, 7} and twice to {5, 8, 9, 10}, node 11 once to each,
    and both ties go to the aggregate whose smallest member comes first ({2, 3, 7}); stage IV has
    nothing left.  Coarse nodes in order of smallest member: {0,1,4}, {2,3,6,7,11}, {5,8,9,10}."""
    o, e = synth.tensor_layout([[4], [3]])
    lay = Layout(2, o, e, 0)
    L = hybrid.finest_level(lay, assembly.split_composite(lay, assembly.composite_fd5(lay)))
    R = L.regions[0]
    agg, points = hybrid.aggregate_region(R, True, np.zeros(R.comp.size, dtype=bool), L.shape, L.mask)
    first = {}
    for i, a in enumerate(agg):
        first.setdefault(a, i)
    order = {a: c for c, a in enumerate(sorted(first, key=first.get))}
    np.testing.assert_array_equal([order[a] for a in agg], [0, 0, 1, 1, 0, 2, 1, 1, 2, 2, 2, 1])
    assert points == {}  # no aggregate came from the structured rule
