"""Oracle pins of the AMG coarse solver for 3D elasticity (Section 3.5: the AMG hierarchy needs the
coarse operator and its near-null space, taken from the region hierarchy).

* The rigid-body modes at the coarsest nodes' finest-lattice positions span the null space of the
  coarsest composite operator of a pure-Neumann problem (A B = 0 to rounding): pins the position
  chain through the levels and the six modes.
* The tentative prolongator has orthonormal columns and reproduces the near-null space exactly on
  aggregated rows (T B_c = B).
* The node graph couples two nodes exactly when their block is non-negligible.
* The AMG V-cycle on elasticity contracts the error as a stationary iteration, and the region PCG
  with it converges to 1e-8.
"""
import numpy as np
import scipy.sparse as sp

import synth
from oracle import amg, assembly, regional
from oracle.regions import Layout


# uneven slabs of 3^k + 1 nodes: the coarse lattices are not uniform, while every region's linear
# interpolation stays exact on linear functions
UNEVEN = ((10, 4, 10), (10, 10), (4, 10))


def elasticity_levels(mask, nlevels=3, slabs=UNEVEN, coarse_amg=False, coarse_size=30):
    o, e = synth.tensor_layout([list(s) for s in slabs])
    lay = Layout(3, o, e, mask, 3)
    youngs = [10.0 ** (k % 3) for k in range(lay.nreg)]
    coefs = regional.build_operator(lay, "elasticity", h=1.0 / 18, youngs=youngs, nu=0.3)
    opt = regional.Options(nlevels=nlevels, degree=2, coarse_amg=coarse_amg, amg_coarse_size=coarse_size)
    return lay, coefs, opt, regional.setup(lay, coefs, opt)



def test_rigid_body_modes_are_the_coarse_null_space():
    lay, coefs, opt, levels = elasticity_levels(0)
    L = levels[-1]
    A = assembly.assemble_from_regions(L.lay, L.coefs)
    X = regional.finest_coordinates(levels)
    B = amg.rigid_body_modes(X)
    scale = abs(A).max() * np.abs(B).max()
    assert np.abs(A @ B).max() <= 1e-10 * scale, np.abs(A @ B).max() / scale
    # wrong positions do not: the coarsest lattice's own (uniform) indices, or x and y swapped
    n = L.lay.shape_xyz
    g = np.stack([a.reshape(-1) for a in np.meshgrid(*[np.arange(v) for v in n[::-1]], indexing="ij")[::-1]], axis=1)
    assert np.abs(A @ amg.rigid_body_modes(g.astype(float))).max() > 1e-3 * scale
    assert np.abs(A @ amg.rigid_body_modes(X[:, [1, 0, 2]])).max() > 1e-3 * scale


def test_tentative_prolongator_is_orthonormal_and_keeps_the_null_space():
    lay, coefs, opt, levels = elasticity_levels(0)
    L = levels[-1]
    A = sp.csr_matrix(assembly.assemble_from_regions(L.lay, L.coefs))
    B = amg.rigid_body_modes(regional.finest_coordinates(levels))
    nodes = np.arange(0, A.shape[0] + 1, 3)
    agg = amg.aggregates(amg.node_graph(A, nodes), np.ones(nodes.size - 1, dtype=bool))
    T, Bc = amg.tentative_system(agg, nodes, B)
    assert T.shape == (A.shape[0], 6 * (agg.max() + 1))
    np.testing.assert_allclose((T.T @ T).toarray(), np.eye(T.shape[1]), atol=1e-12)
    rows = np.repeat(agg >= 0, 3)
    np.testing.assert_allclose((T @ Bc)[rows], B[rows], rtol=0, atol=1e-12 * np.abs(B).max())


def test_node_graph_pattern():
    # 3 nodes of 2 dofs: block (0,1) large, block (0,2) tiny, block (1,2) zero
    A = np.eye(6) * 4.0
    A[0, 2] = A[2, 0] = 1.0
    A[1, 5] = A[5, 1] = 1e-15
    G = amg.node_graph(sp.csr_matrix(A), np.array([0, 2, 4, 6])).toarray()
    assert (G != 0).tolist() == [[True, True, False], [True, True, False], [False, False, True]]


def test_system_amg_cycle_and_region_pcg():
    lay, coefs, opt, levels = elasticity_levels(0b010101, nlevels=2, coarse_amg=True, coarse_size=100)
    L = levels[-1]
    assert L.amg is not None and len(L.amg) >= 2 and L.amg[0].agg.max() >= 9
    A = L.amg[0].A
    g = np.random.default_rng(3)
    x = g.standard_normal(A.shape[0]) * np.repeat(~L.lay.dirichlet.reshape(-1), 3)
    e0 = np.sqrt(x @ (A @ x))
    for _ in range(5):
        x = x - amg.vcycle(L.amg, A @ x)
    rate = (np.sqrt(x @ (A @ x)) / e0) ** (1 / 5)
    assert rate < 0.6, rate
    b = g.uniform(-1, 1, lay.shape + (3,))
    b[lay.dirichlet] = 0.0
    out = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-8, maxit=100)
    assert out.converged
