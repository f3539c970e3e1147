"""Non-invasive construction from an assembled composite CSR matrix (Section 4): the device split
into region matrices against the oracle's split of the same matrix, the solve on the split
operator, and the input errors."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from tests import harness

pytestmark = pytest.mark.gpu

CASES = [("c1_small", 5), ("c2_small", 27), ("c5_small", 27), ("c4_small", 27)]


def composite_matrix(w, lay):
    from oracle import assembly

    if w.pde == "fd5":
        return assembly.composite_fd5(lay)
    ec = synth.jump_coefficients(w) if w.pde == "diffusion" else None
    return assembly.composite_q1(lay, w.pde, h=w.h, elem_coef=ec)


@pytest.mark.parametrize("name,npts", CASES, ids=[c[0] for c in CASES])
def test_csr_split_and_solve(hip_device, name, npts):
    import torch

    from oracle import assembly, regional
    from oracle.regions import Layout
    from paper_2103_11962_amd import regmg

    w = synth.workload(name)
    lay = Layout(w.dim, w.origins, w.extents, w.dirichlet_mask)
    A = composite_matrix(w, lay)
    coefs = assembly.split_composite(lay, A)
    A = sp.csr_matrix(A)  # the matrix as an application hands it over
    h = regmg.Handle(0)
    h.build_regions(w.dim, w.ndof, w.extents, w.origins, w.dirichlet_mask)
    h.set_composite_csr(npts, A)
    h.setup_hierarchy(nlevels=w.nlevels, cheb_degree=w.cheb_degree)
    for k in range(lay.nreg):
        ref = coefs[k].reshape(coefs[k].shape[0], -1)
        got = h.level_stencil(0, k, npts, ref.shape[1])
        if npts == 5:  # the oracle stores five-point rows in the 9-point order
            ref = ref[[1, 3, 4, 5, 7]]
        harness.assert_close(got, ref, 1e-14, what=repr(k))
    opt = regional.Options(nlevels=w.nlevels, degree=w.cheb_degree)
    levels = regional.setup(lay, coefs, opt)
    b = synth.rhs(w)
    ref = regional.pcg(levels, lay.to_regional(b), opt, rtol=1e-8, maxit=100)
    x = torch.zeros(lay.n_composite, dtype=torch.float64, device="cuda:0")
    out = h.solve(harness.to_dev(b), x, rtol=1e-8, maxit=100)
    assert out["iterations"] == ref.iterations
    harness.assert_close(x.cpu().numpy(), lay.to_composite_owner(ref.x).reshape(-1), 1e-10)
    h.close()


def test_duplicate_entries_add_up(hip_device):
    from oracle import assembly
    from oracle.regions import Layout
    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    lay = Layout(w.dim, w.origins, w.extents, w.dirichlet_mask)
    A = sp.csr_matrix(composite_matrix(w, lay))
    coo = A.tocoo()
    half = coo.data / 2.0
    # every entry given twice, halves in reverse order
    D = sp.coo_matrix((np.concatenate([half, half[::-1]]),
                       (np.concatenate([coo.row, coo.row[::-1]]), np.concatenate([coo.col, coo.col[::-1]]))),
                      shape=A.shape)
    order = np.lexsort((np.arange(D.nnz), D.row))
    rows, cols, vals = D.row[order], D.col[order], D.data[order]
    indptr = np.searchsorted(rows, np.arange(A.shape[0] + 1))
    Dcsr = sp.csr_matrix((vals, cols, indptr), shape=A.shape)
    assert Dcsr.nnz == 2 * A.nnz  # duplicates kept
    h = regmg.Handle(0)
    h.build_regions(w.dim, w.ndof, w.extents, w.origins, w.dirichlet_mask)
    h.set_composite_csr(27, Dcsr)
    coefs = assembly.split_composite(lay, A)
    got = h.level_stencil(0, 0, 27, coefs[0][0].size)
    harness.assert_close(got, coefs[0].reshape(27, -1), 1e-14)
    h.close()


def test_csr_input_errors(hip_device):
    import ctypes

    from oracle.regions import Layout
    from paper_2103_11962_amd import regmg

    w = synth.workload("c2_small")
    lay = Layout(w.dim, w.origins, w.extents, w.dirichlet_mask)
    A = sp.csr_matrix(composite_matrix(w, lay)).tolil()
    h = regmg.Handle(0)
    h.build_regions(w.dim, w.ndof, w.extents, w.origins, w.dirichlet_mask)
    far = A.copy()
    far[5, 5 + 3] = -1.0  # a coupling two nodes away
    with pytest.raises(regmg.RmgError) as e:
        h.set_composite_csr(27, far.tocsr())
    assert e.value.status == "RMG_ERR_SHAPE"
    bad = A.tocsr()
    bad.data[7] = np.nan
    with pytest.raises(regmg.RmgError) as e:
        h.set_composite_csr(27, bad)
    assert e.value.status == "RMG_ERR_NUMERIC"
    # decreasing row pointers and out-of-range columns, through the C entry point directly
    good = A.tocsr()
    rp = np.ascontiguousarray(good.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(good.indices, dtype=np.int32)
    v = np.ascontiguousarray(good.data)
    rp_bad = rp.copy()
    rp_bad[10] = rp_bad[11] + 1
    ci_bad = ci.copy()
    ci_bad[3] = lay.n_composite + 7
    lib = regmg.load()
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    assert lib.rmg_set_composite_csr(h._h, 27, v.size, ptr(rp_bad), ptr(ci), ptr(v), 0) == 1
    assert lib.rmg_set_composite_csr(h._h, 27, v.size, ptr(rp), ptr(ci_bad), ptr(v), 0) == 1
    assert lib.rmg_set_composite_csr(h._h, 27, v.size + 1, ptr(rp), ptr(ci), ptr(v), 0) == 1
    h.close()
