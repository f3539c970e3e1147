"""Learned prolongation weights (not in the paper; modelled on the paper's remark that
operator-dependent interpolation such as black-box multigrid produces stencils that must be
averaged over shared interfaces to satisfy the interpolation conditions of Section 3.2).

A coarse cell is the 3x3x3 block of fine elements between 2x2x2 coarse nodes; its 4x4x4 fine
nodes are the 8 coarse corners (injected), 24 edge nodes (interpolating from the 2 corners of
their edge), 24 face nodes (4 corners of their face) and 8 interior nodes (8 corners).
A small MLP (27 -> 64 -> 64 -> 208, ReLU) maps the centred log-coefficients of the cell's 27
elements to one logit per (node, corner) pair; a softmax over each node's corners gives
weights that sum to 1.  A fine node shared by several cells (faces, edges) takes the average
of their predictions, so co-located rows match across regions.

Storage of weights per fine node ("stored P"): 8 values for the corners (ix, iy, iz) of its
canonical cell c = min(x // 3, ncx - 2) per axis, slot ix + 2 iy + 4 iz.

Readings (spec variant, not the paper): loss per (cell, sample) =
sum_f (e_f - sum_c w_fc e_c)^2 / sum_f e_f^2 over the cell's 64 nodes, e a smooth error
produced by 20 applications of the method's own Chebyshev smoother to A e = 0 from a random
start (with only 4, the damped but not yet removed high frequencies of the random start still
carry most of the energy and even linear interpolation scores a loss near 1); Adam with beta1
0.9, beta2 0.999, eps 1e-8.  Parameter order of the flat vector: W1 (64x27), b1, W2 (64x64), b2, W3 (208x64), b3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem
from .regions import Layout

NIN, NH, NOUT = 27, 64, 208
NPARAM = NH * NIN + NH + NH * NH + NH + NOUT * NH + NOUT


def cell_nodes():
    """Non-corner fine nodes of a cell in x-fastest order: (i, j, k, corners), corners as slots."""
    out = []
    for k in range(4):
        for j in range(4):
            for i in range(4):
                c = (i, j, k)
                if all(v in (0, 3) for v in c):
                    continue
                opts = [((0, 1) if v in (1, 2) else ((0,) if v == 0 else (1,))) for v in c]
                corners = [ix + 2 * iy + 4 * iz for iz in opts[2] for iy in opts[1] for ix in opts[0]]
                out.append((i, j, k, corners))
    return out


NODES = cell_nodes()
LOGIT_OFFSET = np.cumsum([0] + [len(n[3]) for n in NODES])[:-1]
assert int(sum(len(n[3]) for n in NODES)) == NOUT and len(NODES) == 56


def unpack(theta):
    o = 0
    W1 = theta[o:o + NH * NIN].reshape(NH, NIN); o += NH * NIN
    b1 = theta[o:o + NH]; o += NH
    W2 = theta[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = theta[o:o + NH]; o += NH
    W3 = theta[o:o + NOUT * NH].reshape(NOUT, NH); o += NOUT * NH
    b3 = theta[o:o + NOUT]; o += NOUT
    return W1, b1, W2, b2, W3, b3


def forward(theta, X):
    """Logits (N, 208) and the activations needed by the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64))
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (X, a1, h1, a2, h2)


def weights_from_logits(z):
    """Per-node softmax: list over the 56 nodes of arrays (N, ncorners)."""
    out = []
    for n, (_, _, _, corners) in enumerate(NODES):
        s = z[:, LOGIT_OFFSET[n]:LOGIT_OFFSET[n] + len(corners)]
        s = s - s.max(axis=1, keepdims=True)
        e = np.exp(s)
        out.append(e / e.sum(axis=1, keepdims=True))
    return out


def corner_values(E):
    """E: (N, 4, 4, 4) cell node values [k, j, i] -> coarse corner values (N, 8), slot ix+2iy+4iz."""
    return np.stack([E[:, 3 * ((s >> 2) & 1), 3 * ((s >> 1) & 1), 3 * (s & 1)] for s in range(8)], axis=1)


def cell_matrix(X):
    """Local operator of a cell for the energy loss: sum over its 27 elements of c_e K_e, with
    c_e = exp(X_e) (the centred log-coefficients; the loss is a ratio, so the common scale drops
    out) and K_e the Q1 Laplace element matrix of a unit cube, on the 64 cell nodes [k, j, i]
    flattened x fastest.  Returns (N, 64, 64)."""
    K = fem.q1_laplace(1.0)
    N = X.shape[0]
    A = np.zeros((N, 64, 64))
    for e in range(27):
        ex, ey, ez = e % 3, (e // 3) % 3, e // 9
        nodes = [(ez + c[2]) * 16 + (ey + c[1]) * 4 + (ex + c[0]) for c in fem.CORNERS3]
        A[:, np.ix_(nodes, nodes)[0], np.ix_(nodes, nodes)[1]] += np.exp(X[:, e])[:, None, None] * K[None]
    return A


def loss_and_grad(theta, X, E, kind="l2"):
    """Mean loss over samples and its gradient (flat, same order as theta).

    X: (N, 27) features, E: (N, 4, 4, 4) smooth-error values on the cell's nodes [k, j, i].
    kind "l2": per sample sum_f (e_f - sum_c w_fc e_c)^2 / sum_f e_f^2.
    kind "energy": the interpolation error delta (zero at the corners) in the cell operator's
    energy norm, delta^T A_cell delta / (cbar sum_f e_f^2), cbar the mean element coefficient.
    """
    z, (X, a1, h1, a2, h2) = forward(theta, X)
    N = X.shape[0]
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64))
    ec = corner_values(E)
    norm = np.sum(E.reshape(N, -1) ** 2, axis=1)
    norm = np.where(norm > 0, norm, 1.0)
    ws = weights_from_logits(z)
    dz = np.zeros_like(z)
    # interpolation error on the 64 cell nodes (zero at the corners)
    delta = np.zeros((N, 64))
    for n, (i, j, k, corners) in enumerate(NODES):
        pred = np.sum(ws[n] * ec[:, corners], axis=1)
        delta[:, (k * 4 + j) * 4 + i] = E[:, k, j, i] - pred
    if kind == "l2":
        loss = np.sum(delta ** 2, axis=1) / norm
        g = 2.0 * delta / norm[:, None]  # d loss / d delta
    elif kind == "energy":
        A = cell_matrix(X)
        Ad = np.einsum("nij,nj->ni", A, delta)
        enorm = np.mean(np.exp(X), axis=1) * norm
        loss = np.sum(delta * Ad, axis=1) / enorm
        g = 2.0 * Ad / enorm[:, None]
    else:
        raise ValueError(kind)
    for n, (i, j, k, corners) in enumerate(NODES):
        w = ws[n]
        # d loss / d pred_f = -g_f ; d pred / d w_c = e_c ; softmax backward
        dpred = -g[:, (k * 4 + j) * 4 + i]
        dw = dpred[:, None] * ec[:, corners]
        s = np.sum(dw * w, axis=1, keepdims=True)
        dz[:, LOGIT_OFFSET[n]:LOGIT_OFFSET[n] + len(corners)] = w * (dw - s)
    L = float(np.mean(loss))
    dz /= N
    dW3 = dz.T @ h2
    db3 = dz.sum(axis=0)
    dh2 = dz @ W3
    da2 = dh2 * (a2 > 0)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    dW1 = da1.T @ X
    db1 = da1.sum(axis=0)
    grad = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return L, grad


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), t counted from 1; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------- features
def cell_features(lay: Layout, elem_coef):
    """Centred log-coefficients of every coarse cell, region by region, cells x-fastest.

    Returns X (ncells, 27) with element order x-fastest inside the cell, and a list of
    (region, cx, cy, cz) per row.
    """
    rows, ids = [], []
    logc = np.log(np.asarray(elem_coef, dtype=np.float64))
    for k in range(lay.nreg):
        o, e = lay.origins[k], lay.extents[k]
        nc = [(int(e[d]) - 1) // 3 for d in range(3)]
        for cz in range(nc[2]):
            for cy in range(nc[1]):
                for cx in range(nc[0]):
                    x0, y0, z0 = int(o[0]) + 3 * cx, int(o[1]) + 3 * cy, int(o[2]) + 3 * cz
                    patch = logc[z0:z0 + 3, y0:y0 + 3, x0:x0 + 3].reshape(-1)
                    rows.append(patch - patch.mean())
                    ids.append((k, cx, cy, cz))
    return np.asarray(rows), ids


def cell_values(lay: Layout, comp, ids):
    """Composite nodal values on the 4x4x4 nodes of each cell: (ncells, 4, 4, 4) [k, j, i]."""
    out = np.zeros((len(ids), 4, 4, 4))
    for r, (k, cx, cy, cz) in enumerate(ids):
        o = lay.origins[k]
        x0, y0, z0 = int(o[0]) + 3 * cx, int(o[1]) + 3 * cy, int(o[2]) + 3 * cz
        out[r] = comp[z0:z0 + 4, y0:y0 + 4, x0:x0 + 4]
    return out


# ----------------------------------------------------------- assembly of P
def node_weights(lay: Layout, coarse: Layout, theta, elem_coef):
    """Stored-P weights of the finest level: list per region of arrays (ez, ey, ex, 8).

    Cell predictions are averaged over all cells (in any region) containing a fine node,
    coarse corner nodes are injected, and weights from Dirichlet coarse nodes to free fine
    nodes are dropped.
    """
    X, ids = cell_features(lay, elem_coef)
    z, _ = forward(theta, X)
    ws = weights_from_logits(z)
    # accumulate per composite fine node: sum of predicted weights over its composite corners
    shape = lay.shape
    acc = {}
    for r, (k, cx, cy, cz) in enumerate(ids):
        o = lay.origins[k]
        X0, Y0, Z0 = int(o[0]) + 3 * cx, int(o[1]) + 3 * cy, int(o[2]) + 3 * cz
        for n, (i, j, kk, corners) in enumerate(NODES):
            key = (Z0 + kk, Y0 + j, X0 + i)
            for c_slot, w in zip(corners, ws[n][r]):
                C = (Z0 // 3 + ((c_slot >> 2) & 1), Y0 // 3 + ((c_slot >> 1) & 1), X0 // 3 + (c_slot & 1))
                d = acc.setdefault(key, {})
                d[C] = d.get(C, 0.0) + w
    count = {}
    for r, (k, cx, cy, cz) in enumerate(ids):
        o = lay.origins[k]
        X0, Y0, Z0 = int(o[0]) + 3 * cx, int(o[1]) + 3 * cy, int(o[2]) + 3 * cz
        for (i, j, kk, _) in NODES:
            key = (Z0 + kk, Y0 + j, X0 + i)
            count[key] = count.get(key, 0) + 1
    out = []
    for k in range(lay.nreg):
        o, e = lay.origins[k], lay.extents[k]
        ez, ey, ex = int(e[2]), int(e[1]), int(e[0])
        ncx = [(int(e[d]) - 1) // 3 + 1 for d in range(3)]
        W = np.zeros((ez, ey, ex, 8))
        for z in range(ez):
            for y in range(ey):
                for x in range(ex):
                    G = (int(o[2]) + z, int(o[1]) + y, int(o[0]) + x)
                    cell = [min(v // 3, ncx[d] - 2) for d, v in enumerate((x, y, z))]
                    base = (int(o[2]) // 3 + cell[2], int(o[1]) // 3 + cell[1], int(o[0]) // 3 + cell[0])
                    if x % 3 == 0 and y % 3 == 0 and z % 3 == 0:
                        C = (int(o[2]) // 3 + z // 3, int(o[1]) // 3 + y // 3, int(o[0]) // 3 + x // 3)
                        wts = {C: 1.0}
                    else:
                        wts = {C: v / count[G] for C, v in acc[G].items()}
                    fdir = lay.dirichlet[G]
                    for C, v in wts.items():
                        slot = (C[2] - base[2]) + 2 * (C[1] - base[1]) + 4 * (C[0] - base[0])
                        if not fdir and coarse.dirichlet[C]:
                            continue
                        W[z, y, x, slot] = v
        out.append(W)
    return out


def stored_prolongator(fine: Layout, coarse: Layout, k, W):
    """Region k's block of P from stored weights W (ez, ey, ex, 8) (scalar problems)."""
    o, e = fine.origins[k], fine.extents[k]
    ez, ey, ex = int(e[2]), int(e[1]), int(e[0])
    cshape = coarse.region_shape(k)
    ncx = [(int(e[d]) - 1) // 3 + 1 for d in range(3)]
    rows, cols, vals = [], [], []
    for z in range(ez):
        for y in range(ey):
            for x in range(ex):
                cell = [min(v // 3, ncx[d] - 2) for d, v in enumerate((x, y, z))]
                f = (z * ey + y) * ex + x
                for slot in range(8):
                    v = W[z, y, x, slot]
                    if v == 0.0:
                        continue
                    cx, cy, cz = cell[0] + (slot & 1), cell[1] + ((slot >> 1) & 1), cell[2] + ((slot >> 2) & 1)
                    rows.append(f)
                    cols.append((cz * cshape[1] + cy) * cshape[2] + cx)
                    vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(ez * ey * ex, int(np.prod(cshape))))


def geometric_weights(fine: Layout, coarse: Layout):
    """Stored-P weights equal to the geometric linear interpolation (with the Dirichlet rule)."""
    out = []
    for k in range(fine.nreg):
        o, e = fine.origins[k], fine.extents[k]
        ez, ey, ex = int(e[2]), int(e[1]), int(e[0])
        ncx = [(int(e[d]) - 1) // 3 + 1 for d in range(3)]
        W = np.zeros((ez, ey, ex, 8))
        for z in range(ez):
            for y in range(ey):
                for x in range(ex):
                    cell = [min(v // 3, ncx[d] - 2) for d, v in enumerate((x, y, z))]
                    t = [v - 3 * c for v, c in zip((x, y, z), cell)]
                    fdir = fine.dirichlet[int(o[2]) + z, int(o[1]) + y, int(o[0]) + x]
                    for slot in range(8):
                        b = (slot & 1, (slot >> 1) & 1, (slot >> 2) & 1)
                        w = 1.0
                        for d in range(3):
                            w *= (t[d] / 3.0) if b[d] else ((3 - t[d]) / 3.0)
                        if w == 0.0:
                            continue
                        C = (int(o[2]) // 3 + cell[2] + b[2], int(o[1]) // 3 + cell[1] + b[1],
                             int(o[0]) // 3 + cell[0] + b[0])
                        if not fdir and coarse.dirichlet[C]:
                            continue
                        W[z, y, x, slot] = w
        out.append(W)
    return out


def smooth_errors(levels, opt, nsamples, seed, sweeps=20):
    """Smooth errors e = S^sweeps e0 of the finest level (b = 0), composite arrays.

    e0: counter-based uniform values (stream 32 + sample of the SplitMix64 generator), zero on
    Dirichlet nodes; S = one degree-K Chebyshev application from the current iterate.
    """
    from . import regional, rng

    L = levels[0]
    lay = L.lay
    zero = lay.zeros_regional()
    out = []
    for s in range(nsamples):
        e0 = rng.uniform_pm1(lay.n_composite, 32 + s, seed).reshape(lay.shape)
        e0[lay.dirichlet] = 0.0
        e = lay.to_regional(e0)
        for _ in range(sweeps):
            e = regional.chebyshev(L, e, zero, L.residual(zero, e), opt)
        out.append(lay.to_composite_owner(e))
    return out


def training_set(lay, levels, opt, elem_coef, nsamples, seed, sweeps=20):
    """(X, E): features repeated per sample and the cell values of each smooth error."""
    X, ids = cell_features(lay, elem_coef)
    Xs, Es = [], []
    for e in smooth_errors(levels, opt, nsamples, seed, sweeps):
        Xs.append(X)
        Es.append(cell_values(lay, e, ids))
    return np.concatenate(Xs), np.concatenate(Es)
