"""Element matrices for the model problems (paper Section 6.2: linear hexahedral
finite elements for Poisson and elasticity; Section 6.1: a 2D five-point Laplacian).

Q1 (trilinear) element on a cube of side h, node a = (ax, ay, az) in {0,1}^3
numbered a = ax + 2 ay + 4 az.  Integrals use 2x2x2 Gauss-Legendre points,
which integrate these polynomial integrands exactly.
"""
from __future__ import annotations

import itertools

import numpy as np

_G = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))  # Gauss points on [0, 1]
_W = 0.5  # Gauss weight on [0, 1]

CORNERS3 = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]


def _shape_grad(a, xi):
    """Gradient w.r.t. reference coordinates of the trilinear shape function of corner a."""
    f = [xi[d] if a[d] else 1.0 - xi[d] for d in range(3)]
    df = [1.0 if a[d] else -1.0 for d in range(3)]
    return np.array([df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]])


def _quadrature():
    for p in itertools.product(_G, _G, _G):
        yield np.array(p), _W ** 3


def q1_laplace(h: float = 1.0) -> np.ndarray:
    """8x8 stiffness matrix int grad(phi_a) . grad(phi_b) over a cube of side h."""
    K = np.zeros((8, 8))
    for xi, w in _quadrature():
        g = np.array([_shape_grad(a, xi) for a in CORNERS3]) / h  # physical gradients
        K += w * h ** 3 * (g @ g.T)
    return K


def lame(E: float, nu: float):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def q1_elasticity(E: float, nu: float, h: float = 1.0) -> np.ndarray:
    """24x24 isotropic linear-elastic stiffness, dofs ordered (node a, component i) -> 3a+i.

    Textbook B^T D B form with Voigt strains (xx, yy, zz, yz, xz, xy).
    """
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    K = np.zeros((24, 24))
    for xi, w in _quadrature():
        B = np.zeros((6, 24))
        for a, c in enumerate(CORNERS3):
            gx, gy, gz = _shape_grad(c, xi) / h
            B[0, 3 * a + 0] = gx
            B[1, 3 * a + 1] = gy
            B[2, 3 * a + 2] = gz
            B[3, 3 * a + 1] = gz
            B[3, 3 * a + 2] = gy
            B[4, 3 * a + 0] = gz
            B[4, 3 * a + 2] = gx
            B[5, 3 * a + 0] = gy
            B[5, 3 * a + 1] = gx
        K += w * h ** 3 * (B.T @ D @ B)
    return K


def fd5_offsets():
    """Five-point Laplacian [4; -1 x 4] (mesh-size factor dropped): offset -> value."""
    return {(0, 0): 4.0, (-1, 0): -1.0, (1, 0): -1.0, (0, -1): -1.0, (0, 1): -1.0}
