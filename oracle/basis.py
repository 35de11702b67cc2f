"""Local polynomial basis (oracle; test infrastructure).

V_h is the space of piecewise polynomials of total degree p in the physical
frame (Sec. 2, definition of V_h). The paper leaves the basis open; the
reading used here is the tensor Legendre family restricted to total degree,
scaled to be orthonormal on the cell's axis-aligned bounding box B:

  phi_ij(x, y) = sqrt((2i+1)(2j+1) / (dx dy)) L_i(2(x-xc)/dx) L_j(2(y-yc)/dy),
  i + j <= p, ordered by degree d = 0..p, then j = 0..d with i = d - j.

The coarse space V_0 uses the same construction on coarse-cell boxes with
degree q.

Pins: orthonormality on a rectangle (mass matrix = I), span = P_p checked by
exact reproduction of monomials through an L2 fit.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def index_pairs(p: int):
    return [(d - j, j) for d in range(p + 1) for j in range(d + 1)]


def n_basis(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def _legendre_table(p: int, t: np.ndarray):
    """L_k(t) and L_k'(t) for k = 0..p, shape [p+1, *t.shape]."""
    val = np.empty((p + 1,) + t.shape)
    der = np.empty((p + 1,) + t.shape)
    for k in range(p + 1):
        c = np.zeros(k + 1)
        c[k] = 1.0
        val[k] = npleg.legval(t, c)
        der[k] = npleg.legval(t, npleg.legder(c)) if k > 0 else 0.0
    return val, der


def eval_basis(p: int, box: np.ndarray, pts: np.ndarray):
    """Values [..., n_p] and gradients [..., n_p, 2] at pts [..., 2].

    box broadcasts against pts[..., 0]: shape [..., 4] = xmin, xmax, ymin, ymax."""
    box = np.asarray(box, dtype=np.float64)
    dx = (box[..., 1] - box[..., 0])
    dy = (box[..., 3] - box[..., 2])
    xc = 0.5 * (box[..., 1] + box[..., 0])
    yc = 0.5 * (box[..., 3] + box[..., 2])
    xi = 2.0 * (pts[..., 0] - xc) / dx
    eta = 2.0 * (pts[..., 1] - yc) / dy
    Lx, dLx = _legendre_table(p, xi)
    Ly, dLy = _legendre_table(p, eta)
    pairs = index_pairs(p)
    val = np.empty(pts.shape[:-1] + (len(pairs),))
    grad = np.empty(pts.shape[:-1] + (len(pairs), 2))
    for a, (i, j) in enumerate(pairs):
        s = np.sqrt((2 * i + 1) * (2 * j + 1) / (dx * dy))
        val[..., a] = s * Lx[i] * Ly[j]
        grad[..., a, 0] = s * dLx[i] * (2.0 / dx) * Ly[j]
        grad[..., a, 1] = s * Lx[i] * dLy[j] * (2.0 / dy)
    return val, grad
