"""Quadrature rules (oracle; test infrastructure).

The paper does not fix a quadrature. The reading used throughout: cells are
split into the triangles (area centroid, v_k, v_{k+1}); each triangle uses a
collapsed tensor Gauss-Legendre rule with m points per direction, exact for
total degree 2m-2; edges use m-point Gauss-Legendre (exact to 2m-1). With
m = p + 2 every bilinear form of the SIPG matrix is integrated exactly.

Pins: tests check exactness on monomial moments (1D closed form, polygon
moments by Green's theorem) and failure one degree beyond.
"""
from __future__ import annotations

import numpy as np


def gauss_legendre_01(m: int):
    """m-point Gauss-Legendre nodes and weights on [0, 1] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def collapsed_triangle_rule(m: int):
    """Reference rule in (s, t) in [0,1]^2 for the collapsed map
    X(s,t) = (1-s) a + s((1-t) b + t c), Jacobian 2|T| s.

    Returns (s, t, w) flattened with the Jacobian factor s folded into w
    (still to be multiplied by 2|T|)."""
    g, wg = gauss_legendre_01(m)
    S, T = np.meshgrid(g, g, indexing="ij")
    W = np.outer(wg, wg) * S
    return S.ravel(), T.ravel(), W.ravel()


def triangles_rule(a: np.ndarray, b: np.ndarray, c: np.ndarray, m: int):
    """Points [n_tri, m*m, 2] and weights [n_tri, m*m] on triangles (a, b, c).

    Weights carry the (unsigned) area, so orientation does not matter."""
    s, t, w = collapsed_triangle_rule(m)
    s = s[None, :, None]
    t = t[None, :, None]
    pts = (1.0 - s) * a[:, None, :] + s * ((1.0 - t) * b[:, None, :] + t * c[:, None, :])
    e1 = b - a
    e2 = c - a
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    return pts, 2.0 * area[:, None] * w[None, :]


def segments_rule(p0: np.ndarray, p1: np.ndarray, m: int):
    """Points [n_seg, m, 2] and weights [n_seg, m] (length included)."""
    g, wg = gauss_legendre_01(m)
    pts = p0[:, None, :] + g[None, :, None] * (p1 - p0)[:, None, :]
    length = np.linalg.norm(p1 - p0, axis=1)
    return pts, length[:, None] * wg[None, :]
