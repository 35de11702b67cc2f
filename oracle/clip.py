"""Convex polygon intersection (oracle; test infrastructure).

Needed for the L2 prolongation onto V_h from a coarse mesh that is not
nested in the fine one (Sec. 3, eq. (R0T)): the integrals over a fine cell
against a coarse basis function split into integrals over the pieces
kappa intersected with D_j. Voronoi cells are convex, so Sutherland-Hodgman
clipping of one convex polygon by another is exact up to rounding.

Pins: clipped areas of a fine cell against all coarse cells sum to the
fine-cell area, and over all fine cells to each coarse-cell area; clipping a
square by a square against the closed-form overlap rectangle.
"""
from __future__ import annotations

import numpy as np


def clip_convex(subject: np.ndarray, clipper: np.ndarray) -> np.ndarray:
    """Intersection of convex polygon ``subject`` with convex CCW ``clipper``.

    Both are [k, 2] vertex arrays; returns the (possibly empty) intersection
    polygon as an [m, 2] array in CCW order."""
    out = [np.asarray(v, dtype=np.float64) for v in subject]
    k = clipper.shape[0]
    for i in range(k):
        a = clipper[i]
        e = clipper[(i + 1) % k] - a
        inp = out
        out = []
        if not inp:
            break
        n = len(inp)
        for j in range(n):
            P = inp[j]
            Q = inp[(j + 1) % n]
            sP = e[0] * (P[1] - a[1]) - e[1] * (P[0] - a[0])
            sQ = e[0] * (Q[1] - a[1]) - e[1] * (Q[0] - a[0])
            if sP >= 0.0:
                out.append(P)
                if sQ < 0.0:
                    out.append(P + (Q - P) * (sP / (sP - sQ)))
            elif sQ >= 0.0:
                out.append(P + (Q - P) * (sP / (sP - sQ)))
    if len(out) < 3:
        return np.zeros((0, 2))
    return np.asarray(out)
