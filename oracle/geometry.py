"""Polygon geometry and mesh faces (oracle; test infrastructure).

Follows the mesh notation of Sec. 2: cells kappa with diameter h_kappa,
faces F = polygon edges, interior faces shared by kappa+ and kappa-,
boundary faces on the boundary of the domain, outward unit normals.

Pins: area/centroid against closed forms on rectangles and triangles;
face extraction against the edge-count invariant (every interior edge is
shared by exactly two cells, boundary edges lie on the square's sides).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class CellGeometry:
    area: np.ndarray      # [N]
    centroid: np.ndarray  # [N, 2] area centroid
    diam: np.ndarray      # [N] max vertex-vertex distance (convex cells)
    box: np.ndarray       # [N, 4] xmin, xmax, ymin, ymax


def polygon_area_centroid(P: np.ndarray):
    """Shoelace area (signed, CCW positive) and area centroid of one polygon."""
    x, y = P[:, 0], P[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    a = 0.5 * cr.sum()
    cx = ((x + xn) * cr).sum() / (6.0 * a)
    cy = ((y + yn) * cr).sum() / (6.0 * a)
    return a, np.array([cx, cy])


def cell_geometry(mesh) -> CellGeometry:
    n = mesh.n_cells
    area = np.empty(n)
    cen = np.empty((n, 2))
    diam = np.empty(n)
    box = np.empty((n, 4))
    for k in range(n):
        P = mesh.xy[mesh.cell(k)]
        a, c = polygon_area_centroid(P)
        area[k] = a
        cen[k] = c
        d = P[:, None, :] - P[None, :, :]
        diam[k] = np.sqrt((d ** 2).sum(-1)).max()
        box[k] = [P[:, 0].min(), P[:, 0].max(), P[:, 1].min(), P[:, 1].max()]
    return CellGeometry(area, cen, diam, box)


@dataclasses.dataclass
class Faces:
    """Interior faces: plus/minus cells; boundary faces: minus = -1.
    Endpoints v0 -> v1 follow the CCW order of the plus cell, so the normal
    (dy, -dx)/|F| is the outward normal of the plus cell."""

    plus: np.ndarray
    minus: np.ndarray
    v0: np.ndarray
    v1: np.ndarray


def mesh_faces(mesh, boundary_tol: float = 1e-12) -> Faces:
    seen = {}
    plus, minus, v0s, v1s = [], [], [], []
    for k in range(mesh.n_cells):
        vs = mesh.cell(k)
        for i in range(len(vs)):
            a, b = int(vs[i]), int(vs[(i + 1) % len(vs)])
            key = (min(a, b), max(a, b))
            if key in seen:
                fidx = seen.pop(key)
                if minus[fidx] != -1:
                    raise ValueError("edge shared by more than two cells")
                minus[fidx] = k
            else:
                seen[key] = len(plus)
                plus.append(k)
                minus.append(-1)
                v0s.append(a)
                v1s.append(b)
    plus = np.asarray(plus)
    minus = np.asarray(minus)
    v0s = np.asarray(v0s)
    v1s = np.asarray(v1s)
    # every unmatched edge must lie on the boundary of the unit square
    bd = minus < 0
    P0, P1 = mesh.xy[v0s[bd]], mesh.xy[v1s[bd]]
    on_side = np.zeros(P0.shape[0], dtype=bool)
    for d in range(2):
        for s in (0.0, 1.0):
            on_side |= (np.abs(P0[:, d] - s) < boundary_tol) & (np.abs(P1[:, d] - s) < boundary_tol)
    if not on_side.all():
        raise ValueError("non-conforming mesh: unmatched edge inside the domain")
    return Faces(plus, minus, v0s, v1s)
