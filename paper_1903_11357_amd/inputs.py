"""Seeded synthetic inputs for the two-level Schwarz PCG path.

This module produces problem data only: polygon meshes of the unit square,
subdomain partitions, coarse partitions (nested agglomerates or an
independent coarse polygon mesh), piecewise-constant coefficients and
right-hand-side functions. It contains none of the discretisation or solver
arithmetic; both the CPU oracle and the GPU library consume what it returns.

Random numbers come from ``numpy.random.default_rng(seed)``. For a Voronoi
mesh the N seed points are drawn first with ``rng.random((N, 2))`` and then
relaxed by two Lloyd steps; any further draws (coarse seeds, coefficients,
RHS coefficients) continue the same stream in that order.

The named workloads mirror the problem classes of the paper's experiments
(unit-square Poisson, Voronoi polygonal meshes, nested agglomerated and
independent non-nested coarse meshes, piecewise-constant coefficient jumps;
Sections 7.1-7.5) at sizes chosen for one GPU.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np


@dataclasses.dataclass
class Mesh:
    """Conforming polygon mesh: shared vertex ids, counter-clockwise cells."""

    xy: np.ndarray            # [n_vertices, 2] float64
    cell_ptr: np.ndarray      # [n_cells + 1] int32 CSR offsets
    cell_vertices: np.ndarray  # [cell_ptr[-1]] int32 vertex ids, CCW

    @property
    def n_cells(self) -> int:
        return int(self.cell_ptr.shape[0] - 1)

    @property
    def n_vertices(self) -> int:
        return int(self.xy.shape[0])

    def cell(self, k: int) -> np.ndarray:
        return self.cell_vertices[self.cell_ptr[k]:self.cell_ptr[k + 1]]

    def vertex_mean(self) -> np.ndarray:
        """Arithmetic mean of each cell's vertices (used only for binning)."""
        counts = np.diff(self.cell_ptr).astype(np.float64)
        owner = np.repeat(np.arange(self.n_cells), np.diff(self.cell_ptr))
        sx = np.bincount(owner, weights=self.xy[self.cell_vertices, 0], minlength=self.n_cells)
        sy = np.bincount(owner, weights=self.xy[self.cell_vertices, 1], minlength=self.n_cells)
        return np.stack([sx / counts, sy / counts], axis=1)


def square_mesh(nx: int, ny: Optional[int] = None) -> Mesh:
    """nx-by-ny uniform squares on (0,1)^2, cells ordered x-fastest."""
    ny = nx if ny is None else ny
    gx = np.linspace(0.0, 1.0, nx + 1)
    gy = np.linspace(0.0, 1.0, ny + 1)
    X, Y = np.meshgrid(gx, gy, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    cells = []
    for j in range(ny):
        for i in range(nx):
            v0 = j * (nx + 1) + i
            cells.append([v0, v0 + 1, v0 + nx + 2, v0 + nx + 1])
    cv = np.asarray(cells, dtype=np.int32).ravel()
    ptr = np.arange(0, 4 * nx * ny + 1, 4, dtype=np.int32)
    return Mesh(xy=xy, cell_ptr=ptr, cell_vertices=cv)


def _signed_area(xy: np.ndarray) -> float:
    x, y = xy[:, 0], xy[:, 1]
    return 0.5 * float(np.dot(x, np.roll(y, -1)) - np.dot(np.roll(x, -1), y))


def voronoi_mesh(seeds: np.ndarray, tol: float = 1e-12) -> Mesh:
    """Voronoi tessellation of the unit square from seed points.

    The seeds are mirrored across the four sides so that the cells of the
    original seeds are exactly the Voronoi cells clipped to the square.
    Coordinates within ``tol`` of 0 or 1 are snapped onto the boundary and
    vertices closer than ``tol`` are merged, so the result is conforming.
    """
    from scipy.spatial import Voronoi, cKDTree

    seeds = np.asarray(seeds, dtype=np.float64)
    n = seeds.shape[0]
    # Only seeds near a side need a mirror image. If every vertex of every
    # original cell then lies in the closed square, the cells equal those of
    # the fully mirrored set (inside the square a mirror image is never
    # closer than its original); otherwise fall back to mirroring all seeds.
    for margin in (min(1.0, 8.0 / math.sqrt(max(n, 1))), 1.0):
        parts = [seeds]
        for d, side in ((0, 0.0), (0, 1.0), (1, 0.0), (1, 1.0)):
            near = np.abs(seeds[:, d] - side) <= margin
            m = seeds[near].copy()
            m[:, d] = 2.0 * side - m[:, d]
            parts.append(m)
        vor = Voronoi(np.concatenate(parts))
        regions = [vor.regions[vor.point_region[i]] for i in range(n)]
        used = np.unique(np.concatenate([np.asarray(r, dtype=np.int64) for r in regions]))
        if used.size and used.min() < 0:
            continue
        v = vor.vertices[used]
        if v.min() >= -tol and v.max() <= 1.0 + tol:
            break
    else:
        raise RuntimeError("Voronoi clipping failed")
    xy = vor.vertices[used].copy()
    for d in range(2):
        xy[np.abs(xy[:, d]) < tol, d] = 0.0
        xy[np.abs(xy[:, d] - 1.0) < tol, d] = 1.0
    # merge near-coincident vertices (union-find over close pairs)
    parent = np.arange(xy.shape[0])
    pairs = cKDTree(xy).query_pairs(r=tol, output_type="ndarray")

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in pairs:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    root = parent.copy()
    while True:
        nxt = root[root]
        if np.array_equal(nxt, root):
            break
        root = nxt
    keep, new_id = np.unique(root, return_inverse=True)
    xy = xy[keep]
    remap = np.full(vor.vertices.shape[0], -1, dtype=np.int64)
    remap[used] = new_id

    ptr = [0]
    verts = []
    for r in regions:
        ids = remap[np.asarray(r, dtype=np.int64)]
        # drop consecutive duplicates produced by merging
        out = [int(ids[0])]
        for v in ids[1:]:
            if v != out[-1]:
                out.append(int(v))
        while len(out) > 1 and out[-1] == out[0]:
            out.pop()
        if len(out) < 3:
            raise RuntimeError("degenerate Voronoi cell")
        if _signed_area(xy[out]) < 0.0:
            out.reverse()
        verts.extend(out)
        ptr.append(len(verts))
    return Mesh(xy=xy, cell_ptr=np.asarray(ptr, dtype=np.int32),
                cell_vertices=np.asarray(verts, dtype=np.int32))


LLOYD_STEPS = 2


def _cell_centroids(mesh: Mesh) -> np.ndarray:
    """Area centroids of all cells (shoelace), used by the Lloyd step."""
    xy, cv, ptr = mesh.xy, mesh.cell_vertices, mesh.cell_ptr
    N = mesh.n_cells
    owner = np.repeat(np.arange(N), np.diff(ptr))
    nxt = np.arange(cv.shape[0]) + 1
    nxt[ptr[1:] - 1] = ptr[:-1]
    a, b = xy[cv], xy[cv[nxt]]
    cr = a[:, 0] * b[:, 1] - b[:, 0] * a[:, 1]
    area = 0.5 * np.bincount(owner, cr, N)
    cx = np.bincount(owner, (a[:, 0] + b[:, 0]) * cr, N) / (6.0 * area)
    cy = np.bincount(owner, (a[:, 1] + b[:, 1]) * cr, N) / (6.0 * area)
    return np.stack([cx, cy], axis=1)


def relaxed_voronoi_mesh(seeds: np.ndarray, steps: int = LLOYD_STEPS) -> Mesh:
    """Voronoi mesh after ``steps`` Lloyd iterations (seeds moved to the area
    centroids of their cells). Uniform random seeds give occasional sliver
    cells whose trace-inverse constant is far outside the shape-regularity
    the method assumes; two Lloyd steps remove them while keeping the mesh
    random."""
    mesh = voronoi_mesh(seeds)
    for _ in range(steps):
        mesh = voronoi_mesh(_cell_centroids(mesh))
    return mesh


def bins_partition(points: np.ndarray, bx: int, by: int) -> np.ndarray:
    """Cell -> bin id for a bx-by-by grid of bins over (0,1)^2 (x-fastest)."""
    ix = np.minimum(np.floor(points[:, 0] * bx).astype(np.int64), bx - 1)
    iy = np.minimum(np.floor(points[:, 1] * by).astype(np.int64), by - 1)
    return (iy * bx + ix).astype(np.int32)


def warped_bins_256(points: np.ndarray) -> np.ndarray:
    """256 uneven subdomains: 16x16 bins of (x^2, y), with the first column
    split at x = 1/8 and the last two columns merged (16 columns remain)."""
    w = points[:, 0] ** 2
    col = np.minimum(np.floor(w * 16).astype(np.int64), 15)
    # first column split in two halves in x, shift the others right by one
    col = np.where(col == 0, np.where(points[:, 0] < 0.125, 0, 1), col + 1)
    col = np.minimum(col, 15)  # columns 15 and 16 (old 14, 15) merge
    row = np.minimum(np.floor(points[:, 1] * 16).astype(np.int64), 15)
    return (row * 16 + col).astype(np.int32)


def block_partition_squares(nx: int, block: int) -> np.ndarray:
    """Partition of an nx-by-nx square mesh into block-by-block agglomerates."""
    nb = nx // block
    ids = np.empty(nx * nx, dtype=np.int32)
    for j in range(nx):
        for i in range(nx):
            ids[j * nx + i] = (j // block) * nb + (i // block)
    return ids


def compact_labels(labels: np.ndarray) -> np.ndarray:
    """Relabel to 0..k-1 (drops empty bins), preserving label order."""
    _, inv = np.unique(labels, return_inverse=True)
    return inv.astype(np.int32)


# ---------------------------------------------------------------- RHS data
def f_sinsin(xy: np.ndarray) -> np.ndarray:
    """f = 2 pi^2 sin(pi x) sin(pi y), the load of u = sin(pi x) sin(pi y)."""
    return 2.0 * math.pi ** 2 * np.sin(math.pi * xy[:, 0]) * np.sin(math.pi * xy[:, 1])


def u_sinsin(xy: np.ndarray) -> np.ndarray:
    return np.sin(math.pi * xy[:, 0]) * np.sin(math.pi * xy[:, 1])


def grad_u_sinsin(xy: np.ndarray) -> np.ndarray:
    x, y = xy[:, 0], xy[:, 1]
    return math.pi * np.stack([np.cos(math.pi * x) * np.sin(math.pi * y),
                               np.sin(math.pi * x) * np.cos(math.pi * y)], axis=1)


def f_one(xy: np.ndarray) -> np.ndarray:
    return np.ones(xy.shape[0])


class SineSeries:
    """f = sum_{k,l=1..K} c_kl sin(k pi x) sin(l pi y) (picklable)."""

    def __init__(self, coef):
        self.coef = np.asarray(coef, dtype=np.float64)

    @staticmethod
    def _sines(t: np.ndarray, K: int) -> np.ndarray:
        """[K, n] with row k-1 = sin(k pi t), by the three-term recurrence
        sin((k+1)a) = 2 cos(a) sin(ka) - sin((k-1)a): one sin and one cos per
        point instead of K sines."""
        a = math.pi * t
        out = np.empty((K, t.shape[0]))
        out[0] = np.sin(a)
        if K > 1:
            c2 = 2.0 * np.cos(a)
            np.multiply(c2, out[0], out=out[1])
            for k in range(2, K):
                np.multiply(c2, out[k - 1], out=out[k])
                out[k] -= out[k - 2]
        return out

    @property
    def sine_series_coef(self) -> np.ndarray:
        """[K, L] coefficients (lets the library evaluate the series natively)."""
        return self.coef

    def __call__(self, xy: np.ndarray) -> np.ndarray:
        sx = self._sines(np.ascontiguousarray(xy[:, 0]), self.coef.shape[0])
        sy = self._sines(np.ascontiguousarray(xy[:, 1]), self.coef.shape[1])
        t = self.coef @ sy  # [K, n]: sum_l c_kl sin(l pi y)
        t *= sx
        return t.sum(axis=0)


def make_f_series(coef: np.ndarray) -> Callable[[np.ndarray], np.ndarray]:
    return SineSeries(coef)


# ------------------------------------------------------------- workloads
@dataclasses.dataclass
class Problem:
    """Everything the method takes as input."""

    name: str
    mesh: Mesh
    p: int
    c_sigma: float
    rho: np.ndarray                 # [n_cells] float64, piecewise constant
    subdomain: np.ndarray           # [n_cells] int32 in 0..n_sub-1
    q: int
    coarse_of_cell: Optional[np.ndarray]   # nested: [n_cells] int32
    coarse_mesh: Optional[Mesh]            # non-nested: independent mesh
    f: Callable[[np.ndarray], np.ndarray]
    rtol: float = 1e-8
    max_iter: int = 20000

    @property
    def n_sub(self) -> int:
        return int(self.subdomain.max()) + 1

    @property
    def dim(self) -> int:
        return getattr(self.mesh, "dim", 2)

    @property
    def n_p(self) -> int:
        if self.dim == 3:
            return (self.p + 1) * (self.p + 2) * (self.p + 3) // 6
        return (self.p + 1) * (self.p + 2) // 2

    @property
    def n_dofs(self) -> int:
        return self.mesh.n_cells * self.n_p


def squares_problem(nx: int, p: int, sub_block: int, coarse_block: Optional[int],
                    q: Optional[int] = None, c_sigma: float = 10.0,
                    f=f_sinsin, name: str = "squares") -> Problem:
    """nx-by-nx squares; subdomains of sub_block^2 cells; nested coarse of
    coarse_block^2 cells (None: one coarse cell per subdomain)."""
    mesh = square_mesh(nx)
    sub = block_partition_squares(nx, sub_block)
    coarse = block_partition_squares(nx, coarse_block if coarse_block else sub_block)
    return Problem(name=name, mesh=mesh, p=p, c_sigma=c_sigma,
                   rho=np.ones(mesh.n_cells), subdomain=sub,
                   q=p if q is None else q, coarse_of_cell=coarse, coarse_mesh=None, f=f)


def voronoi_problem(n_cells: int, seed: int, p: int, bx: int, by: int, q: int,
                    nonnested_coarse: int = 0, log10_rho_range: float = 0.0,
                    f=f_sinsin, warped: bool = False, name: str = "voronoi") -> Problem:
    rng = np.random.default_rng(seed)
    mesh = relaxed_voronoi_mesh(rng.random((n_cells, 2)))
    coarse_mesh = None
    if nonnested_coarse:
        coarse_mesh = relaxed_voronoi_mesh(rng.random((nonnested_coarse, 2)))
    pts = mesh.vertex_mean()
    sub = warped_bins_256(pts) if warped else bins_partition(pts, bx, by)
    sub = compact_labels(sub)
    n_sub = int(sub.max()) + 1
    if log10_rho_range > 0.0:
        rho_sub = 10.0 ** rng.uniform(-log10_rho_range, log10_rho_range, size=n_sub)
        rho = rho_sub[sub]
    else:
        rho = np.ones(mesh.n_cells)
    return Problem(name=name, mesh=mesh, p=p, c_sigma=10.0, rho=rho, subdomain=sub,
                   q=q, coarse_of_cell=None if coarse_mesh is not None else sub.copy(),
                   coarse_mesh=coarse_mesh, f=f)


# ---------------------------------------------------------------- 3D (tetrahedra)
@dataclasses.dataclass
class TetMesh:
    """Conforming tetrahedral mesh: shared vertex ids, four per cell."""

    xyz: np.ndarray   # [n_vertices, 3] float64
    tets: np.ndarray  # [n_cells, 4] int32
    dim: int = 3

    @property
    def n_cells(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(self.xyz.shape[0])

    def vertex_mean(self) -> np.ndarray:
        return self.xyz[self.tets].mean(axis=1)


# the six orderings of the axes; Kuhn simplex s of a cube walks from its
# lowest to its highest corner along the axes in the order KUHN[s]
KUHN = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def cube_tet_mesh(n: int, jitter: float = 0.0, seed: int = 0) -> TetMesh:
    """The unit cube as n^3 cubes of 6 Kuhn tetrahedra each (6 n^3 cells;
    cell 6 c + s is simplex s of cube c = (k n + j) n + i). Kuhn
    triangulations of the n- and 2n-grids are nested, so the tetrahedra of
    a coarser grid are agglomerates of finer ones. jitter > 0 moves interior
    vertices by U[-jitter, jitter] h per coordinate (h = 1/n)."""
    g = np.arange(n + 1) / n
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        inner = np.all((xyz > 0.5 / n) & (xyz < 1.0 - 0.5 / n), axis=1)
        xyz[inner] += rng.uniform(-jitter, jitter, size=(int(inner.sum()), 3)) / n

    def vid(i, j, k):
        return (k * (n + 1) + j) * (n + 1) + i

    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i0, j0, k0 = kk.ravel(), jj.ravel(), ii.ravel()  # cube c = (k n + j) n + i
    order = np.argsort((k0 * n + j0) * n + i0, kind="stable")
    i0, j0, k0 = i0[order], j0[order], k0[order]
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for s, ax in enumerate(KUHN):
        c = np.stack([i0, j0, k0], axis=1)
        verts = [vid(c[:, 0], c[:, 1], c[:, 2])]
        for a in ax:
            c = c.copy()
            c[:, a] += 1
            verts.append(vid(c[:, 0], c[:, 1], c[:, 2]))
        tets[:, s, :] = np.stack(verts, axis=1)
    tets = tets.reshape(-1, 4)
    P = xyz[tets]
    det = np.einsum("ij,ij->i", np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), P[:, 3] - P[:, 0])
    flip = det < 0
    tets[flip, 1], tets[flip, 2] = tets[flip, 2].copy(), tets[flip, 1].copy()
    if jitter > 0.0 and np.abs(det).min() < 0.2 / (6.0 * n ** 3):
        raise ValueError("jitter too large: a tetrahedron nearly degenerates")
    return TetMesh(xyz=xyz, tets=tets.astype(np.int32))


def kuhn_agglomerates(mesh: TetMesh, n_coarse: int) -> np.ndarray:
    """Coarse id of every tetrahedron: the Kuhn tetrahedron of the
    n_coarse-grid that contains its centroid (6 n_coarse^3 nested
    agglomerates when the fine grid refines the coarse one)."""
    c = mesh.vertex_mean() * n_coarse
    cube = np.minimum(np.floor(c).astype(np.int64), n_coarse - 1)
    fr = c - cube
    order = np.argsort(-fr, axis=1, kind="stable")  # axes by decreasing fractional part
    perm_id = {ax: s for s, ax in enumerate(KUHN)}
    s = np.array([perm_id[tuple(o)] for o in order.tolist()], dtype=np.int64)
    cid = (cube[:, 2] * n_coarse + cube[:, 1]) * n_coarse + cube[:, 0]
    return (6 * cid + s).astype(np.int32)


def box_agglomerates(mesh: TetMesh, b: int) -> np.ndarray:
    """Coarse id of every tetrahedron: its centroid's cell of a b^3 grid of
    boxes (non-empty boxes renumbered consecutively)."""
    c = np.minimum(np.floor(mesh.vertex_mean() * b).astype(np.int64), b - 1)
    return compact_labels(((c[:, 2] * b + c[:, 1]) * b + c[:, 0]).astype(np.int32))


def f_sin3(p: np.ndarray) -> np.ndarray:
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) (u = sin sin sin, rho = 1)."""
    return 3.0 * np.pi ** 2 * np.sin(np.pi * p[..., 0]) * np.sin(np.pi * p[..., 1]) * np.sin(np.pi * p[..., 2])


def u_sin3(p: np.ndarray) -> np.ndarray:
    return np.sin(np.pi * p[..., 0]) * np.sin(np.pi * p[..., 1]) * np.sin(np.pi * p[..., 2])


def grad_u_sin3(p: np.ndarray) -> np.ndarray:
    s = np.sin(np.pi * p)
    c = np.cos(np.pi * p)
    return np.pi * np.stack([c[..., 0] * s[..., 1] * s[..., 2], s[..., 0] * c[..., 1] * s[..., 2],
                             s[..., 0] * s[..., 1] * c[..., 2]], axis=-1)


def tet_problem(n: int, p: int, n_coarse: int, q: Optional[int] = None, per_element: bool = True,
                sub_boxes: int = 0, jitter: float = 0.0, seed: int = 0, f=f_sin3, name: str = "tet") -> Problem:
    """Cube of 6 n^3 Kuhn tetrahedra, coarse grid = the 6 n_coarse^3 Kuhn
    tetrahedra of the n_coarse-grid (nested agglomerates, n divisible by
    n_coarse); subdomains: one element each, or sub_boxes^3 boxes."""
    mesh = cube_tet_mesh(n, jitter=jitter, seed=seed)
    sub = (np.arange(mesh.n_cells, dtype=np.int32) if per_element or not sub_boxes
           else box_agglomerates(mesh, sub_boxes))
    return Problem(name=name, mesh=mesh, p=p, c_sigma=10.0, rho=np.ones(mesh.n_cells), subdomain=sub,
                   q=p if q is None else q, coarse_of_cell=kuhn_agglomerates(mesh, n_coarse), coarse_mesh=None,
                   f=f)


def make_config(name: str) -> Problem:
    """The five named workloads (C1-C5 sample) plus small test variants."""
    if name == "C1":
        # 16x16 squares, p=1, 2x2 subdomains of 8x8, coarse = subdomains, q=1
        return squares_problem(16, 1, 8, None, q=1, name="C1")
    if name == "C2":
        return voronoi_problem(16384, 1, p=2, bx=8, by=8, q=1, name="C2")
    if name == "C3":
        return voronoi_problem(65536, 2, p=3, bx=16, by=16, q=2, warped=True, name="C3")
    if name == "C3x":
        # labelled extra at ~1M DoFs: C3's design (256 warped bins, nested q=2) on 104858 cells,
        # p=3, 1048580 DoFs, subdomains of 2060..8920 DoFs
        return voronoi_problem(104858, 4, p=3, bx=16, by=16, q=2, warped=True, name="C3x")
    if name == "C4":
        return voronoi_problem(131072, 3, p=2, bx=32, by=16, q=1, nonnested_coarse=64,
                               log10_rho_range=4.0, f=f_one, name="C4")
    if name == "C4h":
        # C4's mesh, coefficients and load with one element per subdomain and
        # the 512 bins as nested agglomerated coarse cells (aligned with the
        # rho jumps), q=1: the setting of the paper's experiments (Sec. 7)
        P = make_config("C4")
        P.coarse_of_cell = P.subdomain.copy()
        P.coarse_mesh = None
        P.subdomain = np.arange(P.mesh.n_cells, dtype=np.int32)
        P.name = "C4h"
        return P
    if name == "T1":
        # 32^3 cubes of 6 Kuhn tetrahedra (196608 cells), p = q = 1, one element per
        # subdomain, 384 nested Kuhn agglomerates: the design of Example 3
        return tet_problem(32, 1, 4, name="T1")
    if name == "T1b":
        # the T1 mesh with 512 box subdomains (8^3 boxes of 384 tetrahedra, 1536 DoFs)
        return tet_problem(32, 1, 4, per_element=False, sub_boxes=8, name="T1b")
    if name == "T3":
        # 16^3 cubes (24576 tetrahedra), p = q = 3, one element per subdomain, 384 agglomerates
        return tet_problem(16, 3, 4, name="T3")
    raise KeyError(name)


def serving_requests(n_requests: int = 2000, seed: int = 5, n_min: int = 4096,
                     n_max: int = 65536):
    """Request descriptors for the serving workload: log-uniform cell count,
    p in {1,2,3}, about 64 cells per subdomain, log10 rho ~ U[-2,2] per
    subdomain, random sine-series RHS. Meshes are generated lazily from the
    per-request seed so the stream itself stays small."""
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n_requests):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        p = int(rng.integers(1, 4))
        reqs.append({"id": k, "n_cells": n, "p": p, "seed": int(rng.integers(1 << 31))})
    return reqs


def serving_mesh_specs(n_meshes: int = 128, seed: int = 5, n_min: int = 4096, n_max: int = 65536):
    """Meshes of the serving workload's mesh pool: one per stratum of
    log(n_cells) (n_meshes equal strata of [log n_min, log n_max], a
    log-uniform draw inside each), each with its own seed. Requests that pick
    a mesh of the pool uniformly have log-uniform mesh sizes."""
    rng = np.random.default_rng(seed)
    edges = np.linspace(math.log(n_min), math.log(n_max), n_meshes + 1)
    return [{"mesh_id": k, "n_cells": int(round(math.exp(rng.uniform(edges[k], edges[k + 1])))),
             "seed": int(rng.integers(1 << 31))} for k in range(n_meshes)]


def serving_mesh(spec: dict):
    """(mesh, subdomain labels) of one pool mesh: relaxed Voronoi of
    spec['n_cells'] seeds, subdomains = bins of about 64 cells."""
    rng = np.random.default_rng(spec["seed"])
    n = spec["n_cells"]
    mesh = relaxed_voronoi_mesh(rng.random((n, 2)))
    b = max(1, int(round(math.sqrt(n) / 8)))
    return mesh, compact_labels(bins_partition(mesh.vertex_mean(), b, b))


def serving_pool_requests(n_requests: int, n_meshes: int, seed: int = 6):
    """Request descriptors over a mesh pool: mesh uniform over the pool, p
    uniform in {1, 2, 3}, and a seed for the request's own coefficients and
    right-hand side."""
    rng = np.random.default_rng(seed)
    return [{"id": k, "mesh_id": int(rng.integers(n_meshes)), "p": int(rng.integers(1, 4)),
             "seed": int(rng.integers(1 << 31))} for k in range(n_requests)]


def serving_pool_problem(req: dict, pool) -> Problem:
    """The request's problem on its pool mesh: rho = 10^U[-2,2] per
    subdomain and a random sine-series load, both from the request's seed;
    nested coarse space = the subdomains, q = 1."""
    mesh, sub = pool[req["mesh_id"]]
    rng = np.random.default_rng(req["seed"])
    n_sub = int(sub.max()) + 1
    rho = (10.0 ** rng.uniform(-2.0, 2.0, size=n_sub))[sub]
    coef = rng.standard_normal((4, 4))
    return Problem(name=f"req{req['id']}", mesh=mesh, p=req["p"], c_sigma=10.0, rho=rho,
                   subdomain=sub, q=1, coarse_of_cell=sub.copy(), coarse_mesh=None,
                   f=make_f_series(coef))


def serving_problem(req: dict) -> Problem:
    rng = np.random.default_rng(req["seed"])
    n = req["n_cells"]
    mesh = relaxed_voronoi_mesh(rng.random((n, 2)))
    b = max(1, int(round(math.sqrt(n) / 8)))
    sub = compact_labels(bins_partition(mesh.vertex_mean(), b, b))
    n_sub = int(sub.max()) + 1
    rho = (10.0 ** rng.uniform(-2.0, 2.0, size=n_sub))[sub]
    coef = rng.standard_normal((4, 4))
    return Problem(name=f"req{req['id']}", mesh=mesh, p=req["p"], c_sigma=10.0, rho=rho,
                   subdomain=sub, q=1, coarse_of_cell=sub.copy(), coarse_mesh=None,
                   f=make_f_series(coef))
