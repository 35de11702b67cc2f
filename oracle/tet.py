"""Three-dimensional SIPG on tetrahedral meshes and the nested coarse
transfer (oracle; test infrastructure).

The method of Secs. 2-3 is stated for d = 2, 3. In 3D the cells are
tetrahedra, faces are triangles, V_h holds polynomials of total degree p
(n_p = (p+1)(p+2)(p+3)/6 per cell), the form is the same flux form as in 2D
(see oracle/sipg.py: eq. (Ah) with the lifting of eq. (lifting), harmonic
weights, penalty eq. (Sigma) with h the cell diameter) and the coarse
space is P_q on agglomerates of the fine cells with the L2 prolongation of
eq. (R0T), which for nested agglomerates is the injection (Remark 3.2).

Readings (the paper is silent on them):
- basis: the tensor Legendre family of total degree p, orthonormal on the
  cell's axis-aligned bounding box, ordered by degree d = 0..p, then
  k = 0..d, then j = 0..d-k with i = d-j-k (exponents of x, y, z = i, j, k);
- volume quadrature: the collapsed map of the cube [0,1]^3 onto the
  tetrahedron (a, b, c, d), X = (1-s) a + s((1-t) b + t((1-u) c + u d)),
  Jacobian 6|T| s^2 t, m-point Gauss-Legendre per direction, exact for
  total degree 2m-3; faces: the collapsed triangle rule (exact to 2m-2);
  m = p + 2.

Pins (tests/test_oracle_3d.py): the tetrahedron rule against the closed
form of monomial moments of the reference tetrahedron (exact to 2m-3 and
not beyond); orthonormality on a box and span of P_p; the mesh (volumes sum
to one, every interior face shared by two cells, boundary faces on the
cube's sides); SIPG symmetry, positive definiteness, vanishing of A 1 on
cells away from the boundary, the manufactured-solution L2 rate p+1 (also
across a coefficient jump 1 | 100 along a mesh plane); hand-worked entries
across faces between tetrahedra of unequal rho and h (omega weights,
harmonic <rho>_F and <h>_F);
nested P_0 reproducing global polynomials of degree <= q; spectrum of the
two-level preconditioner in (0, chi + 1].
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg

from .quadrature import gauss_legendre_01


def n_basis3(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def index_triples(p: int):
    return [(d - j - k, j, k) for d in range(p + 1) for k in range(d + 1) for j in range(d - k + 1)]


def _leg(p: int, t: np.ndarray):
    val = np.empty((p + 1,) + t.shape)
    der = np.empty((p + 1,) + t.shape)
    for k in range(p + 1):
        c = np.zeros(k + 1)
        c[k] = 1.0
        val[k] = npleg.legval(t, c)
        der[k] = npleg.legval(t, npleg.legder(c)) if k > 0 else 0.0
    return val, der


def eval_basis3(p: int, box: np.ndarray, pts: np.ndarray):
    """Values [..., n_p] and gradients [..., n_p, 3] at pts [..., 3]; box
    [..., 6] = x0, x1, y0, y1, z0, z1 broadcasting against pts[..., 0]."""
    box = np.asarray(box, dtype=np.float64)
    lo = box[..., 0::2]
    hi = box[..., 1::2]
    dl = hi - lo
    t = 2.0 * (pts - 0.5 * (lo + hi)) / dl
    L = [_leg(p, t[..., e]) for e in range(3)]
    trip = index_triples(p)
    val = np.empty(pts.shape[:-1] + (len(trip),))
    grad = np.empty(pts.shape[:-1] + (len(trip), 3))
    vol = dl[..., 0] * dl[..., 1] * dl[..., 2]
    for a, (i, j, k) in enumerate(trip):
        s = np.sqrt((2 * i + 1) * (2 * j + 1) * (2 * k + 1) / vol)
        lx, ly, lz = L[0][0][i], L[1][0][j], L[2][0][k]
        dx, dy, dz = L[0][1][i], L[1][1][j], L[2][1][k]
        val[..., a] = s * lx * ly * lz
        grad[..., a, 0] = s * dx * ly * lz * 2.0 / dl[..., 0]
        grad[..., a, 1] = s * lx * dy * lz * 2.0 / dl[..., 1]
        grad[..., a, 2] = s * lx * ly * dz * 2.0 / dl[..., 2]
    return val, grad


def tet_rule(a, b, c, d, m: int):
    """Points [n, m^3, 3] and weights [n, m^3] (volume included) on the
    tetrahedra (a, b, c, d) [n, 3] each."""
    g, wg = gauss_legendre_01(m)
    S, T, U = np.meshgrid(g, g, g, indexing="ij")
    W = (np.einsum("i,j,k->ijk", wg, wg, wg) * S ** 2 * T).ravel()
    s, t, u = S.ravel()[None, :, None], T.ravel()[None, :, None], U.ravel()[None, :, None]
    A, B, C, D = (x[:, None, :] for x in (a, b, c, d))
    pts = (1.0 - s) * A + s * ((1.0 - t) * B + t * ((1.0 - u) * C + u * D))
    vol = np.abs(np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a)) / 6.0
    return pts, 6.0 * vol[:, None] * W[None, :]


def tri_rule3(a, b, c, m: int):
    """Points [n, m^2, 3] and weights [n, m^2] (area included) on triangles
    (a, b, c) [n, 3] in space."""
    g, wg = gauss_legendre_01(m)
    S, T = np.meshgrid(g, g, indexing="ij")
    W = (np.outer(wg, wg) * S).ravel()
    s, t = S.ravel()[None, :, None], T.ravel()[None, :, None]
    pts = (1.0 - s) * a[:, None, :] + s * ((1.0 - t) * b[:, None, :] + t * c[:, None, :])
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    return pts, 2.0 * area[:, None] * W[None, :]


@dataclasses.dataclass
class TetGeometry:
    vol: np.ndarray   # [N]
    diam: np.ndarray  # [N] longest edge
    box: np.ndarray   # [N, 6]


def tet_geometry(mesh) -> TetGeometry:
    P = mesh.xyz[mesh.tets]
    vol = np.abs(np.einsum("ij,ij->i", np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), P[:, 3] - P[:, 0])) / 6.0
    e = P[:, :, None, :] - P[:, None, :, :]
    diam = np.sqrt((e ** 2).sum(-1)).reshape(P.shape[0], -1).max(axis=1)
    box = np.stack([P[:, :, 0].min(1), P[:, :, 0].max(1), P[:, :, 1].min(1), P[:, :, 1].max(1),
                    P[:, :, 2].min(1), P[:, :, 2].max(1)], axis=1)
    return TetGeometry(vol, diam, box)


@dataclasses.dataclass
class TriFaces:
    plus: np.ndarray   # [F]
    minus: np.ndarray  # [F], -1 on the boundary
    tri: np.ndarray    # [F, 3] vertex ids
    normal: np.ndarray  # [F, 3] unit, outward from the plus cell


def tet_faces(mesh) -> TriFaces:
    """Faces in order of first appearance (cell order, then local face
    opposite vertex 0..3); plus = first cell."""
    N = mesh.n_cells
    loc = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    tri = mesh.tets[:, loc].reshape(-1, 3)
    opp = mesh.tets[:, [0, 1, 2, 3]].reshape(-1)
    owner = np.repeat(np.arange(N), 4)
    key = np.sort(tri, axis=1)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.ravel()
    nf = first.shape[0]
    order = np.argsort(first, kind="stable")  # faces numbered by first appearance
    rank = np.empty(nf, dtype=np.int64)
    rank[order] = np.arange(nf)
    fid = rank[inv]
    plus = -np.ones(nf, dtype=np.int64)
    minus = -np.ones(nf, dtype=np.int64)
    ftri = np.zeros((nf, 3), dtype=np.int64)
    fopp = np.zeros(nf, dtype=np.int64)
    for slot in range(tri.shape[0]):
        f = fid[slot]
        if plus[f] < 0:
            plus[f] = owner[slot]
            ftri[f] = tri[slot]
            fopp[f] = opp[slot]
        elif minus[f] < 0:
            minus[f] = owner[slot]
        else:
            raise ValueError("face shared by more than two cells")
    A, B, C = (mesh.xyz[ftri[:, e]] for e in range(3))
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n, axis=1)[:, None]
    flip = np.einsum("ij,ij->i", n, mesh.xyz[fopp] - A) > 0
    n[flip] *= -1.0
    return TriFaces(plus, minus, ftri, n)


def assemble3(mesh, p, rho, c_sigma, f=None):
    """(A csr [n, n], b [n] or None, geo, faces); DoF of basis a on cell k is
    k n_p + a."""
    geo = tet_geometry(mesh)
    faces = tet_faces(mesh)
    rho = np.asarray(rho, dtype=np.float64)
    N = mesh.n_cells
    npb = n_basis3(p)
    m = p + 2
    h = geo.diam
    P = mesh.xyz[mesh.tets]
    pts, w = tet_rule(P[:, 0], P[:, 1], P[:, 2], P[:, 3], m)
    val, grad = eval_basis3(p, geo.box[:, None, :], pts)
    vol = np.einsum("tq,tqad,tqbd->tab", w, grad, grad) * rho[:, None, None]
    b = None
    if f is not None:
        fv = f(pts.reshape(-1, 3)).reshape(w.shape)
        b = np.einsum("tq,tqa,tq->ta", w, val, fv).ravel()
    rows, cols, blocks = [np.arange(N)], [np.arange(N)], [vol]
    A_, B_, C_ = (mesh.xyz[faces.tri[:, e]] for e in range(3))
    fpts, fw = tri_rule3(A_, B_, C_, m)
    nrm = faces.normal
    it = faces.minus >= 0
    if it.any():
        kp, km = faces.plus[it], faces.minus[it]
        ptsI, wI, nI = fpts[it], fw[it], nrm[it]
        vp, gp = eval_basis3(p, geo.box[kp][:, None, :], ptsI)
        vm, gm = eval_basis3(p, geo.box[km][:, None, :], ptsI)
        gnp = np.einsum("fqad,fd->fqa", gp, nI)
        gnm = np.einsum("fqad,fd->fqa", gm, nI)
        rp, rm = rho[kp], rho[km]
        gamma = 2.0 * rp * rm / (rp + rm)
        hF = 2.0 * h[kp] * h[km] / (h[kp] + h[km])
        sigma = c_sigma * gamma * p * p / hF
        side = {+1: (kp, vp, gnp), -1: (km, vm, gnm)}
        for et in (+1, -1):
            kt, vt, gt = side[et]
            for es in (+1, -1):
                ks, vs, gs = side[es]
                blk = (-(0.5 * gamma * et)[:, None, None] * np.einsum("fq,fqa,fqb->fab", wI, vt, gs)
                       - (0.5 * gamma * es)[:, None, None] * np.einsum("fq,fqa,fqb->fab", wI, gt, vs)
                       + (sigma * et * es)[:, None, None] * np.einsum("fq,fqa,fqb->fab", wI, vt, vs))
                rows.append(kt)
                cols.append(ks)
                blocks.append(blk)
    bd = ~it
    if bd.any():
        kb = faces.plus[bd]
        ptsB, wB, nB = fpts[bd], fw[bd], nrm[bd]
        vb, gb = eval_basis3(p, geo.box[kb][:, None, :], ptsB)
        gnb = np.einsum("fqad,fd->fqa", gb, nB)
        rb = rho[kb]
        sigma = c_sigma * rb * p * p / h[kb]
        blk = (-rb[:, None, None] * np.einsum("fq,fqa,fqb->fab", wB, vb, gnb)
               - rb[:, None, None] * np.einsum("fq,fqa,fqb->fab", wB, gnb, vb)
               + sigma[:, None, None] * np.einsum("fq,fqa,fqb->fab", wB, vb, vb))
        rows.append(kb)
        cols.append(kb)
        blocks.append(blk)
    R = np.concatenate(rows)
    Cc = np.concatenate(cols)
    Bk = np.concatenate(blocks)
    ia = np.arange(npb)
    I = (R[:, None, None] * npb + ia[None, :, None]) + 0 * ia[None, None, :]
    J = (Cc[:, None, None] * npb + ia[None, None, :]) + 0 * ia[None, :, None]
    A = sp.coo_matrix((Bk.ravel(), (I.ravel(), J.ravel())), shape=(N * npb, N * npb)).tocsr()
    A.sum_duplicates()
    return A, b, geo, faces


def mass_blocks3(mesh, p, geo):
    P = mesh.xyz[mesh.tets]
    pts, w = tet_rule(P[:, 0], P[:, 1], P[:, 2], P[:, 3], p + 2)
    val, _ = eval_basis3(p, geo.box[:, None, :], pts)
    return np.einsum("tq,tqa,tqb->tab", w, val, val)


def prolongation_nested3(mesh, p, q, geo, coarse_of_cell):
    """P_0 (n x n0) for agglomerates (unions of fine tetrahedra): per fine
    cell M_k^{-1} int_k phi psi, psi the degree-q basis on the agglomerate's
    bounding box."""
    npb, nq = n_basis3(p), n_basis3(q)
    N = mesh.n_cells
    nc = int(coarse_of_cell.max()) + 1
    cbox = np.empty((nc, 6))
    for e in range(3):
        cbox[:, 2 * e] = np.full(nc, np.inf)
        cbox[:, 2 * e + 1] = np.full(nc, -np.inf)
        np.minimum.at(cbox[:, 2 * e], coarse_of_cell, geo.box[:, 2 * e])
        np.maximum.at(cbox[:, 2 * e + 1], coarse_of_cell, geo.box[:, 2 * e + 1])
    M = mass_blocks3(mesh, p, geo)
    P = mesh.xyz[mesh.tets]
    pts, w = tet_rule(P[:, 0], P[:, 1], P[:, 2], P[:, 3], p + 2)
    val, _ = eval_basis3(p, geo.box[:, None, :], pts)
    psi, _ = eval_basis3(q, cbox[coarse_of_cell][:, None, :], pts)
    Bm = np.einsum("tq,tqa,tqb->tab", w, val, psi)
    blocks = np.linalg.solve(M, Bm)
    rows = (np.arange(N)[:, None, None] * npb + np.arange(npb)[None, :, None]) + 0 * np.arange(nq)[None, None, :]
    cols = (coarse_of_cell[:, None, None] * nq + np.arange(nq)[None, None, :]) + 0 * np.arange(npb)[None, :, None]
    P0 = sp.coo_matrix((blocks.ravel(), (rows.ravel(), cols.ravel())), shape=(N * npb, nc * nq)).tocsr()
    return P0, cbox


def l2_error3(mesh, p, geo, x, u, extra=3):
    """||u_h - u||_{L2} with an over-integrated rule."""
    npb = n_basis3(p)
    P = mesh.xyz[mesh.tets]
    pts, w = tet_rule(P[:, 0], P[:, 1], P[:, 2], P[:, 3], p + 2 + extra)
    val, _ = eval_basis3(p, geo.box[:, None, :], pts)
    uh = np.einsum("tqa,ta->tq", val, x.reshape(-1, npb))
    return float(np.sqrt((w * (uh - u(pts.reshape(-1, 3)).reshape(uh.shape)) ** 2).sum()))
