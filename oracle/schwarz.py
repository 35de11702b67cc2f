"""Two-level non-overlapping additive Schwarz preconditioner (oracle; test
infrastructure). Sec. 3 of the paper.

Local solvers: V_i = V_h restricted to the subdomain Omega_i (a union of fine
cells); A_i(u,v) = A_h(R_i^T u, R_i^T v), so the matrix of A_i is the
principal submatrix of A on the DoFs of Omega_i, factorised by dense
Cholesky (exact local solves, local stability constant 1).

Coarse solver: V_0 = piecewise P_q on the coarse mesh T_H (1 <= q <= p),
basis = scaled Legendre on coarse-cell boxes. R_0^T is the L2 prolongation
of eq. (R0T): for every fine cell kappa its coefficients are
M_kappa^{-1} int_kappa phi^kappa psi^D, summed over the coarse cells D that
overlap kappa, so R_0^T v_0 is the L2 projection of v_0 onto V_h (the
identity Pi^0 v_0 = R_0^T v_0 stated in the non-nested analysis). In the
nested case this reduces to the injection (Remark 3.2). A_0 is the Galerkin
operator of eq. (A0): A_0 = P_0^T A P_0 with P_0 the matrix of R_0^T.

Preconditioner in matrix form (from the projections P_i of Sec. 3: A_i
P~_i v = R_i A v, A_0 P~_0 v = P_0^T A v, hence P_ad = M^{-1} A with)
   M^{-1} r = P_0 A_0^{-1} P_0^T r + sum_i R_i^T A_i^{-1} R_i r.

Pins: A_i equals the principal submatrix; exact zero coupling between
non-adjacent subdomains (Lemma 5.12); nested P_0 is the injection; non-nested
P_0 reproduces global polynomials of degree <= q and preserves integrals;
spectrum of M^{-1}A within (0, chi + 1] with chi the number of colours of a
greedy colouring of the subdomain adjacency graph (Assumption 6.2 with
exact local solvers); one subdomain plus coarse space gives a spectrum in
{1, 2}; Example 5's printed K(P_ad) for the nested 16x16 square series.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

from .basis import eval_basis, n_basis
from .clip import clip_convex
from .geometry import cell_geometry, polygon_area_centroid
from .quadrature import triangles_rule
from .sipg import fan_triangles, mass_blocks


def subdomain_dofs(subdomain: np.ndarray, npb: int):
    """DoF index lists of every subdomain (cells in increasing order)."""
    out = []
    for i in range(int(subdomain.max()) + 1):
        cells = np.flatnonzero(subdomain == i)
        out.append((cells[:, None] * npb + np.arange(npb)[None, :]).ravel())
    return out


def _polygon_fan_rule(P: np.ndarray, m: int):
    """Quadrature on a convex polygon by its centroid fan."""
    _, c = polygon_area_centroid(P)
    k = P.shape[0]
    a = np.repeat(c[None, :], k, axis=0)
    pts, w = triangles_rule(a, P, np.roll(P, -1, axis=0), m)
    return pts.reshape(-1, 2), w.ravel()


def prolongation_nested(mesh, p, q, geo, coarse_of_cell):
    """P_0 (n x n0) for coarse cells that are unions of fine cells."""
    npb, nq = n_basis(p), n_basis(q)
    N = mesh.n_cells
    nc = int(coarse_of_cell.max()) + 1
    cbox = np.empty((nc, 4))
    for j in range(nc):
        cells = np.flatnonzero(coarse_of_cell == j)
        bx = geo.box[cells]
        cbox[j] = [bx[:, 0].min(), bx[:, 1].max(), bx[:, 2].min(), bx[:, 3].max()]
    M = mass_blocks(mesh, p, geo)
    owner, A_, B_, C_ = fan_triangles(mesh, geo)
    pts, w = triangles_rule(A_, B_, C_, p + 2)
    val, _ = eval_basis(p, geo.box[owner][:, None, :], pts)
    psi, _ = eval_basis(q, cbox[coarse_of_cell[owner]][:, None, :], pts)
    Bm = np.zeros((N, npb, nq))
    np.add.at(Bm, owner, np.einsum("tq,tqa,tqb->tab", w, val, psi))
    blocks = np.linalg.solve(M, Bm)
    rows = (np.arange(N)[:, None, None] * npb + np.arange(npb)[None, :, None]) + 0 * np.arange(nq)[None, None, :]
    cols = (coarse_of_cell[:, None, None] * nq + np.arange(nq)[None, None, :]) + 0 * np.arange(npb)[None, :, None]
    P0 = sp.coo_matrix((blocks.ravel(), (rows.ravel(), cols.ravel())), shape=(N * npb, nc * nq)).tocsr()
    return P0, cbox


def prolongation_nonnested(mesh, p, q, geo, coarse_mesh, min_rel_area=0.0):
    """P_0 (n x n0) for an independent convex coarse mesh."""
    npb, nq = n_basis(p), n_basis(q)
    N = mesh.n_cells
    cgeo = cell_geometry(coarse_mesh)
    nc = coarse_mesh.n_cells
    M = mass_blocks(mesh, p, geo)
    rows, cols, vals = [], [], []
    for k in range(N):
        P = mesh.xy[mesh.cell(k)]
        bx = geo.box[k]
        cand = np.flatnonzero((cgeo.box[:, 0] <= bx[1]) & (cgeo.box[:, 1] >= bx[0])
                              & (cgeo.box[:, 2] <= bx[3]) & (cgeo.box[:, 3] >= bx[2]))
        for j in cand:
            Q = clip_convex(P, coarse_mesh.xy[coarse_mesh.cell(j)])
            if Q.shape[0] < 3:
                continue
            a, _ = polygon_area_centroid(Q)
            if a <= min_rel_area * geo.area[k]:
                continue
            pts, w = _polygon_fan_rule(Q, p + 2)
            val, _ = eval_basis(p, geo.box[k], pts)
            psi, _ = eval_basis(q, cgeo.box[j], pts)
            blk = np.linalg.solve(M[k], np.einsum("q,qa,qb->ab", w, val, psi))
            r = k * npb + np.arange(npb)
            c = j * nq + np.arange(nq)
            rows.append(np.repeat(r, nq))
            cols.append(np.tile(c, npb))
            vals.append(blk.ravel())
    P0 = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(N * npb, nc * nq)).tocsr()
    return P0, cgeo.box


class TwoLevelSchwarz:
    """M^{-1} = P_0 A_0^{-1} P_0^T + sum_i R_i^T A_i^{-1} R_i."""

    def __init__(self, A, mesh, p, geo, subdomain, q=None, coarse_of_cell=None,
                 coarse_mesh=None, coarse=True, local=True, P0=None, npb=None):
        """P0 (with npb, the DoFs per cell): a prolongation built elsewhere
        (the 3D nested transfer of oracle/tet.py)."""
        self.A = A
        self.n = A.shape[0]
        self.npb = n_basis(p) if npb is None else npb
        self.dofs = subdomain_dofs(np.asarray(subdomain), self.npb) if local else []
        self.factors = []
        for d in self.dofs:
            Ai = A[d][:, d].toarray()
            self.factors.append(la.cho_factor(Ai, lower=True))
        self.P0 = None
        if coarse:
            if P0 is not None:
                self.P0, self.cbox = P0, None
            elif coarse_mesh is not None:
                self.P0, self.cbox = prolongation_nonnested(mesh, p, q, geo, coarse_mesh)
            else:
                self.P0, self.cbox = prolongation_nested(mesh, p, q, geo, np.asarray(coarse_of_cell))
            self.A0 = (self.P0.T @ (A @ self.P0)).toarray()
            self.A0 = 0.5 * (self.A0 + self.A0.T)
            self.A0_factor = la.cho_factor(self.A0, lower=True)

    def local_apply(self, r):
        z = np.zeros_like(r)
        for d, fac in zip(self.dofs, self.factors):
            z[d] = la.cho_solve(fac, r[d])
        return z

    def coarse_apply(self, r):
        if self.P0 is None:
            return np.zeros_like(r)
        return self.P0 @ la.cho_solve(self.A0_factor, self.P0.T @ r)

    def apply(self, r):
        return self.local_apply(r) + self.coarse_apply(r)

    def dense_inverse(self):
        """M^{-1} as a dense matrix (tiny problems only)."""
        Minv = np.zeros((self.n, self.n))
        for d, fac in zip(self.dofs, self.factors):
            Minv[np.ix_(d, d)] += la.cho_solve(fac, np.eye(len(d)))
        if self.P0 is not None:
            P0 = self.P0.toarray()
            Minv += P0 @ la.cho_solve(self.A0_factor, P0.T)
        return Minv


def preconditioned_spectrum(A, Minv):
    """Eigenvalues of M^{-1} A via the symmetric form C^T A C, C C^T = M^{-1}."""
    Cf = la.cholesky(0.5 * (Minv + Minv.T), lower=True)
    Ad = A.toarray() if sp.issparse(A) else A
    S = Cf.T @ Ad @ Cf
    return la.eigvalsh(0.5 * (S + S.T))


def subdomain_colouring(A, subdomain, npb):
    """Greedy colouring of the subdomain graph (edge = nonzero coupling)."""
    sub = np.asarray(subdomain)
    ns = int(sub.max()) + 1
    C = sp.coo_matrix(A)
    si = sub[C.row // npb]
    sj = sub[C.col // npb]
    nz = C.data != 0.0
    adj = [set() for _ in range(ns)]
    for a, b in zip(si[nz], sj[nz]):
        if a != b:
            adj[a].add(b)
    colour = -np.ones(ns, dtype=int)
    for i in range(ns):
        used = {colour[j] for j in adj[i] if colour[j] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour, adj
