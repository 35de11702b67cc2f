"""SIPG matrix and load vector (oracle; test infrastructure).

The bilinear form is eq. (Ah) with the lifting operator of eq. (lifting) and
weight omega = rho^- / (rho^+ + rho^-) on interior faces. Because rho is
constant on each cell (Remark 2.1) and rho grad v lies in [V_h]^d, the lifting
terms equal face integrals of the weighted average (the same step the paper
takes in the proof of Lemma 5.12), giving the flux form

  A(u,v) = sum_K int_K rho grad u . grad v
         - sum_F int_F {rho grad u}_w . [[v]] + {rho grad v}_w . [[u]]
         + sum_F int_F sigma [[u]] . [[v]],

with {rho grad u}_w = (gamma_F / 2)(grad u^+ + grad u^-) on interior faces,
gamma_F = <rho>_F the harmonic average, and on boundary faces {.}_w = trace,
[[v]] = v n. The penalty is eq. (Sigma): sigma_F = C_sigma <rho>_F p^2 / <h>_F
with <h>_F the harmonic average of the two cell diameters on interior faces
and h_kappa on boundary faces. The load is b_a = int f phi_a (homogeneous
Dirichlet data, u in H^1_0).

Pins: symmetry; positive definiteness at C_sigma = 10 (Lemma 5.1); A applied
to the global constant vanishes on every cell not touching the boundary;
manufactured-solution L2 rate h^{p+1}, also across a coefficient jump 1 | 100
along a mesh line with nonzero normal flux (fails for a face average that is
not consistent for that flux); entries of A on two rectangles with unequal
rho and h worked out by hand (fix the omega weights, the harmonic <rho>_F and
<h>_F, and the boundary-face penalty); the printed condition number of the
Example 5 nested square series (via the Schwarz module).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import eval_basis, n_basis
from .geometry import cell_geometry, mesh_faces
from .quadrature import segments_rule, triangles_rule


def fan_triangles(mesh, geo):
    """Triangles (centroid, v_k, v_{k+1}) of every cell and their owner."""
    counts = np.diff(mesh.cell_ptr)
    owner = np.repeat(np.arange(mesh.n_cells), counts)
    cv = mesh.cell_vertices
    nxt = np.arange(cv.shape[0]) + 1
    last = mesh.cell_ptr[1:] - 1
    nxt[last] = mesh.cell_ptr[:-1]
    return owner, geo.centroid[owner], mesh.xy[cv], mesh.xy[cv[nxt]]


def assemble(mesh, p, rho, c_sigma, f=None, geo=None, faces=None, h=None, chunk=40000):
    """Return (A csr [n, n], b [n] or None, geo, faces).

    DoF index of basis function a on cell k is k * n_p + a."""
    geo = cell_geometry(mesh) if geo is None else geo
    faces = mesh_faces(mesh) if faces is None else faces
    h = geo.diam if h is None else np.asarray(h, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    N = mesh.n_cells
    npb = n_basis(p)
    m = p + 2
    rows, cols, blocks = [], [], []
    b = np.zeros(N * npb) if f is not None else None

    # volume terms: rho int grad phi_a . grad phi_b
    owner, A_, B_, C_ = fan_triangles(mesh, geo)
    vol = np.zeros((N, npb, npb))
    for s in range(0, owner.shape[0], chunk):
        e = slice(s, s + chunk)
        pts, w = triangles_rule(A_[e], B_[e], C_[e], m)
        own = owner[e]
        val, grad = eval_basis(p, geo.box[own][:, None, :], pts)
        K = np.einsum("tq,tqad,tqbd->tab", w, grad, grad) * rho[own][:, None, None]
        np.add.at(vol, own, K)
        if f is not None:
            fv = f(pts.reshape(-1, 2)).reshape(w.shape)
            bl = np.einsum("tq,tqa,tq->ta", w, val, fv)
            np.add.at(b, (own[:, None] * npb + np.arange(npb)[None, :]), bl)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    blocks.append(vol)

    P0 = mesh.xy[faces.v0]
    P1 = mesh.xy[faces.v1]
    d = P1 - P0
    L = np.linalg.norm(d, axis=1)
    nrm = np.stack([d[:, 1], -d[:, 0]], axis=1) / L[:, None]
    pts, w = segments_rule(P0, P1, m)
    pp = faces.plus
    mm = faces.minus

    # interior faces
    it = mm >= 0
    if it.any():
        kp, km = pp[it], mm[it]
        ptsI, wI, nI = pts[it], w[it], nrm[it]
        vp, gp = eval_basis(p, geo.box[kp][:, None, :], ptsI)
        vm, gm = eval_basis(p, geo.box[km][:, None, :], ptsI)
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

    # boundary faces
    bd = ~it
    if bd.any():
        kb = pp[bd]
        ptsB, wB, nB = pts[bd], w[bd], nrm[bd]
        vb, gb = eval_basis(p, geo.box[kb][:, None, :], ptsB)
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
    C = np.concatenate(cols)
    Bk = np.concatenate(blocks)
    ia = np.arange(npb)
    I = (R[:, None, None] * npb + ia[None, :, None]) + 0 * ia[None, None, :]
    J = (C[:, None, None] * npb + ia[None, None, :]) + 0 * ia[None, :, None]
    A = sp.coo_matrix((Bk.ravel(), (I.ravel(), J.ravel())), shape=(N * npb, N * npb)).tocsr()
    A.sum_duplicates()
    return A, b, geo, faces


def mass_blocks(mesh, p, geo, chunk=40000):
    """Per-cell mass matrices M_kappa [N, n_p, n_p]."""
    npb = n_basis(p)
    owner, A_, B_, C_ = fan_triangles(mesh, geo)
    M = np.zeros((mesh.n_cells, npb, npb))
    for s in range(0, owner.shape[0], chunk):
        e = slice(s, s + chunk)
        pts, w = triangles_rule(A_[e], B_[e], C_[e], p + 2)
        val, _ = eval_basis(p, geo.box[owner[e]][:, None, :], pts)
        np.add.at(M, owner[e], np.einsum("tq,tqa,tqb->tab", w, val, val))
    return M


def l2_and_broken_h1_error(mesh, p, geo, x, u, grad_u, extra=3):
    """||u_h - u||_{L2} and |u_h - u|_{H1(T_h)} with an over-integrated rule."""
    npb = n_basis(p)
    owner, A_, B_, C_ = fan_triangles(mesh, geo)
    pts, w = triangles_rule(A_, B_, C_, p + 2 + extra)
    val, grad = eval_basis(p, geo.box[owner][:, None, :], pts)
    coef = x.reshape(-1, npb)[owner]
    uh = np.einsum("tqa,ta->tq", val, coef)
    guh = np.einsum("tqad,ta->tqd", grad, coef)
    P = pts.reshape(-1, 2)
    e0 = (uh - u(P).reshape(uh.shape)) ** 2
    e1 = ((guh - grad_u(P).reshape(guh.shape)) ** 2).sum(-1)
    return float(np.sqrt((w * e0).sum())), float(np.sqrt((w * e1).sum()))
