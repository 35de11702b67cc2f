"""Pins of the 3D oracle (oracle/tet.py) against closed forms, invariants
and limiting cases, independent of the oracle's own formulas."""
import math

import numpy as np
import pytest
import scipy.linalg as la
import scipy.sparse.linalg as spla

from oracle.tet import (assemble3, eval_basis3, index_triples, l2_error3, n_basis3, prolongation_nested3,
                        tet_faces, tet_geometry, tet_rule, tri_rule3)
from paper_1903_11357_amd import inputs as I

REF = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])


def _moment(a, b, c):
    """Closed form of the integral of x^a y^b z^c over the reference tetrahedron."""
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


@pytest.mark.parametrize("m", [2, 3, 4])
def test_tet_rule_exact_to_2m_minus_3_and_not_beyond(m):
    pts, w = tet_rule(*(REF[i][None, :] for i in range(4)), m)
    X, W = pts[0], w[0]
    for d in range(2 * m - 2):
        for a in range(d + 1):
            for b in range(d - a + 1):
                c = d - a - b
                q = (W * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c).sum()
                assert abs(q - _moment(a, b, c)) <= 1e-14, (m, a, b, c)
    k = 2 * m - 2
    assert abs((W * X[:, 0] ** k).sum() - _moment(k, 0, 0)) > 1e-8


def test_tet_rule_affine_invariance_and_volume():
    """Moments scale with the Jacobian: the tetrahedron 2*REF + t has volume
    8/6 and first moments (volume) x centroid."""
    T = 2.0 * REF + np.array([0.3, -0.1, 0.7])
    pts, w = tet_rule(*(T[i][None, :] for i in range(4)), 3)
    assert abs(w.sum() - 8.0 / 6.0) <= 1e-14
    assert np.allclose((w[0][:, None] * pts[0]).sum(0), w.sum() * T.mean(0), atol=1e-14)


def test_triangle_rule_in_space():
    """A triangle in the plane z = 0.5 carries the planar rule: area and
    second moments equal their 2D closed forms."""
    a, b, c = np.array([[0.0, 0, 0.5]]), np.array([[2.0, 0, 0.5]]), np.array([[0.0, 1, 0.5]])
    pts, w = tri_rule3(a, b, c, 3)
    assert abs(w.sum() - 1.0) <= 1e-15
    # int x^2 over the triangle (0,0),(2,0),(0,1): area * (sum of x_i^2 + sum x_i x_j)/6
    xs = np.array([0.0, 2.0, 0.0])
    exact = 1.0 * (np.sum(xs ** 2) + xs[0] * xs[1] + xs[0] * xs[2] + xs[1] * xs[2]) / 6.0
    assert abs((w[0] * pts[0, :, 0] ** 2).sum() - exact) <= 1e-14
    assert np.allclose(pts[0, :, 2], 0.5)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_basis_orthonormal_on_box_and_spans_Pp(p):
    box = np.array([0.2, 1.0, -0.5, 0.25, 0.1, 0.4])
    cube = I.cube_tet_mesh(1)
    lo, hi = box[0::2], box[1::2]
    X = lo + cube.xyz * (hi - lo)
    T = X[cube.tets]
    pts, w = tet_rule(T[:, 0], T[:, 1], T[:, 2], T[:, 3], p + 2)
    val, _ = eval_basis3(p, box, pts)
    M = np.einsum("tq,tqa,tqb->ab", w, val, val)
    assert np.abs(M - np.eye(n_basis3(p))).max() <= 1e-12
    # every monomial of total degree <= p is reproduced exactly by its L2 projection
    P = pts.reshape(-1, 3)
    V = val.reshape(-1, n_basis3(p))
    W = w.ravel()
    for (i, j, k) in index_triples(p):
        g = P[:, 0] ** i * P[:, 1] ** j * P[:, 2] ** k
        coef = V.T @ (W * g)
        assert np.abs(V @ coef - g).max() <= 1e-11


@pytest.mark.parametrize("n", [1, 2, 3])
def test_cube_mesh_faces(n):
    mesh = I.cube_tet_mesh(n)
    geo = tet_geometry(mesh)
    assert abs(geo.vol.sum() - 1.0) <= 1e-13
    F = tet_faces(mesh)
    bd = F.minus < 0
    assert bd.sum() == 12 * n * n  # two triangles per boundary square
    assert (~bd).sum() == (4 * mesh.n_cells - 12 * n * n) // 2
    X = mesh.xyz[F.tri[bd]]
    on_side = np.zeros(bd.sum(), dtype=bool)
    for e in range(3):
        for v in (0.0, 1.0):
            on_side |= np.all(np.abs(X[:, :, e] - v) <= 1e-14, axis=1)
    assert on_side.all()
    # boundary normals point out of the cube
    cen = X.mean(1)
    assert (np.einsum("ij,ij->i", F.normal[bd], cen - 0.5) > 0).all()


def _tiny(n=2, p=1, jitter=0.0):
    return I.tet_problem(n, p, 1, jitter=jitter, seed=5)


@pytest.mark.parametrize("p", [1, 2])
def test_sipg3_symmetric_spd_and_constants(p):
    P = _tiny(2, p, jitter=0.1)
    A, b, geo, F = assemble3(P.mesh, p, P.rho, 10.0, P.f)
    Ad = A.toarray()
    assert np.abs(Ad - Ad.T).max() <= 1e-12 * np.abs(Ad).max()
    assert la.eigvalsh(Ad)[0] > 0.0
    # the constant 1 has coefficient sqrt(box volume) on phi_0 only
    npb = n_basis3(p)
    x = np.zeros(A.shape[0])
    bx = geo.box
    x[::npb] = np.sqrt((bx[:, 1] - bx[:, 0]) * (bx[:, 3] - bx[:, 2]) * (bx[:, 5] - bx[:, 4]))
    r = (A @ x).reshape(-1, npb)
    touch = np.zeros(P.mesh.n_cells, dtype=bool)
    touch[F.plus[F.minus < 0]] = True
    assert np.abs(r[~touch]).max() <= 1e-12 * np.abs(Ad).max()
    assert np.abs(r[touch]).max() > 1e-3


def test_sipg3_manufactured_rate():
    """u = sin(pi x) sin(pi y) sin(pi z), p = 2 on jittered cube meshes:
    L2 error rate p + 1 (observed 2.89, 2.99)."""
    errs = []
    for n in (2, 4, 8):
        P = I.tet_problem(n, 2, 1, jitter=0.1, seed=3)
        A, b, geo, _ = assemble3(P.mesh, 2, P.rho, 10.0, P.f)
        x = spla.spsolve(A.tocsc(), b)
        errs.append(l2_error3(P.mesh, 2, geo, x, I.u_sin3))
    assert math.log2(errs[-2] / errs[-1]) >= 2.75


@pytest.mark.parametrize("q", [1, 2])
def test_nested_prolongation_reproduces_global_polynomials(q):
    """P_0 c0 = fine coefficients of any global polynomial of degree <= q,
    with c0 its coefficients on every agglomerate (injection, Remark 3.2)."""
    P = I.tet_problem(4, 2, 2, q=q)
    geo = tet_geometry(P.mesh)
    P0, cbox = prolongation_nested3(P.mesh, 2, q, geo, P.coarse_of_cell)
    rng = np.random.default_rng(0)
    trip = index_triples(q)
    coeff = rng.standard_normal(len(trip))

    def g(X):
        return sum(c * X[..., 0] ** i * X[..., 1] ** j * X[..., 2] ** k for c, (i, j, k) in zip(coeff, trip))

    nc = int(P.coarse_of_cell.max()) + 1
    nq = n_basis3(q)
    c0 = np.zeros(nc * nq)
    for J in range(nc):
        Xs = rng.uniform(cbox[J, 0::2], cbox[J, 1::2], size=(4 * nq, 3))
        V, _ = eval_basis3(q, cbox[J], Xs)
        c0[J * nq:(J + 1) * nq] = np.linalg.lstsq(V, g(Xs), rcond=None)[0]
    x = P0 @ c0
    T = P.mesh.xyz[P.mesh.tets]
    pts, w = tet_rule(T[:, 0], T[:, 1], T[:, 2], T[:, 3], 4)
    val, _ = eval_basis3(2, geo.box[:, None, :], pts)
    uh = np.einsum("tqa,ta->tq", val, x.reshape(-1, n_basis3(2)))
    assert np.abs(uh - g(pts)).max() <= 1e-9 * np.abs(g(pts)).max()


def test_schwarz3_spectrum_bounds():
    """lambda(M^{-1} A) in (0, chi + 1] (exact local solvers), and one
    subdomain plus a coarse space gives eigenvalues in {1, 2}."""
    from oracle.schwarz import TwoLevelSchwarz, preconditioned_spectrum, subdomain_colouring

    P = I.tet_problem(2, 1, 1, per_element=False, sub_boxes=2)
    A, b, geo, _ = assemble3(P.mesh, 1, P.rho, 10.0, P.f)
    P0, _ = prolongation_nested3(P.mesh, 1, 1, geo, P.coarse_of_cell)
    M = TwoLevelSchwarz(A, P.mesh, 1, geo, P.subdomain, q=1, P0=P0, npb=4)
    ev = preconditioned_spectrum(A, M.dense_inverse())
    chi = int(subdomain_colouring(A, P.subdomain, 4)[0].max()) + 1
    assert ev[0] > 0 and ev[-1] <= chi + 1 + 1e-10
    one = np.zeros(P.mesh.n_cells, dtype=np.int32)
    M1 = TwoLevelSchwarz(A, P.mesh, 1, geo, one, q=1, P0=P0, npb=4)
    ev1 = preconditioned_spectrum(A, M1.dense_inverse())
    assert np.all((np.abs(ev1 - 1.0) < 1e-8) | (np.abs(ev1 - 2.0) < 1e-8))
