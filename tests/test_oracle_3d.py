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


def test_sipg3_weighted_face_terms_two_cells():
    """Entries of A across one triangular face between two tetrahedra with
    rho_L != rho_R and h_L != h_R, worked out by hand from Sec. 2: eq. (Ah)
    with the lifting of eq. (lifting), omega = rho-/(rho+ + rho-), the
    harmonic average <.>, and eq. (Sigma) sigma_F = C_sigma <rho>_F p^2 / <h>_F.

    Mesh: the Kuhn triangulation of the 2x2x2 grid with its middle x-plane
    moved to x = a = 1/3, so a tetrahedron L left of that plane has the box
    [0,a]x(1/2)x(1/2) (volume V_L = a/4, diameter h_L = sqrt(a^2 + 1/2)) and
    one on the right R has [a,1]x... (V_R = b/4, b = 1 - a, h_R =
    sqrt(b^2 + 1/2)). p = 1, C_sigma = 10, rho random per cell. On a shared
    face F (in the plane x = a, area |F|, n_L = (1,0,0)): phi0 = 1/sqrt(V),
    the x-mode phi_x = sqrt(3/V) L_1(2(x - xc)/dx) is +sqrt(3/V_L) on F from
    L with gradient sqrt(3/V_L)(2/a,0,0), and -sqrt(3/V_R) from R with
    gradient sqrt(3/V_R)(2/b,0,0). The omega-weighted average of rho grad u
    gives rho_L rho_R/(rho_L + rho_R) =: w times the one-sided gradient (as in
    2D, the lifting term equals -int_F jump(v) . {rho grad u}_w because rho grad u
    lies in [V_h]^3). Hence
      A[0_L, 0_R] = -sigma_F |F| / sqrt(V_L V_R)
      A[0_L, x_R] = |F| sqrt(3/V_R) / sqrt(V_L) (sigma_F - (2/b) w)
      A[0_R, x_L] = |F| sqrt(3/V_L) / sqrt(V_R) ((2/a) w - sigma_F)."""
    a = 1.0 / 3.0
    b = 1.0 - a
    mesh = I.cube_tet_mesh(2)
    mid = np.abs(mesh.xyz[:, 0] - 0.5) < 1e-12
    mesh.xyz[mid, 0] = a
    rho = 10.0 ** np.random.default_rng(7).uniform(-3, 3, mesh.n_cells)
    A, *_ = assemble3(mesh, 1, rho, 10.0)
    A = A.toarray()
    npb = n_basis3(1)
    X = mesh.xyz[mesh.tets]
    left = np.flatnonzero(X[:, :, 0].max(1) <= a + 1e-12)
    right = np.flatnonzero(X[:, :, 0].min(1) >= a - 1e-12)
    hL, hR = math.sqrt(a * a + 0.5), math.sqrt(b * b + 0.5)
    VL, VR = a / 4.0, b / 4.0
    hF = 2.0 * hL * hR / (hL + hR)
    pairs = 0
    for L in left:
        for R in right:
            shared = sorted(set(mesh.tets[L].tolist()) & set(mesh.tets[R].tolist()))
            if len(shared) != 3:
                continue
            T = mesh.xyz[shared]
            area = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))
            rL, rR = rho[L], rho[R]
            w = rL * rR / (rL + rR)
            sF = 10.0 * (2.0 * w) / hF
            s3L, s3R = math.sqrt(3.0 / VL), math.sqrt(3.0 / VR)
            expect = {
                (L * npb, R * npb): -sF * area / math.sqrt(VL * VR),
                (L * npb, R * npb + 1): area * s3R / math.sqrt(VL) * (sF - (2.0 / b) * w),
                (R * npb, L * npb + 1): area * s3L / math.sqrt(VR) * ((2.0 / a) * w - sF),
            }
            for (i, j), v in expect.items():
                assert abs(A[i, j] - v) <= 1e-12 * abs(v), ((L, R), (i, j), A[i, j], v)
            pairs += 1
    assert pairs == 8  # the 2x2 squares of the plane x = a, two triangles each


def test_sipg3_manufactured_rate_with_coefficient_jump():
    """rho = 1 | 100 across the mesh plane x = 1/2, u = g(x) sin(pi y)
    sin(pi z) with g and rho g' continuous there (g as in the 2D test:
    x(1-x)/rho + c x on the left, c' (1-x) on the right), p = 2: L2 rate
    p + 1 (observed 3.04 on 4 -> 8 cubes; with the arithmetic mean of rho in
    the face average and penalty it drops to 1.24)."""
    r1, r2 = 1.0, 100.0
    c1 = (r1 - r2) / (2.0 * r1 * (r1 + r2))
    c2 = -r1 * c1 / r2

    def parts(x):
        left = x < 0.5
        g = np.where(left, x * (1 - x) / r1 + c1 * x, x * (1 - x) / r2 + c2 * (1 - x))
        return np.where(left, r1, r2), g

    def u(X):
        return parts(X[..., 0])[1] * np.sin(math.pi * X[..., 1]) * np.sin(math.pi * X[..., 2])

    def f(X):
        rho, g = parts(X[..., 0])
        return (2.0 + rho * 2.0 * math.pi ** 2 * g) * np.sin(math.pi * X[..., 1]) * np.sin(math.pi * X[..., 2])

    errs = []
    for n in (4, 8):
        mesh = I.cube_tet_mesh(n)
        rho = np.where(mesh.vertex_mean()[:, 0] < 0.5, r1, r2)
        A, b, geo, _ = assemble3(mesh, 2, rho, 10.0, f)
        x = spla.spsolve(A.tocsc(), b)
        errs.append(l2_error3(mesh, 2, geo, x, u))
    assert math.log2(errs[0] / errs[1]) >= 2.75, errs


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
