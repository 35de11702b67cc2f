"""GPU parity on tetrahedral meshes (the 3D case): every hot-path step and
the PCG iteration against the 3D oracle, through the C ABI, for one element
per subdomain (whole small inverses) and box subdomains (tiles: triangular
sweeps and explicit inverses), p = 1, 2, 3."""
import math

import numpy as np
import pytest

from paper_1903_11357_amd import inputs as I
from test_gpu_parity import _check_pcg_parity, _rel, _vec

pytestmark = pytest.mark.gpu

CASES3 = {
    # one element per subdomain (n_p = 4), nested coarse Kuhn agglomerates, q = 1
    "tet_p1_elem": lambda: I.tet_problem(4, 1, 2, jitter=0.1, seed=11),
    # 8 box subdomains of 48 tetrahedra (480 DoFs: ragged tiles), q = 1, rho jumps
    "tet_p2_boxes": lambda: _jumps(I.tet_problem(4, 2, 2, q=1, per_element=False, sub_boxes=2, jitter=0.1, seed=12)),
    # one element per subdomain, n_p = 20, q = 2
    "tet_p3_elem": lambda: I.tet_problem(2, 3, 1, q=2, jitter=0.05, seed=13),
    # 8 box subdomains of 48 tetrahedra (960 DoFs), q = 3
    "tet_p3_boxes": lambda: I.tet_problem(4, 3, 2, q=3, per_element=False, sub_boxes=2, seed=14),
}


def _jumps(P):
    P.rho = np.where(P.coarse_of_cell % 2 == 0, 100.0, 1.0)
    return P


_cache = {}


def _setup(name, precision, inverse=False):
    import torch

    from oracle import OracleSolver
    from paper_1903_11357_amd import asdg

    key = (name, precision, inverse)
    if key not in _cache:
        if (name, "oracle") not in _cache:
            P = CASES3[name]()
            _cache[(name, "oracle")] = (P, OracleSolver(P))
        P, orc = _cache[(name, "oracle")]
        print(f"[setup] {name} precision={precision} inverse={inverse} n={P.n_dofs}", flush=True)
        pr = asdg.setup_problem(P, precision, device="cuda:0", local_inverse=inverse)
        torch.cuda.synchronize()
        _cache[key] = (P, orc, pr)
    return _cache[key]


def _kappa_local(orc):
    return max(np.linalg.cond(orc.A[d][:, d].toarray()) for d in orc.M.dofs)


@pytest.mark.parametrize("name", sorted(CASES3))
def test_tet_operator_apply(name):
    import torch

    from paper_1903_11357_amd import asdg

    P, orc, pr = _setup(name, asdg.FP64)
    v = _vec(pr.n, 1)
    out = pr.apply(asdg.APPLY_OPERATOR, torch.from_numpy(v).cuda()).cpu().numpy()
    ref = orc.A @ v
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("name", sorted(CASES3))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("inverse", [False, True], ids=["sweeps", "inverse"])
def test_tet_local_and_coarse_apply(name, prec, inverse):
    import torch

    from paper_1903_11357_amd import asdg

    P, orc, pr = _setup(name, asdg.FP64 if prec == "fp64" else asdg.FP32_LOCAL, inverse)
    v = _vec(pr.n, 2)
    loc = pr.apply(asdg.APPLY_LOCAL, torch.from_numpy(v).cuda()).cpu().numpy()
    tol = 1e-10 if prec == "fp64" else 64 * 2.0 ** -24 * _kappa_local(orc)
    assert _rel(loc, orc.M.local_apply(v)) <= tol
    crs = pr.apply(asdg.APPLY_COARSE, torch.from_numpy(v).cuda()).cpu().numpy()
    assert _rel(crs, orc.M.coarse_apply(v)) <= 1e-10


@pytest.mark.parametrize("name", sorted(CASES3))
def test_tet_pcg_fp64_matches_oracle(name):
    from paper_1903_11357_amd import asdg

    P, orc, pr = _setup(name, asdg.FP64)
    x, st = pr.solve(rtol=1e-8)
    _check_pcg_parity("tet/" + name, orc, st, x.cpu().numpy())


@pytest.mark.parametrize("name", sorted(CASES3))
def test_tet_pcg_fp32_solution_within_1e8(name):
    import scipy.sparse.linalg as spla

    from paper_1903_11357_amd import asdg

    P, orc, pr = _setup(name, asdg.FP32_LOCAL, True)
    x, st = pr.solve(rtol=1e-12, max_iter=5000)
    xd = spla.spsolve(orc.A.tocsc(), orc.b)
    xg = x.cpu().numpy()
    e = xg - xd
    erra = math.sqrt(e @ (orc.A @ e)) / math.sqrt(xd @ (orc.A @ xd))
    print(f"{name}: fp32-local iterations={st['iterations']} rel2={_rel(xg, xd):.2e} relA={erra:.2e}")
    assert _rel(xg, xd) <= 1e-8 and erra <= 1e-8
