"""The 32-row tile layout of the local Cholesky factors (ASDG_TUNE_TILE 32,
triangular sweeps) against the FP64 CPU oracle, through the C ABI: the
factor tiles against a dense Cholesky factorisation of the oracle's A_i,
the local solves subdomain by subdomain, FP64 PCG under the same rule as
the 64-row layout, FP32-local PCG to 1e-8, both factorisation schedules
bitwise equal, one subdomain of 188 tile rows, and the autotuner's switch
between the two edges inside the bound buffers."""
import numpy as np
import pytest

from paper_1903_11357_amd import inputs as I
from test_gpu_parity import CASES, _assert_per_subdomain, _check_pcg_parity, _rel, _vec

pytestmark = pytest.mark.gpu

_cache = {}


def _oracle(name):
    from oracle import OracleSolver

    if name not in _cache:
        P = CASES[name]()
        _cache[name] = (P, OracleSolver(P))
    return _cache[name]


def _setup(name, precision, tile=32):
    import torch

    from paper_1903_11357_amd import asdg

    P, orc = _oracle(name)
    print(f"[tile {tile}] {name} precision={precision} n={P.n_dofs}", flush=True)
    pr = asdg.setup_problem(P, precision, device="cuda:0", tile=tile)
    torch.cuda.synchronize()
    assert pr.info()[7] == tile
    return P, orc, pr


def _tiles(pr, sub, word, tile):
    """Raw factor tiles of subdomain `sub` (packed lower by tile rows, each
    tile row-major tile x tile; diagonal tiles hold inv(L_bb))."""
    import ctypes

    from paper_1903_11357_amd import asdg

    nb = (int(pr._sub_sizes()[sub]) + tile - 1) // tile
    buf = np.empty(nb * (nb + 1) // 2 * tile * tile, dtype=np.float32 if word == 4 else np.float64)
    st = asdg.lib().asdg_export_factor_tiles(pr.h, sub, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes)
    assert st == asdg.OK
    return buf.reshape(-1, tile, tile).astype(np.float64)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_factor_tiles_match_dense_cholesky(prec):
    """Every stored 32x32 tile of three subdomains' factors: off-diagonal
    tiles equal the blocks of L_i = chol(A_i) (A_i the oracle's principal
    submatrix, padded by the identity to whole tiles), diagonal tiles equal
    inv(L_bb), within the perturbation bound of the factorisation,
    64 u kappa(A_i) relative to the tile's largest entry (u = 2^-53 in FP64,
    2^-24 in FP32)."""
    from paper_1903_11357_amd import asdg

    name = "vor_p2_big"
    P, orc, pr = _setup(name, asdg.FP64 if prec == "fp64" else asdg.FP32_LOCAL)
    word = 8 if prec == "fp64" else 4
    T = 32
    for i in sorted({0, P.n_sub // 2, P.n_sub - 1}):
        d = orc.M.dofs[i]
        Ai = orc.A[d][:, d].toarray()
        n = Ai.shape[0]
        nb = (n + T - 1) // T
        Ap = np.eye(nb * T)
        Ap[:n, :n] = Ai
        L = np.linalg.cholesky(Ap)
        ev = np.linalg.eigvalsh(Ai)
        tol = 64 * 2.0 ** (-53 if prec == "fp64" else -24) * ev[-1] / ev[0]
        tiles = _tiles(pr, i, word, T)
        worst = 0.0
        for b in range(nb):
            for j in range(b + 1):
                ref = L[b * T:(b + 1) * T, j * T:(j + 1) * T]
                if b == j:
                    ref = np.linalg.inv(ref)
                got = tiles[b * (b + 1) // 2 + j]
                e = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
                worst = max(worst, e)
        print(f"{name} sub {i} n={n} {prec}: worst tile error {worst:.2e} (bound {tol:.2e})")
        assert worst <= tol, (i, worst, tol)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_local_apply_matches_oracle(name, prec):
    import torch

    from paper_1903_11357_amd import asdg

    P, orc, pr = _setup(name, asdg.FP64 if prec == "fp64" else asdg.FP32_LOCAL)
    v = _vec(pr.n, 2)
    loc = pr.apply(asdg.APPLY_LOCAL, torch.from_numpy(v).cuda()).cpu().numpy()
    _assert_per_subdomain(name, orc, loc, orc.M.local_apply(v), prec, "32-row sweeps local apply")


@pytest.mark.parametrize("name", sorted(CASES))
def test_pcg_fp64_matches_oracle(name):
    from paper_1903_11357_amd import asdg

    P, orc, pr = _setup(name, asdg.FP64)
    x, st = pr.solve(rtol=1e-8)
    _check_pcg_parity(name, orc, st, x.cpu().numpy())


@pytest.mark.parametrize("name", ["C4r", "vor_p3_nonnested", "vor_p2_big"])
def test_pcg_fp32_local_solution_within_1e8(name):
    import math

    import scipy.sparse.linalg as spla

    from paper_1903_11357_amd import asdg

    P, orc, pr = _setup(name, asdg.FP32_LOCAL)
    x, st = pr.solve(rtol=1e-12, max_iter=5000)
    xd = spla.spsolve(orc.A.tocsc(), orc.b)
    xg = x.cpu().numpy()
    e = xg - xd
    err2 = _rel(xg, xd)
    erra = math.sqrt(e @ (orc.A @ e)) / math.sqrt(xd @ (orc.A @ xd))
    print(f"{name}: 32-row fp32-local iterations={st['iterations']} rel2={err2:.2e} relA={erra:.2e}")
    assert err2 <= 1e-8 and erra <= 1e-8


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_factor_schedules_bitwise_equal(prec):
    """Tile tasks and one work-group per subdomain run the same products in
    the same order with 32-row tiles too."""
    from paper_1903_11357_amd import asdg

    P, orc = _oracle("C4r")
    precision = asdg.FP64 if prec == "fp64" else asdg.FP32_LOCAL
    word = 8 if prec == "fp64" else 4
    out = []
    for sched in (1, 2):
        print(f"[tile 32] schedule {sched} {prec}", flush=True)
        pr = asdg.setup_problem(P, precision, device="cuda:0", tile=32, factor=False)
        pr.set_tuning(asdg.TUNE_FACTOR_SCHEDULE, sched)
        pr.factor()
        pr.setup_coarse()
        tiles = [_tiles(pr, i, word, 32) for i in (0, P.n_sub - 1)]
        x, st = pr.solve(rtol=1e-8)
        out.append((tiles, x.cpu().numpy(), st["iterations"]))
        del pr
    (t1, x1, k1), (t2, x2, k2) = out
    for a, b in zip(t1, t2):
        assert np.array_equal(a, b)
    assert k1 == k2 and np.array_equal(x1, x2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_large_subdomain(prec):
    """One subdomain of 6000 DoFs in 188 tile rows (17766 stored tiles): the
    longest task chains of the 32-row factorisation and sweeps."""
    import torch

    from oracle import OracleSolver
    from paper_1903_11357_amd import asdg

    if "one_large" not in _cache:
        P = I.voronoi_problem(1000, 33, p=2, bx=1, by=1, q=1)
        orc = OracleSolver(P)
        ev = np.linalg.eigvalsh(orc.A.toarray())
        _cache["one_large"] = (P, orc, ev[-1] / ev[0])
    P, orc, kappa = _cache["one_large"]
    assert P.n_sub == 1 and P.n_dofs == 6000
    precision = asdg.FP64 if prec == "fp64" else asdg.FP32_LOCAL
    print(f"[tile 32] one large subdomain {prec}", flush=True)
    pr = asdg.setup_problem(P, precision, device="cuda:0", tile=32)
    v = _vec(pr.n, 4)
    loc = pr.apply(asdg.APPLY_LOCAL, torch.from_numpy(v).cuda()).cpu().numpy()
    ref = orc.M.local_apply(v)
    x, st = pr.solve(rtol=1e-8)
    if prec == "fp64":
        assert _rel(loc, ref) <= 1e-10, _rel(loc, ref)
        _check_pcg_parity("one_large", orc, st, x.cpu().numpy())
    else:
        assert _rel(loc, ref) <= 64 * 2.0 ** -24 * kappa, _rel(loc, ref)
        assert st["converged"] == 1
        res = np.linalg.norm(orc.b - orc.A @ x.cpu().numpy()) / np.linalg.norm(orc.b)
        assert res <= 1.05e-8, res


def test_autotuner_switches_edges_inside_bound_buffers(tmp_path):
    """With the automatic edge the plan has room for both layouts: the
    autotuner times both, keeps one, and the solve after tuning is bitwise
    the solve of a problem planned with that edge; a cached entry moves a
    second problem of the size class to the cached edge without timing, and
    the edge survives a save / load of the cache."""
    from paper_1903_11357_amd import asdg

    P, orc = _oracle("C4r")
    pr = asdg.setup_problem(P, asdg.FP32_LOCAL, device="cuda:0", factor=False)
    assert pr.info()[7] == 64
    rep = pr.autotune(asdg.AUTOTUNE_FACTOR | asdg.AUTOTUNE_LOCAL)
    print(f"[tile search] report {rep}", flush=True)
    tile = rep["tile"]
    assert tile in (32, 64) and pr.info()[7] == tile
    pr.setup_coarse()
    x1, st1 = pr.solve(rtol=1e-8)
    ref = asdg.setup_problem(P, asdg.FP32_LOCAL, device="cuda:0", tile=tile)
    x0, st0 = ref.solve(rtol=1e-8)
    assert st1["iterations"] == st0["iterations"]
    assert np.array_equal(x1.cpu().numpy(), x0.cpu().numpy())
    del ref

    # the other edge forced into the cache entry of this size class: a second
    # problem takes it from the cache (relaid out in its bound buffers)
    path = tmp_path / "tune.txt"
    asdg.tune_cache_save(str(path))
    lines = path.read_text().splitlines()
    key = [ln for ln in lines if "|fp32|sweeps|ns2^7|" in ln]
    assert key and key[0].split()[-1] == str(tile)
    other = 32 if tile == 64 else 64
    fields = key[0].split()
    fields[1] = "8" if other == 32 else "2"  # Cholesky work-groups per CU of that edge
    fields[-1] = str(other)
    path.write_text(" ".join(fields) + "\n")
    assert asdg.tune_cache_load(str(path)) == 1
    second = asdg.setup_problem(P, asdg.FP32_LOCAL, device="cuda:0", factor=False)
    rep2 = second.autotune(asdg.AUTOTUNE_FACTOR | asdg.AUTOTUNE_LOCAL | asdg.AUTOTUNE_REUSE)
    assert rep2["from_cache"] == 1 and rep2["tile"] == other and second.info()[7] == other
    second.setup_coarse()
    x2, st2 = second.solve(rtol=1e-8)
    ref2 = asdg.setup_problem(P, asdg.FP32_LOCAL, device="cuda:0", tile=other)
    x3, st3 = ref2.solve(rtol=1e-8)
    assert st2["iterations"] == st3["iterations"]
    assert np.array_equal(x2.cpu().numpy(), x3.cpu().numpy())
    # a line without the edge field (older files) loads as 64-row tiles
    path.write_text(" ".join(fields[:-1]) + "\n")
    assert asdg.tune_cache_load(str(path)) == 1
