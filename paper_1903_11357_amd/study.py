"""Condition-number study harness: the experiments of Sec. 7 on this
package's own meshes, solved on the GPU through the C ABI.

The paper's experiments use one element per subdomain, C_sigma = 10, CG
from a zero initial guess to a relative residual of 1e-8, and report the
extreme-eigenvalue estimate K(P_ad) from the CG coefficients with the
iteration count. Its meshes (an L-shaped domain, METIS agglomerates,
PolyMesher grids) are not available; the sweeps below run the same designs
on seeded Voronoi grids of the unit square with bin agglomerates as the
nested coarse grids:

- example1: dependence on coefficient jumps (Example 1). rho = 1 or rho_e in
  a checkerboard over the coarse agglomerates (aligned) or over the fine
  elements by index parity (not aligned); K should stay flat when aligned
  and grow like rho_e otherwise.
- example2: nested agglomerates, H/h sweeps (Example 2, Tables 3-4): K grows
  like (H/h)^2 along a row and stays roughly constant along diagonals.
- example3: tetrahedral fine grids of the unit cube (6 n^3 Kuhn tetrahedra)
  with the tetrahedra of coarser grids as nested agglomerates (Example 3,
  Tables 5-6): K grows like (H/h)^2 along a row and stays roughly constant
  along diagonals; plain CG rows give K(A_h).
- example4: independent (non-nested) coarse Voronoi grids (Example 4).
- example5: K(P_ad) against the polynomial degree p = q = 1..9 on nested
  square grids (Example 5, Fig. 6): n x n squares, coarse cells of
  block x block squares, f = 1; this design is the paper's own, so its
  printed values can be compared directly. With nonnested=True the coarse
  grid is an independent relaxed Voronoi grid of (n / block)^2 cells, the
  non-nested series of Fig. 6 (whose polygonal grids are not available);
  the analysis bounds the growth by O(p) (nested) and O(p^2) (non-nested).
- unpreconditioned CG on each fine grid: K(A_h) and its iteration count (the
  extra rows of Example 3's tables).

    python -m paper_1903_11357_amd.study --example 2 --p 1
"""
from __future__ import annotations

import argparse
import json
import math
from dataclasses import dataclass

import numpy as np

from . import asdg
from . import inputs as I


@dataclass
class Run:
    K: float
    iterations: int
    lambda_min: float
    lambda_max: float
    converged: bool


def run(P: I.Problem, precision: int = asdg.FP64, identity: bool = False, device: str = "cuda:0",
        rtol: float = 1e-8, max_iter: int = 20000) -> Run:
    """One CG solve of problem P on the GPU: preconditioned by the two-level
    additive Schwarz operator, or plain CG with identity=True."""
    pr = asdg.setup_problem(P, precision, device=device)
    if identity:
        pr.set_tuning(asdg.TUNE_NO_PRECOND, 1)
    _, st = pr.solve(rtol=rtol, max_iter=max_iter, raise_on_noconv=False)
    lo, hi = st["lambda_min"], st["lambda_max"]
    return Run(hi / lo if lo > 0 else math.inf, int(st["iterations"]), lo, hi, bool(st["converged"]))


def fine_grid(n_cells: int, seed: int) -> I.Mesh:
    return I.relaxed_voronoi_mesh(np.random.default_rng(seed).random((n_cells, 2)))


def agglomerates(mesh: I.Mesh, bins: int) -> np.ndarray:
    """Nested coarse grid: the non-empty cells of a bins x bins grid of
    the unit square, by the mean of each element's vertices."""
    return I.compact_labels(I.bins_partition(mesh.vertex_mean(), bins, bins))


def per_element(mesh: I.Mesh, p: int, coarse_of_cell=None, coarse_mesh=None, rho=None, q=None,
                f=I.f_sinsin, name: str = "study") -> I.Problem:
    n = mesh.n_cells
    return I.Problem(name=name, mesh=mesh, p=p, c_sigma=10.0, rho=np.ones(n) if rho is None else rho,
                     subdomain=np.arange(n, dtype=np.int32), q=p if q is None else q,
                     coarse_of_cell=coarse_of_cell, coarse_mesh=coarse_mesh, f=f)


def example5(ps=range(1, 10), n: int = 32, block: int = 4, device: str = "cuda:0", nonnested: bool = False,
             seed: int = 61) -> dict:
    """Example 5 (Fig. 6): one element per subdomain on n x n squares,
    coarse agglomerates of block x block squares (nested) or an independent
    relaxed Voronoi grid of as many cells (nonnested), q = p, rho = 1, f = 1."""
    out = {}
    coarse_mesh = fine_grid((n // block) ** 2, seed) if nonnested else None
    for p in ps:
        P = I.squares_problem(n, p, 1, block, q=p, f=I.f_one)
        cpl = None if nonnested else P.coarse_of_cell
        out[p] = run(per_element(P.mesh, p, coarse_of_cell=cpl, coarse_mesh=coarse_mesh, q=p, f=I.f_one,
                                 name="example5"), device=device)
    return out


def example1(p: int = 1, n_fine: int = 2000, bins: int = 4, rho_e=(1e1, 1e2, 1e3, 1e4, 1e5, 1e6), seed: int = 31,
             device: str = "cuda:0"):
    """Rows 'aligned' and 'not aligned': {rho_e: Run}."""
    mesh = fine_grid(n_fine, seed)
    coarse = agglomerates(mesh, bins)
    bx = np.minimum((mesh.vertex_mean()[:, 0] * bins).astype(int), bins - 1)
    by = np.minimum((mesh.vertex_mean()[:, 1] * bins).astype(int), bins - 1)
    even_agg = (bx + by) % 2 == 0
    even_elem = np.arange(mesh.n_cells) % 2 == 0
    out = {"aligned": {}, "not aligned": {}}
    for re in rho_e:
        for row, even in (("aligned", even_agg), ("not aligned", even_elem)):
            rho = np.where(even, re, 1.0)
            out[row][re] = run(per_element(mesh, p, coarse_of_cell=coarse, rho=rho), device=device)
    return out


def example2(p: int = 1, n_finest: int = 4096, levels: int = 4, seed: int = 41, device: str = "cuda:0",
             with_identity: bool = True):
    """Fine grids of n_finest / 4^k elements (h = 2^k hbar, k = levels-1..0)
    and nested agglomerates with H = 2^m hbar (bins = sqrt(n_finest) / 2^m),
    H >= 2h. Returns ({(m, k): Run}, {k: Run of plain CG})."""
    side = int(round(math.sqrt(n_finest)))
    table, plain = {}, {}
    for k in range(levels - 1, -1, -1):
        mesh = fine_grid(n_finest // 4 ** k, seed + k)
        for m in range(k + 1, levels + 1):
            bins = side >> m
            if bins < 1:
                continue
            P = per_element(mesh, p, coarse_of_cell=agglomerates(mesh, bins))
            table[(m, k)] = run(P, device=device)
        if with_identity:
            plain[k] = run(per_element(mesh, p, coarse_of_cell=agglomerates(mesh, 1)), identity=True,
                           device=device)
    return table, plain


def example4(p: int = 1, fine=(256, 1024, 4096), coarse=(16, 64, 256), seed: int = 51, device: str = "cuda:0"):
    """Independent coarse Voronoi grids (non-nested prolongation). Returns
    {(n_coarse, n_fine): Run} for n_coarse < n_fine."""
    out = {}
    for i, nf in enumerate(fine):
        mesh = fine_grid(nf, seed + i)
        for j, nc in enumerate(coarse):
            if nc >= nf:
                continue
            cmesh = fine_grid(nc, seed + 100 + j)
            out[(nc, nf)] = run(per_element(mesh, p, coarse_mesh=cmesh), device=device)
    return out


def example3(p: int = 1, fine=(4, 8, 16, 32), coarse=(2, 4, 8), device: str = "cuda:0", with_identity: bool = True,
             max_coarse_dofs: int = 16384):
    """Cube meshes of 6 n^3 tetrahedra for n in `fine`, coarse grids of the
    6 nc^3 Kuhn tetrahedra for nc in `coarse` (nc < n, n divisible by nc),
    one element per subdomain, q = p. Coarse spaces above max_coarse_dofs
    are skipped (A_0 is formed dense on the host). Returns
    ({(N_H, N_h): Run}, {N_h: Run of plain CG})."""
    nq = (p + 1) * (p + 2) * (p + 3) // 6
    table, plain = {}, {}
    for n in fine:
        for nc in coarse:
            if nc >= n or n % nc or 6 * nc ** 3 * nq > max_coarse_dofs:
                continue
            table[(6 * nc ** 3, 6 * n ** 3)] = run(I.tet_problem(n, p, nc), device=device)
        if with_identity:
            plain[6 * n ** 3] = run(I.tet_problem(n, p, 1), identity=True, device=device)
    return table, plain


def table_example3(p: int, table, plain) -> str:
    nh = sorted({k[1] for k in table} | set(plain))
    nH = sorted({k[0] for k in table})
    lines = [f"K(P_ad) (CG iterations), tetrahedra, nested Kuhn agglomerates, p = q = {p}",
             "| N_H \\ N_h | " + " | ".join(str(v) for v in nh) + " |", "|---" * (len(nh) + 1) + "|"]
    for H in nH:
        lines.append(f"| {H} | " + " | ".join(_fmt(table[(H, h)]) if (H, h) in table else "-" for h in nh) + " |")
    if plain:
        lines.append("| K(A_h), plain CG | " + " | ".join(_fmt(plain[h]) if h in plain else "-" for h in nh) + " |")
    return "\n".join(lines)


def _fmt(r: Run) -> str:
    return f"{r.K:.4g} ({r.iterations})" + ("" if r.converged else "*")


def table_example2(p: int, table, plain, levels: int) -> str:
    cols = list(range(levels - 1, -1, -1))
    lines = [f"K(P_ad) (CG iterations), nested agglomerates, p = q = {p}; hbar: the finest grid",
             "| H \\ h | " + " | ".join(f"{2 ** k} hbar" for k in cols) + " |",
             "|---" * (len(cols) + 1) + "|"]
    for m in range(levels, 0, -1):
        cells = [(_fmt(table[(m, k)]) if (m, k) in table else "-") for k in cols]
        lines.append(f"| {2 ** m} hbar | " + " | ".join(cells) + " |")
    if plain:
        lines.append("| K(A_h), plain CG | " + " | ".join(_fmt(plain[k]) for k in cols) + " |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--example", type=int, choices=(1, 2, 3, 4, 5), default=2)
    ap.add_argument("--p", type=int, default=1)
    ap.add_argument("--n-finest", type=int, default=4096)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--json", action="store_true")
    a = ap.parse_args(argv)
    if a.example == 1:
        res = example1(a.p)
        if a.json:
            print(json.dumps({row: {str(k): vars(v) for k, v in d.items()} for row, d in res.items()}))
        else:
            keys = list(res["aligned"])
            print("| rho_e | " + " | ".join(f"{k:.0e}" for k in keys) + " |")
            print("|---" * (len(keys) + 1) + "|")
            for row, d in res.items():
                print(f"| {row}, p={a.p} | " + " | ".join(_fmt(d[k]) for k in keys) + " |")
    elif a.example == 3:
        fine = (4, 8, 16, 32) if a.p == 1 else (4, 8, 16)
        table, plain = example3(a.p, fine=fine)
        if a.json:
            print(json.dumps({"table": {f"{H}/{h}": vars(v) for (H, h), v in table.items()},
                              "plain": {str(h): vars(v) for h, v in plain.items()}}))
        else:
            print(table_example3(a.p, table, plain))
    elif a.example == 2:
        table, plain = example2(a.p, a.n_finest, a.levels)
        if a.json:
            print(json.dumps({"table": {f"H=2^{m},h=2^{k}": vars(v) for (m, k), v in table.items()},
                              "plain": {f"h=2^{k}": vars(v) for k, v in plain.items()}}))
        else:
            print(table_example2(a.p, table, plain, a.levels))
    elif a.example == 5:
        res = {"nested": example5(), "non-nested": example5(nonnested=True)}
        if a.json:
            print(json.dumps({k: {str(p): vars(v) for p, v in d.items()} for k, d in res.items()}))
        else:
            ps = list(res["nested"])
            print("| p = q | " + " | ".join(str(p) for p in ps) + " |")
            print("|---" * (len(ps) + 1) + "|")
            for k, d in res.items():
                print(f"| {k} | " + " | ".join(_fmt(d[p]) for p in ps) + " |")
    else:
        res = example4(a.p)
        if a.json:
            print(json.dumps({f"{nc}/{nf}": vars(v) for (nc, nf), v in res.items()}))
        else:
            for (nc, nf), r in sorted(res.items()):
                print(f"| N_H = {nc} | N_h = {nf} | {_fmt(r)} |")


if __name__ == "__main__":
    main()
