"""Rounding spread of the FP64 oracle's PCG at full size (CPU; the evidence
behind the residual tolerance of the full-size GPU parity tests).

Runs the oracle's preconditioned CG (Sec. 3 preconditioner, Sec. 7 protocol)
on a full workload with the local and coarse solves applied through explicit
inverses (formed by Cholesky solves against the identity) instead of
triangular solves: equal to the oracle in exact arithmetic, different in
rounding. Compares it with the oracle's stored full solve
(make_full_reference.py): the iterate after the oracle's iteration count,
and the ratio of the two recursive residual histories per decade of the
residual. Prints the figures; writes nothing.

With --perturb EPS the variant also assembles differently: every stored
entry of A (symmetrically) and of b is multiplied by 1 + EPS xi, xi uniform
in [-1, 1] from a fixed seed, as an assembly that rounds each entry
differently would, and the local and coarse inverses are formed from that
A (the rounding-level differences two independent assemblies of the same
SIPG form have: an entry-wise median of about 1e-16 and a 99th percentile
of a few 1e-15 between the library's host assembly and the oracle's).

Usage: python tests/golden/full_rounding_spread.py C4 [--perturb 2e-15]   (about 40 min on one core)
"""
from __future__ import annotations

import os
import sys

import numpy as np
import scipy.linalg as la

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def perturbed(A, b, eps, seed=0):
    """A and b with every stored entry scaled by 1 + eps xi (A symmetrically)."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    U = sp.triu(A, format="coo")
    f = 1.0 + eps * rng.uniform(-1.0, 1.0, size=U.nnz)
    Up = sp.coo_matrix((U.data * f, (U.row, U.col)), shape=A.shape)
    Ap = (Up + sp.triu(Up, k=1, format="coo").T).tocsr()
    return Ap, b * (1.0 + eps * rng.uniform(-1.0, 1.0, size=b.shape[0]))


def main(name: str, eps: float = 0.0) -> None:
    from oracle import OracleSolver
    from oracle.pcg import pcg
    from oracle.schwarz import TwoLevelSchwarz
    from paper_1903_11357_amd import inputs as I

    ref = np.load(os.path.join(HERE, f"{name}_oracle_fp64.npz"), allow_pickle=False)
    P = I.make_config(name)
    orc = OracleSolver(P)
    A, b = orc.A, orc.b
    M = orc.M
    if eps > 0.0:
        A, b = perturbed(orc.A.tocsr(), orc.b, eps)
        M = TwoLevelSchwarz(A, P.mesh, P.p, orc.geo, P.subdomain, q=P.q, coarse_of_cell=P.coarse_of_cell,
                            coarse_mesh=P.coarse_mesh)
        print(f"[{name}] A and b perturbed by 1 + {eps:g} xi", flush=True)
    inv = [la.cho_solve(f, np.eye(len(d))) for d, f in zip(M.dofs, M.factors)]
    A0i = la.cho_solve(M.A0_factor, np.eye(M.A0.shape[0]))

    def apply(r):
        z = np.zeros_like(r)
        for d, S in zip(M.dofs, inv):
            z[d] = S @ r[d]
        return z + M.P0 @ (A0i @ (M.P0.T @ r))

    k = int(ref["iterations"])
    xk, info = pcg(A, b, apply, fixed_iters=k)
    h, hv = np.asarray(ref["history"]), np.asarray(info.history)
    print(f"[{name}] iterate after {k} iterations: ||x_var - x_oracle|| / ||x_oracle|| = "
          f"{np.linalg.norm(xk - ref['x']) / np.linalg.norm(ref['x']):.3e}" if "x" in ref.files else
          f"[{name}] (no stored iterate)")
    below = np.flatnonzero(hv <= 1e-8)
    print(f"[{name}] variant first below 1e-8 at iteration {below[0] + 1 if below.size else None}, oracle at {k}")
    ratio = np.maximum(hv / h, h / hv)
    for lo, hi in ((1e-8, 1e-7), (1e-7, 1e-6), (1e-6, 1e-3)):
        sel = (h >= lo) & (h < hi)
        if sel.any():
            print(f"[{name}] residual in [{lo:.0e}, {hi:.0e}): largest ratio of the two histories {ratio[sel].max():.3f}")


if __name__ == "__main__":
    args = sys.argv[1:]
    eps = 0.0
    if "--perturb" in args:
        i = args.index("--perturb")
        eps = float(args[i + 1])
        del args[i:i + 2]
    main(args[0] if args else "C4", eps)
