"""Top-level oracle driver (test infrastructure): assemble, build the
two-level Schwarz preconditioner, run ASPCG. See the package docstring."""
from __future__ import annotations

import numpy as np

from .pcg import pcg
from .schwarz import TwoLevelSchwarz
from .sipg import assemble
from .tet import assemble3, n_basis3, prolongation_nested3


class OracleSolver:
    def __init__(self, problem, coarse=True, local=True, h=None):
        P = problem
        self.problem = P
        if getattr(P.mesh, "dim", 2) == 3:
            self.A, self.b, self.geo, self.faces = assemble3(P.mesh, P.p, P.rho, P.c_sigma, P.f)
            P0 = prolongation_nested3(P.mesh, P.p, P.q, self.geo, np.asarray(P.coarse_of_cell))[0] if coarse else None
            self.M = TwoLevelSchwarz(self.A, P.mesh, P.p, self.geo, P.subdomain, q=P.q, coarse=coarse,
                                     local=local, P0=P0, npb=n_basis3(P.p))
            return
        self.A, self.b, self.geo, self.faces = assemble(P.mesh, P.p, P.rho, P.c_sigma, P.f, h=h)
        self.M = TwoLevelSchwarz(self.A, P.mesh, P.p, self.geo, P.subdomain, q=P.q,
                                 coarse_of_cell=P.coarse_of_cell, coarse_mesh=P.coarse_mesh,
                                 coarse=coarse, local=local)

    def solve(self, rtol=None, max_iter=None, fixed_iters=None, b=None):
        P = self.problem
        rhs = self.b if b is None else b
        return pcg(self.A, rhs, self.M.apply, rtol=P.rtol if rtol is None else rtol,
                   max_iter=P.max_iter if max_iter is None else max_iter, fixed_iters=fixed_iters)


def solve(problem, **kw):
    s = OracleSolver(problem)
    x, info = s.solve(**kw)
    return x, info, s
