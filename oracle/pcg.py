"""Additive Schwarz preconditioned CG and the Lanczos condition estimate
(oracle; test infrastructure).

Protocol of Sec. 7: CG preconditioned by P_ad, trivial initial guess, stop
when the Euclidean norm of the residual relative to the initial residual
(= b for x_0 = 0) drops below the tolerance (1e-8 in the paper), condition
number estimated from the extreme eigenvalues of the Lanczos matrix built
from the CG coefficients.

Iteration (k = 0, 1, ...): q = A p_k; alpha_k = (r_k.z_k)/(p_k.q);
x += alpha_k p_k; r -= alpha_k q; stop if ||r|| <= tol ||b|| (iterations =
k+1); z = M^{-1} r; beta_k = (r_{k+1}.z_{k+1})/(r_k.z_k); p = z + beta_k p.

Lanczos matrix (standard CG-Lanczos relation): T_00 = 1/alpha_0,
T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j.

Pins: agreement with a dense direct solve; Lanczos estimate against the
dense eigenvalues of M^{-1}A on small meshes; at most two iterations when the
spectrum is {1, 2}.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as la


@dataclasses.dataclass
class PCGInfo:
    iterations: int
    converged: bool
    rel_res: float
    true_rel_res: float
    alphas: list
    betas: list
    history: list
    history_after: list = dataclasses.field(default_factory=list)  # residuals past the stop (extra)

    def lanczos(self):
        k = len(self.alphas)
        a = np.asarray(self.alphas)
        b = np.asarray(self.betas)
        d = np.empty(k)
        d[0] = 1.0 / a[0]
        for j in range(1, k):
            d[j] = 1.0 / a[j] + b[j - 1] / a[j - 1]
        e = np.sqrt(b[:k - 1]) / a[:k - 1]
        ev = la.eigvalsh_tridiagonal(d, e) if k > 1 else d
        return float(ev.min()), float(ev.max())

    def condition_estimate(self):
        lo, hi = self.lanczos()
        return hi / lo


def pcg(A, b, apply_Minv, rtol=1e-8, max_iter=10000, fixed_iters=None, extra=0):
    """Returns (x, PCGInfo). With ``fixed_iters`` the loop runs exactly that
    many iterations regardless of the tolerance. With ``extra`` > 0 the same
    iteration continues that many steps past the stop and only their
    residual norms are kept (PCGInfo.history_after); x, the coefficients and
    the statistics are those of the stop."""
    n = b.shape[0]
    x = np.zeros(n)
    r = b.copy()
    bnorm = float(np.linalg.norm(b))
    z = apply_Minv(r)
    p = z.copy()
    rz = float(r @ z)
    alphas, betas, hist = [], [], []
    it = 0
    converged = False
    limit = fixed_iters if fixed_iters is not None else max_iter
    after = []
    stopped = None  # (iterate, iteration count) at the stop while extra steps run
    k = 0
    while limit > 0:
        q = A @ p
        pq = float(p @ q)
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        res = float(np.linalg.norm(r))
        k += 1
        if stopped is None:
            alphas.append(alpha)
            hist.append(res / bnorm)
            it = k
            if fixed_iters is None and res <= rtol * bnorm:
                converged = True
            if converged or it == limit:
                if extra <= 0:
                    break
                stopped = (x.copy(), it)
        else:
            after.append(res / bnorm)
            if len(after) == extra:
                break
        z = apply_Minv(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        if stopped is None:
            betas.append(beta)
        p = z + beta * p
        rz = rz_new
    if stopped is not None:
        x = stopped[0]
    true_res = float(np.linalg.norm(b - A @ x)) / bnorm
    return x, PCGInfo(it, converged, hist[-1] if hist else 0.0, true_res, alphas, betas, hist, after)
