"""Continuous-batching server: results are identical alone and in the mix,
admission respects the HBM budget, served solutions match the oracle,
rejected requests complete with their error while the others are served."""
import numpy as np
import pytest

from paper_1903_11357_amd import inputs as I

pytestmark = pytest.mark.gpu


def _problems(k=6):
    out = []
    for i in range(k):
        n = [600, 900, 1400, 700, 1100, 2000][i % 6]
        p = [1, 2, 3, 2, 1, 3][i % 6]
        out.append(I.serving_problem({"id": i, "n_cells": n, "p": p, "seed": 1000 + i}))
    return out


def _run(problems, arrivals, **kw):
    from paper_1903_11357_amd.serve import Request, Server

    srv = Server(keep_solutions=True, check_every=8, **kw)
    calls = []
    done = srv.run([Request(i, P, a) for i, (P, a) in enumerate(zip(problems, arrivals))],
                   on_done=lambda n, tot, t: calls.append((n, tot, t)))
    # one completion report per request, in completion order
    assert [c[0] for c in calls] == list(range(1, len(problems) + 1))
    assert all(c[1] == len(problems) for c in calls)
    assert [c[2] for c in calls] == [r.t_done for r in done]
    return {r.rid: r for r in done}, srv


@pytest.mark.parametrize("local_inverse", [True, False], ids=["inverse", "sweeps"])
def test_results_identical_alone_and_in_the_mix(local_inverse):
    from paper_1903_11357_amd import asdg

    probs = _problems()
    solo, _ = _run(probs, [0.0] * len(probs), max_active=1, local_inverse=local_inverse)
    mixed, srv = _run(probs, [0.0] * len(probs), max_active=len(probs), local_inverse=local_inverse)
    assert srv.peak_active >= 3
    for i in range(len(probs)):
        a, b = solo[i], mixed[i]
        assert a.status == b.status == "OK"
        assert a.iterations == b.iterations
        assert bool((a.x == b.x).all()), i
    # the same request through the blocking solve entry point
    P = probs[2]
    pr = asdg.setup_problem(P, asdg.FP32_LOCAL, device="cuda:0", local_inverse=local_inverse)
    x, st = pr.solve(rtol=1e-8, check_every=8)
    assert st["iterations"] == mixed[2].iterations
    assert bool((x == mixed[2].x).all())


def test_admission_respects_hbm_budget():
    from paper_1903_11357_amd import asdg

    probs = _problems()
    sizes = []
    for P in probs:
        pr = asdg.Problem()
        pr.assemble(P.mesh, P.p, P.c_sigma, P.rho, P.subdomain, P.f)
        pr.set_tuning(asdg.TUNE_LOCAL_INVERSE, 1)  # the server's default local solvers
        sizes.append(sum(pr.plan(asdg.FP32_LOCAL, P.q, coarse_of_cell=P.coarse_of_cell)))
    budget = int(2.2 * max(sizes))
    arrivals = list(np.arange(len(probs)) * 0.002)
    done, srv = _run(probs, arrivals, max_active=8, hbm_budget=budget)
    assert len(done) == len(probs)
    assert srv.peak_bytes <= budget
    assert all(r.status == "OK" for r in done.values())
    assert all(r.t_admitted >= r.arrival for r in done.values())


def test_served_fp64_solution_matches_oracle():
    from oracle import OracleSolver
    from paper_1903_11357_amd import asdg

    probs = _problems(3)
    done, _ = _run(probs, [0.0, 0.0, 0.0], max_active=3, precision=asdg.FP64)
    for i, P in enumerate(probs):
        orc = OracleSolver(P)
        xk, info = orc.solve(fixed_iters=done[i].iterations)
        xg = done[i].x.cpu().numpy()
        assert np.linalg.norm(xg - xk) <= 1e-10 * np.linalg.norm(xk)


def _bad_problems(P):
    """A clockwise cell (rejected by the assembly) and a degree the library
    does not take (rejected before any work)."""
    import dataclasses

    cw = P.mesh.cell_vertices.copy()
    a, b = P.mesh.cell_ptr[0], P.mesh.cell_ptr[1]
    cw[a:b] = cw[a:b][::-1]
    mesh = dataclasses.replace(P.mesh, cell_vertices=cw)
    return [dataclasses.replace(P, mesh=mesh), dataclasses.replace(P, p=0)]


@pytest.mark.gpu
def test_rejected_requests_complete_with_their_error_and_the_rest_are_served():
    probs = _problems(4)
    bad = _bad_problems(probs[0])
    mix = [probs[0], bad[0], probs[1], bad[1], probs[2], probs[3]]
    done, srv = _run(mix, [0.0] * len(mix), max_active=4)
    assert len(done) == len(mix)
    for i in (1, 3):
        assert done[i].status == "EINVAL" and done[i].error and done[i].iterations == 0
        assert done[i].x is None
    ok = [i for i in range(len(mix)) if i not in (1, 3)]
    assert all(done[i].status == "OK" and not done[i].error for i in ok)
    # the served requests are the ones served without the rejected neighbours
    alone, _ = _run([mix[i] for i in ok], [0.0] * len(ok), max_active=4)
    for k, i in enumerate(ok):
        assert done[i].iterations == alone[k].iterations
        assert bool((done[i].x == alone[k].x).all())
    from paper_1903_11357_amd.serve import latency_stats

    st = latency_stats(list(done.values()))
    assert st["n"] == 4 and st["failed"] == 2 and st["all_converged"]
