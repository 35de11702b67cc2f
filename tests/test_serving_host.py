"""Serving loop on the host alone: requests that the library rejects before
any device work (invalid input at assembly or planning) complete with the
library's status and message, and requests whose device footprint exceeds
the whole HBM budget are rejected without being admitted."""
import dataclasses

from paper_1903_11357_amd import inputs as I


def _server(**kw):
    from paper_1903_11357_amd.serve import Server

    return Server(device="cuda:0", hbm_budget=kw.pop("hbm_budget", 1 << 40), max_active=2, setup_workers=2,
                  host_threads=1, **kw)


def test_requests_rejected_at_assembly_complete_with_their_error():
    from paper_1903_11357_amd.serve import Request, latency_stats

    P = I.serving_problem({"id": 0, "n_cells": 300, "p": 2, "seed": 5})
    cw = P.mesh.cell_vertices.copy()
    a, b = P.mesh.cell_ptr[0], P.mesh.cell_ptr[1]
    cw[a:b] = cw[a:b][::-1]
    bad = [dataclasses.replace(P, mesh=dataclasses.replace(P.mesh, cell_vertices=cw)),
           dataclasses.replace(P, p=0), dataclasses.replace(P, q=P.p + 1)]
    calls = []
    done = _server().run([Request(i, Q, 0.001 * i) for i, Q in enumerate(bad)],
                         on_done=lambda n, tot, t: calls.append((n, tot)))
    assert [c[0] for c in calls] == [1, 2, 3] and all(c[1] == 3 for c in calls)
    by = {r.rid: r for r in done}
    assert by[0].status == "EINVAL" and "clockwise" in by[0].error
    assert by[1].status == "EINVAL" and "p must be" in by[1].error
    assert by[2].status == "EINVAL" and "coarse degree" in by[2].error
    for r in done:
        assert r.iterations == 0 and r.x is None and r.t_done >= r.arrival
    assert latency_stats(done) == {"n": 0, "failed": 3}


def test_request_larger_than_the_budget_is_rejected_without_admission():
    from paper_1903_11357_amd.serve import Request

    P = I.serving_problem({"id": 0, "n_cells": 300, "p": 1, "seed": 6})
    srv = _server(hbm_budget=1024)
    done = srv.run([Request(0, P, 0.0)])
    assert done[0].status == "EBUDGET" and "HBM budget" in done[0].error
    assert srv.peak_active == 0 and srv.peak_bytes == 0
