"""Continuous-batching request loop for two-level Schwarz PCG solves.

Requests (a mesh, coefficients and a right-hand side each) arrive over
time. The server
  * assembles arriving requests on host worker threads (the native assembly
    runs without the Python lock),
  * admits an assembled request when a slot is free and its exact device
    footprint (the four buffer sizes reported by asdg_plan) fits the HBM
    budget, then binds its buffers, factorises (explicit local inverses by
    default, which take 1.3-2.3 times less GPU time per request than the
    triangular sweeps at these sizes; the sweeps with local_inverse=False)
    and sets up the coarse level on the request's own stream,
  * keeps every admitted request's factors resident and advances all active
    solves in chunks of `check_every` PCG iterations, each on its own HIP
    stream (captured graphs), so the iterations of different requests are
    in flight on the device together; new requests join as slots and memory
    free up, finished ones leave at once and release their buffers,
  * records arrival-to-completion latency for every request,
  * completes a request that the library rejects (invalid input at
    assembly or planning, an error at binding, factorisation or coarse
    setup) or that can never fit the HBM budget with an error status and
    message, and goes on serving the others.

Each request's arithmetic is independent of the others' (own buffers,
deterministic kernels), so a result is the same alone and in the mix.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import os
import time
from typing import Callable, List, Optional

import numpy as np

from . import asdg


@dataclasses.dataclass
class Request:
    rid: int
    problem: object                 # inputs.Problem
    arrival: float = 0.0            # seconds after the start of the run
    # filled by the server
    t_assembled: float = -1.0
    t_admitted: float = -1.0
    t_done: float = -1.0
    iterations: int = 0
    status: str = ""               # "OK", a PCG status, or the error's status name
    error: str = ""                # the library's message for a rejected request
    bytes: int = 0
    x: Optional[object] = None      # torch tensor when keep_solutions

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class _Active:
    def __init__(self, req, pr, stream):
        self.req = req
        self.pr = pr
        self.stream = stream


def _host_setup(req, precision, local_inverse, host_threads=0):
    P = req.problem
    pr = asdg.Problem()
    if host_threads:
        pr.set_tuning(asdg.TUNE_HOST_THREADS, host_threads)
    pr.assemble(P.mesh, P.p, P.c_sigma, P.rho, P.subdomain, P.f)
    if local_inverse:
        pr.set_tuning(asdg.TUNE_LOCAL_INVERSE, 1)
    b = pr.plan(precision, P.q, coarse_of_cell=P.coarse_of_cell if P.coarse_mesh is None else None,
                coarse_mesh=P.coarse_mesh)
    return pr, int(sum(b))


def _device_setup(pr, device):
    """Buffers, factorisation and coarse level on a new stream of the request."""
    import torch

    stream = torch.cuda.Stream(device)
    with torch.cuda.stream(stream):  # buffers belong to the request's stream
        pr.bind(device, stream=stream)
    pr.factor(stream=stream)
    pr.setup_coarse(stream=stream)
    return stream


class Server:
    def __init__(self, device="cuda:0", precision=asdg.FP32_LOCAL, hbm_budget: Optional[int] = None,
                 max_active: Optional[int] = None, check_every: int = 16, setup_workers: int = 4,
                 keep_solutions: bool = False, rtol: float = 1e-8, max_iter: int = 20000,
                 local_inverse: bool = True, host_threads: Optional[int] = None):
        import torch

        self.device = torch.device(device)
        self.precision = precision
        if hbm_budget is None:
            free, total = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.5 * free)
        self.hbm_budget = hbm_budget
        # requests on the device at once: by default one per hardware queue
        # the HIP runtime gives the process (GPU_MAX_HW_QUEUES, 4 unless set);
        # more streams than queues only time-slice the queues
        if max_active is None:
            max_active = int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4)
        self.max_active = max_active
        self.check_every = check_every
        self.setup_workers = setup_workers
        self.keep_solutions = keep_solutions
        self.rtol = rtol
        self.max_iter = max_iter
        self.local_inverse = local_inverse
        # host threads per request setup: each worker's share of the host
        # (OMP_NUM_THREADS when set, as on shared machines, else the CPUs
        # this process may run on)
        if host_threads is None:
            share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
            if share <= 0:
                share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
            host_threads = max(1, share // max(1, setup_workers))
        self.host_threads = host_threads
        self.peak_active = 0
        self.peak_bytes = 0

    def run(self, requests: List[Request], on_done: Optional[Callable[[int, int, float], None]] = None
            ) -> List[Request]:
        """Serves `requests` (each admitted at its arrival time, seconds from
        the start) to completion; returns them in completion order.
        on_done(n_done, n_total, t) is called after each request completes."""
        # the host workers already run in parallel: BLAS inside user load
        # callbacks stays single-threaded meanwhile (no oversubscription)
        try:
            from threadpoolctl import threadpool_limits
        except ImportError:  # pragma: no cover
            import contextlib

            def threadpool_limits(limits):
                return contextlib.nullcontext()
        with threadpool_limits(limits=1):
            return self._run(requests, on_done)

    def _run(self, requests: List[Request], on_done=None) -> List[Request]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pool = cf.ThreadPoolExecutor(max_workers=self.setup_workers)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        nxt = 0                      # next request not yet arrived
        preparing = []               # (req, future) in arrival order
        active: List[_Active] = []
        used = 0
        done: List[Request] = []

        def reject(r, status, msg):
            r.status, r.error = status, msg
            r.t_done = now()
            if r.t_assembled < 0:
                r.t_assembled = r.t_done
            if r.t_admitted < 0:
                r.t_admitted = r.t_done
            done.append(r)
            if on_done is not None:
                on_done(len(done), len(reqs), r.t_done)

        try:
            while len(done) < len(reqs):
                t = now()
                # arrivals -> host assembly
                while nxt < len(reqs) and reqs[nxt].arrival <= t:
                    r = reqs[nxt]
                    preparing.append((r, pool.submit(_host_setup, r, self.precision, self.local_inverse,
                                                     self.host_threads)))
                    nxt += 1
                # admission in arrival order (no overtaking)
                while preparing and preparing[0][1].done() and len(active) < self.max_active:
                    r, fut = preparing[0]
                    try:
                        pr, nbytes = fut.result()
                    except asdg.AsdgError as e:
                        preparing.pop(0)
                        reject(r, asdg.STATUS_NAMES.get(e.status, str(e.status)), str(e))
                        continue
                    if r.t_assembled < 0:
                        r.t_assembled = now()
                    if nbytes > self.hbm_budget:
                        preparing.pop(0)
                        del pr
                        reject(r, "EBUDGET", f"request {r.rid} needs {nbytes} B, more than the HBM budget "
                                             f"({self.hbm_budget} B)")
                        continue
                    if used + nbytes > self.hbm_budget:
                        break
                    preparing.pop(0)
                    try:
                        stream = _device_setup(pr, self.device)
                        pr.begin(rtol=self.rtol, max_iter=self.max_iter, check_every=self.check_every,
                                 stream=stream)
                    except asdg.AsdgError as e:
                        del pr
                        reject(r, asdg.STATUS_NAMES.get(e.status, str(e.status)), str(e))
                        continue
                    r.bytes = nbytes
                    used += nbytes
                    self.peak_bytes = max(self.peak_bytes, used)
                    r.t_admitted = now()
                    active.append(_Active(r, pr, stream))
                    self.peak_active = max(self.peak_active, len(active))
                # advance / retire active solves
                progressed = False
                for a in list(active):
                    chunk_done, solve_done, its = a.pr.poll()
                    if not chunk_done:
                        continue
                    progressed = True
                    if solve_done:
                        x, st = a.pr.finish(stream=a.stream, raise_on_noconv=False)
                        r = a.req
                        r.t_done = now()
                        r.iterations = st["iterations"]
                        r.status = st["status"]
                        if self.keep_solutions:
                            import torch

                            with torch.cuda.stream(a.stream):
                                r.x = x.clone()
                            a.stream.synchronize()
                        used -= r.bytes
                        active.remove(a)
                        del a.pr
                        done.append(r)
                        if on_done is not None:
                            on_done(len(done), len(reqs), r.t_done)
                    else:
                        a.pr.step(stream=a.stream)
                if not progressed and not (preparing and preparing[0][1].done()):
                    time.sleep(2e-5)
        finally:
            pool.shutdown(wait=True)
        return done


def latency_stats(done: List[Request]) -> dict:
    """Latency and throughput over the solved requests; rejected requests
    (an error status from the library or the HBM budget) are counted
    apart."""
    failed = [r for r in done if r.error]
    done = [r for r in done if not r.error]
    if not done:
        return {"n": 0, "failed": len(failed)}
    lat = np.array([r.latency for r in done])
    span = max(r.t_done for r in done) - min(r.arrival for r in done)
    # where the latency goes: host assembly (arrival -> assembled), waiting for
    # a slot or HBM (assembled -> admitted, includes the device setup), solve
    asm = np.array([r.t_assembled - r.arrival for r in done])
    adm = np.array([r.t_admitted - r.t_assembled for r in done])
    dev = np.array([r.t_done - r.t_admitted for r in done])
    return {"n": len(done), "failed": len(failed), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "solves_per_s": len(done) / span if span > 0 else None,
            "iterations_mean": float(np.mean([r.iterations for r in done])),
            "all_converged": all(r.status == "OK" for r in done),
            "mean_assembly_ms": float(asm.mean() * 1e3), "mean_admission_ms": float(adm.mean() * 1e3),
            "mean_solve_ms": float(dev.mean() * 1e3)}
