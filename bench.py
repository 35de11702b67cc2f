"""Benchmark: two-level additive Schwarz PCG throughput on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload C4] [--no-cpu-baseline]

A step is one complete preconditioned CG solve (zero initial guess to
relative residual 1e-8: operator apply, fused vector updates and dot
products, batched local solves, coarse restrict/solve/prolong, iteration
control) with the operator, local solvers and coarse solver already resident
in HBM. Setup phases (host assembly, batched factorisation and inversion,
coarse setup) are reported separately. The local solves are applied through
the packed explicit inverses A_i^{-1} (default) and/or the two triangular
sweeps (`--local inverse,sweeps`); subdomains of at most 64 DoFs use whole
small inverses applied inside the prolongation. Each mode reports the true
residual of its solution and, where the FP64 oracle's solve of the workload
is stored (tests/golden), the error against it.

metric = DoF-iterations per second = n_dofs * iterations / PCG wall time,
for the FP32-local mode (local solvers stored and applied in FP32, everything
else FP64) as `value`, with the plain FP64 mode beside it.

Defaults: 2 warm-up solves, then 5 timed solves per mode (captured-graph
replay); each mode also reports the per-solve times and their median, and
one or two eager solves with HIP events around every local-apply launch for
the kernel's roofline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG-ASM DoF-iters/sec at ~1M DoFs; solves/sec + p99 latency, FP32-local vs FP64"
HBM_PEAK_GBS = 8000.0
# dense MFMA peaks of MI355X (TFLOP/s)
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}

WORKLOADS = {
    "C2": "Voronoi 16384 cells (seed 1, two Lloyd steps), p=2, 98304 DoFs, 64 subdomains (8x8 centroid bins), "
          "nested coarse = subdomains, q=1",
    "C3": "Voronoi 65536 cells (seed 2, two Lloyd steps), p=3, 655360 DoFs, 256 uneven subdomains (warped bins), "
          "nested coarse = subdomains, q=2",
    "C3x": "Voronoi 104858 cells (seed 4, two Lloyd steps), p=3, 1048580 DoFs, 256 uneven subdomains (warped bins, 2060..8920 "
           "DoFs), nested coarse = subdomains, q=2 (labelled extra at ~1M DoFs)",
    "C4": "Voronoi 131072 cells (seed 3, two Lloyd steps), p=2, 786432 DoFs, 512 subdomains (32x16 bins of "
          "the cells' vertex means), rho per subdomain 10^U[-4,4], non-nested coarse Voronoi of 64 cells "
          "(two Lloyd steps), q=1, f=1",
    "T1": "unit cube, 32^3 cubes of 6 Kuhn tetrahedra (196608 cells), p=1, 786432 DoFs, one element per "
          "subdomain, 384 nested Kuhn agglomerates (coarse grid 4^3 cubes), q=1, f = 3 pi^2 sin sin sin",
    "T1b": "the T1 mesh and load with 512 box subdomains (8^3 boxes of 384 tetrahedra, 1536 DoFs each), 384 nested "
           "Kuhn agglomerates, p=q=1, 786432 DoFs",
    "T3": "unit cube, 16^3 cubes of 6 Kuhn tetrahedra (24576 cells), p=3, 491520 DoFs, one element per subdomain, "
          "384 nested Kuhn agglomerates, q=3 (7680 coarse DoFs)",
    "C4h": "C4's mesh, rho (10^U[-4,4] per 32x16 bin) and load with one element per subdomain (131072 "
           "subdomains of 6 DoFs) and the 512 bins as nested agglomerated coarse cells, q=1 (1536 coarse DoFs)",
}


def measured_traffic(workload, mode, local="sweeps"):
    """HBM bytes per local-solve launch from the committed rocprofv3 counter
    summary, if it was taken on this workload/mode with the current kernel
    source; else None."""
    import hashlib

    kern = "k_symv" if local == "inverse" else "k_trsv"
    path = os.path.join(ROOT, "profiles", f"{kern}_{workload}_{mode}_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_1903_11357_amd", "csrc",
                       "kern_symv.hip" if local == "inverse" else "kern_trsv.hip")
    if not os.path.exists(path):
        return None
    meta = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("source_sha256_16", "traffic_bytes_per_launch"):
            k, v = line.split(":", 1)
            meta[k] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if meta.get("source_sha256_16") != sha:
        print(f"[bench] WARNING: {os.path.relpath(path, ROOT)} was taken on another kernel source; "
              f"roofline.traffic is reported as null until it is re-taken", file=sys.stderr, flush=True)
        return None
    return float(meta["traffic_bytes_per_launch"])


def local_solve_bytes(pr, word_bytes, inverse=False):
    """Algorithmic bytes of one batched local solve. Triangular sweeps: each
    of the two sweeps reads the packed lower triangle n_i(n_i+1)/2 of every
    factor once; vectors: r (FP64 read), y (write + read), z (write).
    Explicit inverse: one read of the packed lower triangle of every
    A_i^{-1} and of r (FP64); the per-DoF sum of the tile partials is done by
    the prolongation kernel, outside the timed launch."""
    import numpy as np

    n_i = pr._sub_sizes().astype(np.float64)
    if inverse:
        return float((n_i * (n_i + 1) / 2).sum()) * word_bytes + pr.n * 8
    factor = float((n_i * (n_i + 1)).sum()) * word_bytes
    vec = pr.n * (8 + 3 * word_bytes)
    return factor + vec


def oracle_reference(workload):
    """The FP64 oracle's stored solve of this workload (written by
    tests/golden/make_full_reference.py), or None."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", f"{workload}_oracle_fp64.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def run_mode(P, precision, steps, warmup, check_every, inverse=False, autotune=True, ref=None, schedules=(0, 0)):
    import torch

    from paper_1903_11357_amd import asdg

    t0 = time.perf_counter()
    pr = asdg.Problem()
    pr.assemble(P.mesh, P.p, P.c_sigma, P.rho, P.subdomain, P.f)
    if inverse:
        pr.set_tuning(asdg.TUNE_LOCAL_INVERSE, 1)
    pr.set_tuning(asdg.TUNE_FACTOR_SCHEDULE, schedules[0])
    pr.set_tuning(asdg.TUNE_INVERSE_SCHEDULE, schedules[1])
    pr.plan(precision, P.q, coarse_of_cell=P.coarse_of_cell if P.coarse_mesh is None else None,
            coarse_mesh=P.coarse_mesh)
    t1 = time.perf_counter()
    pr.bind("cuda:0")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pr.factor()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    tuned = pr.autotune() if autotune else None
    torch.cuda.synchronize()
    t3b = time.perf_counter()
    pr.setup_coarse()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    x = torch.empty(pr.n, dtype=torch.float64, device="cuda:0")
    for _ in range(warmup):
        pr.solve(x=x, rtol=P.rtol, max_iter=P.max_iter, check_every=check_every, raise_on_noconv=False)
    # kernel-timing pass (untimed for the metric): the same solve launched
    # eagerly with HIP events around every local-solve launch, on the stream
    # it is launched on (events inside a captured graph bracket nothing)
    n_eager = min(steps, 2)
    torch.cuda.synchronize()
    tl, nl, its_e = 0.0, 0, 0
    ta = time.perf_counter()
    for _ in range(n_eager):
        _, st = pr.solve(x=x, rtol=P.rtol, max_iter=P.max_iter, check_every=check_every, time_kernels=True,
                         use_graph=False, raise_on_noconv=False)
        its_e += st["iterations"]
        tl += st["t_local_ms"]
        nl += st["n_local"]
    torch.cuda.synchronize()
    total_eager = time.perf_counter() - ta
    # timed pass: exactly `steps` solves replayed as captured hipGraphs,
    # bracketed by device synchronisation (each solve returns after the
    # host has read its final state)
    its, lat = [], []
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        _, st = pr.solve(x=x, rtol=P.rtol, max_iter=P.max_iter, check_every=check_every, raise_on_noconv=False)
        lat.append(time.perf_counter() - s0)
        its.append(st["iterations"])
    torch.cuda.synchronize()
    total_graph = time.perf_counter() - tg0
    # untimed: the error of this solve against the FP64 oracle's stored
    # solution, and in FP64 mode the iterate after exactly the oracle's
    # iteration count against the oracle's iterate after that count
    err = None
    if ref is not None and "x" in ref and int(ref["n"]) == pr.n:
        import numpy as np

        xo = ref["x"]
        nxo = float(np.linalg.norm(xo))
        err = {"oracle_iterations": int(ref["iterations"]), "oracle_true_rel_res": float(ref["true_rel_res"]),
               "rel_err_vs_oracle": float(np.linalg.norm(x.cpu().numpy() - xo)) / nxo}
        if precision == asdg.FP64:
            xk = torch.empty_like(x)
            pr.solve(x=xk, rtol=0.0, max_iter=int(ref["iterations"]), check_every=check_every,
                     raise_on_noconv=False)
            err["same_iterations_rel_err_vs_oracle"] = float(np.linalg.norm(xk.cpu().numpy() - xo)) / nxo
            del xk
    w = 4 if precision == asdg.FP32_LOCAL else 8
    small = pr.is_small()
    # dense flops of the factorisation: Cholesky sum n_i^3/3, and with explicit
    # inverses X = L^{-1} (n_i^3/3) and S = X^T X (n_i^3/3)
    n_i = pr._sub_sizes().astype(float)
    fl = float((n_i ** 3).sum()) / 3.0 * (3.0 if (inverse or small) else 1.0)
    peak = MFMA_PEAK_TFLOPS["fp32" if precision == asdg.FP32_LOCAL else "fp64"]
    res = {
        "dof_iters_per_s": pr.n * sum(its) / total_graph,
        "iterations": its[-1],
        "ms_per_step": 1e3 * total_graph / steps,
        "ms_per_iteration": 1e3 * total_graph / sum(its),
        "solve_ms": [1e3 * v for v in lat],
        "solve_ms_median": 1e3 * statistics.median(lat),
        "kernel_timing_pass": {"mode": "eager", "solves": n_eager, "ms_per_step": 1e3 * total_eager / n_eager,
                               "dof_iters_per_s": pr.n * its_e / total_eager},
        "converged": st["converged"],
        "rel_res": st["rel_res"],
        "true_rel_res": st["true_rel_res"],
        "vs_fp64_oracle": err,
        "kappa_lanczos": st["lambda_max"] / st["lambda_min"] if st["lambda_min"] > 0 else None,
        "setup_s": {"assemble_plan_host": t1 - t0, "bind_upload": t2 - t1, "factor": t3 - t2,
                    "autotune": t3b - t3, "coarse": t4 - t3b},
        "library_phase_ms": {"assemble": st["t_assemble_ms"], "factor": st["t_factor_ms"],
                             "coarse": st["t_coarse_ms"], "pcg": st["t_solve_ms"]},
        "autotune": tuned,
        "factor_mfma": {"flops": fl, "tflops": fl / (t3 - t2) / 1e12, "peak_tflops": peak,
                        "frac": fl / (t3 - t2) / 1e12 / peak,
                        "note": "dense flops over the wall time of asdg_factor (gather, Cholesky"
                                + (", inverse formation" if inverse else "") + ", status reads)"},
        "local_solve": ({"representation": "whole small inverses applied inside k_prolong (no launch of its own)",
                         "bytes_per_apply": float((pr._sub_sizes().astype(float) ** 2).sum()) * w}
                        if small else
                        {"avg_ms": tl / max(nl, 1), "launches": nl,
                         "algorithmic_bytes": local_solve_bytes(pr, w, inverse),
                         "representation": "explicit inverse" if inverse else "triangular sweeps"}),
    }
    ls = res["local_solve"]
    if ls.get("avg_ms"):
        ls["achieved_gbs"] = ls["algorithmic_bytes"] / (ls["avg_ms"] * 1e-3) / 1e9
        ls["frac_of_hbm_peak"] = ls["achieved_gbs"] / HBM_PEAK_GBS
        ls["share_of_iteration"] = ls["avg_ms"] / res["ms_per_iteration"]
    del pr
    torch.cuda.empty_cache()
    return res


def _cpu_baseline_child(workload, n_iter, conn):
    """Process of the CPU baseline: builds the oracle for the workload
    (untimed, on one host thread), reports ready, waits for the go (sent once
    the GPU work is done, so the timing does not compete with it), then times
    the oracle's PCG and sends the result."""
    from oracle import OracleSolver
    from paper_1903_11357_amd import inputs

    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except ImportError:  # pragma: no cover
        import contextlib

        def threadpool_limits(n):
            return contextlib.nullcontext()

        def threadpool_info():
            return []

    t0 = time.perf_counter()
    # one host thread while it overlaps the serving run (whose host assembly
    # workers take the rest of the host's CPUs)
    with threadpool_limits(1):
        orc = OracleSolver(inputs.make_config(workload))
    conn.send(("ready", time.perf_counter() - t0))
    conn.recv()
    A, M = orc.A, orc.M
    with threadpool_limits(1):
        t = time.perf_counter()
        orc.solve(fixed_iters=n_iter)
        dt = time.perf_counter() - t
    blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    t1 = time.perf_counter()
    orc.solve(fixed_iters=1)
    dt1 = time.perf_counter() - t1
    sfb = sparse_factor_bound(A, M)
    conn.send(({"value": A.shape[0] * n_iter / dt, "unit": "DoF-iters/s", "cores": 1, "kind": "oracle",
                "sample": f"{n_iter} PCG iterations of the full workload (oracle setup untimed, built in a "
                          f"process of its own beside the GPU work), {dt:.1f} s, BLAS limited to 1 thread "
                          f"({os.cpu_count()} host CPUs visible)",
                "all_blas_threads": {"value": A.shape[0] / dt1, "threads": int(blas_threads),
                                     "sample": f"1 PCG iteration, {dt1:.2f} s"}}, sfb))


def start_cpu_baseline(workload, n_iter):
    """The FP64 oracle (NumPy/SciPy) timed on the host, in a process of its
    own: its setup runs beside the GPU work; finish_cpu_baseline() starts the
    timed part (n_iter PCG iterations, BLAS limited to one thread, the
    threads it actually uses: its sparse products and per-subdomain
    triangular solves run on one core; one iteration with all BLAS threads is
    reported beside it and is no faster)."""
    import multiprocessing as mp

    ctx = mp.get_context("spawn")
    parent, child = ctx.Pipe()
    proc = ctx.Process(target=_cpu_baseline_child, args=(workload, n_iter, child), daemon=True)
    proc.start()
    return proc, parent


def finish_cpu_baseline(handle):
    proc, conn = handle
    msg, setup_s = conn.recv()
    assert msg == "ready"
    conn.send("go")
    res, sfb = conn.recv()
    proc.join(timeout=60)
    res["oracle_setup_s"] = setup_s
    return res, sfb


def sparse_factor_bound(A, M, sample=32, seed=0):
    """Bytes a sparse factor of the same A_i would move, as a lower-bound
    context for the dense packed factors: SuperLU with a minimum-degree
    ordering of A_i + A_i^T and diagonal pivoting, nnz(L) per subdomain on a
    seeded sample of subdomains, scaled to all of them by the dense
    lower-triangle sizes. Values in FP32 plus one int32 row index each."""
    import numpy as np
    import scipy.sparse.linalg as spla

    rng = np.random.default_rng(seed)
    pick = rng.choice(len(M.dofs), size=min(sample, len(M.dofs)), replace=False)
    nnz = dense = 0.0
    for i in pick:
        d = M.dofs[i]
        lu = spla.splu(A[d][:, d].tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                       options={"SymmetricMode": True})
        nnz += lu.L.nnz
        dense += len(d) * (len(d) + 1) / 2
    all_dense = float(sum(len(d) * (len(d) + 1) / 2 for d in M.dofs))
    ratio = nnz / dense
    return {"sample_subdomains": int(len(pick)), "nnz_L_over_dense_lower": ratio,
            "sparse_L_bytes_fp32": ratio * all_dense * (4 + 4), "dense_lower_bytes_fp32": all_dense * 4,
            "ordering": "SuperLU MMD_AT_PLUS_A, symmetric mode"}


def start_serving_inputs(n_meshes, seed=5, workers=12):
    """Starts generating the serving workload's mesh pool in worker
    processes (the requests' input data, not part of the served work)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    from paper_1903_11357_amd import inputs

    specs = inputs.serving_mesh_specs(n_meshes, seed=seed)
    ex = ProcessPoolExecutor(max_workers=max(1, min(workers, os.cpu_count() or 1)),
                             mp_context=mp.get_context("spawn"))
    # largest meshes first: the pool finishes sooner
    futs = {sp["mesh_id"]: ex.submit(inputs.serving_mesh, sp)
            for sp in sorted(specs, key=lambda d: -d["n_cells"])}
    return ex, futs, time.perf_counter()


def serving_bench(n_requests, gen, seed=5, local_inverse=True, loads=(0.8,), capacity_requests=400,
                  max_active=4):
    """Continuous batching (C5): requests with log-uniform 4096..65536-cell
    Voronoi meshes (a pool of relaxed Voronoi meshes, one per stratum of
    log n, each request picking one uniformly), p uniform in {1,2,3}, about
    64 cells per subdomain, rho = 10^U[-2,2] per subdomain and a random
    sine-series load from the request's own seed, nested coarse q=1,
    FP32-local. First a burst of `capacity_requests` requests at once
    (capacity), then all n_requests as Poisson streams at the given fractions
    of that capacity; latency = arrival to completion. The top level reports
    the first load, `sweep` all of them."""
    from paper_1903_11357_amd import asdg, inputs
    from paper_1903_11357_amd.serve import Request, Server, latency_stats

    import numpy as np

    ex, futs, t_start = gen
    pool = {k: f.result() for k, f in futs.items()}
    ex.shutdown(wait=True)
    t_gen = time.perf_counter() - t_start
    descs = inputs.serving_pool_requests(n_requests, len(pool), seed=seed + 1)
    problems = [inputs.serving_pool_problem(d, pool) for d in descs]
    print(f"[bench] serving: {len(pool)} pool meshes ready {t_gen:.1f} s after the start; {n_requests} requests",
          file=sys.stderr, flush=True)
    srv = Server(precision=asdg.FP32_LOCAL, max_active=max_active, check_every=16, setup_workers=8,
                 local_inverse=local_inverse)
    ncap = min(capacity_requests, n_requests)
    burst = srv.run([Request(i, P, 0.0) for i, P in enumerate(problems[:ncap])],
                    on_done=lambda n, tot, t: n % 100 == 0 and print(
                        f"[bench] serving: burst {n}/{tot} requests done at {t:.1f} s", file=sys.stderr, flush=True))
    cap = latency_stats(burst)
    print(f"[bench] serving: capacity {cap['solves_per_s']:.2f} solves/s ({ncap} requests at once)",
          file=sys.stderr, flush=True)
    sweep = []
    for k, load in enumerate(loads):
        rate = load * cap["solves_per_s"]
        rng = np.random.default_rng(seed + 10 + k)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
        t0 = time.perf_counter()

        def report(n_done, n_total, t, load=load):
            if n_done % 200 == 0 or n_done == n_total:
                print(f"[bench] serving: load {load}: {n_done}/{n_total} requests done at {t:.1f} s",
                      file=sys.stderr, flush=True)

        st = latency_stats(srv.run([Request(i, P, float(a)) for i, (P, a) in enumerate(zip(problems, arrivals))],
                                   on_done=report))
        st.update({"load": load, "arrival_rate_per_s": rate, "wall_s": time.perf_counter() - t0})
        sweep.append(st)
        print(f"[bench] serving: load {load}: p50 {st['p50_ms']:.0f} ms p99 {st['p99_ms']:.0f} ms",
              file=sys.stderr, flush=True)
    st = sweep[0]
    dofs = [P.n_dofs for P in problems]
    return {"requests": n_requests, "mesh_pool": len(pool), "dofs_min": int(min(dofs)), "dofs_max": int(max(dofs)),
            "capacity_solves_per_s": cap["solves_per_s"], "capacity_requests": ncap,
            "arrival_rate_per_s": st["arrival_rate_per_s"],
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
            "solves_per_s": st["solves_per_s"], "iterations_mean": st["iterations_mean"],
            "all_converged": all(x["all_converged"] for x in sweep) and cap["all_converged"],
            "peak_active": srv.peak_active, "max_active": max_active, "input_generation_s": t_gen,
            "precision": "fp32-local",
            "local_solves": "explicit inverses" if local_inverse else "triangular sweeps",
            "capacity_run": cap, "sweep": sweep}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C4", choices=sorted(WORKLOADS))
    ap.add_argument("--check-every", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--modes", default="fp32,fp64")
    ap.add_argument("--local", default="inverse",
                    help="local-solve representations, the first is the headline: inverse (packed "
                         "A_i^{-1}, one pass) and/or sweeps (Cholesky forward/backward sweeps)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (no asdg_autotune after the factorisation)")
    ap.add_argument("--schedules", default="0,0",
                    help="Cholesky and X = L^-1 schedules before any autotuning (0 automatic, 1 tile tasks, "
                         "2 subdomain / block-column tasks); profiling runs of each kernel")
    ap.add_argument("--max-iter", type=int, default=0,
                    help="cap PCG iterations (profiling runs; 0 = the workload's own limit)")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of the continuous-batching run (0 = skip)")
    ap.add_argument("--serving-meshes", type=int, default=128,
                    help="meshes in the serving workload's mesh pool (log-uniform strata of 4096..65536 cells)")
    ap.add_argument("--serving-capacity-requests", type=int, default=400,
                    help="requests of the burst run that measures the serving capacity")
    ap.add_argument("--serving-max-active", type=int, default=int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4),
                    help="requests on the GPU at once, each with its own stream (default: the HIP runtime's "
                         "hardware queues, GPU_MAX_HW_QUEUES, 4 unless set)")
    ap.add_argument("--only-serving", action="store_true")
    ap.add_argument("--serving-local", default="inverse", choices=("sweeps", "inverse"),
                    help="local solvers of the served requests (explicit inverses: 1.3-2.3x less GPU time per "
                         "request than the sweeps, whose dependency chain dominates at these sizes)")
    ap.add_argument("--serving-loads", default="0.8",
                    help="Poisson arrival rates as fractions of the measured capacity, comma-separated")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (reference kernel for HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU layout is a design "
              f"note, not built", file=sys.stderr)
        sys.exit(2)

    # host-side inputs (the serving mesh pool) and the CPU baseline's oracle
    # setup run in processes of their own, started after the timed solves so
    # that nothing competes with them for the host
    gen = start_serving_inputs(a.serving_meshes) if a.serving_requests > 0 and a.only_serving else None
    baseline = None

    import torch

    from paper_1903_11357_amd import asdg, inputs

    asdg.lib()  # fail loudly if the native library is missing
    if a.calibrate_copy_mib:
        n = a.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    serve_kw = dict(local_inverse=a.serving_local == "inverse", loads=tuple(float(v) for v in a.serving_loads.split(",")),
                    capacity_requests=a.serving_capacity_requests, max_active=a.serving_max_active)
    if a.only_serving:
        print(json.dumps({"serving": serving_bench(a.serving_requests, gen, **serve_kw)}), flush=True)
        return
    P = inputs.make_config(a.workload)
    if a.max_iter:
        P.max_iter = a.max_iter
    print(f"[bench] workload {a.workload}: n={P.n_dofs} subdomains={P.n_sub}", file=sys.stderr, flush=True)
    modes = {}
    ref = oracle_reference(a.workload)
    for loc in a.local.split(","):
        for m in a.modes.split(","):
            prec = asdg.FP32_LOCAL if m == "fp32" else asdg.FP64
            key = m if loc == "inverse" else f"{m}-sweeps"
            modes[key] = run_mode(P, prec, a.steps, a.warmup, a.check_every, inverse=(loc == "inverse"),
                                  autotune=not a.no_autotune, ref=ref,
                                  schedules=tuple(int(v) for v in a.schedules.split(",")))
            print(f"[bench] {key}: {json.dumps(modes[key])}", file=sys.stderr, flush=True)
    if a.serving_requests > 0:
        gen = start_serving_inputs(a.serving_meshes)
    if not a.no_cpu_baseline:
        baseline = start_cpu_baseline(a.workload, a.cpu_iters)
    first = a.local.split(",")[0]
    hk = lambda m: m if first == "inverse" else f"{m}-sweeps"  # noqa: E731
    head = modes.get(hk("fp32")) or modes.get(hk("fp64"))
    ls = head["local_solve"]
    achieved = (ls["algorithmic_bytes"] / (ls["avg_ms"] * 1e-3) / 1e9
                if ls.get("avg_ms") and ls.get("algorithmic_bytes") else None)
    out = {
        "metric": METRIC,
        "value": head["dof_iters_per_s"],
        "unit": "DoF-iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-local+f64" if hk("fp32") in modes else "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {WORKLOADS[a.workload]}", "n_dofs": P.n_dofs,
                   "subdomains": P.n_sub, "rtol": P.rtol, "parallelism": "single GPU"},
        "modes": modes,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic(a.workload, "fp32" if hk("fp32") in modes else "fp64", first),
                     "kernel": ("k_symv_tiles (packed local inverses)" if first == "inverse"
                                else "k_trsv (batched local forward+backward sweeps)"),
                     "algorithmic_bytes": ls.get("algorithmic_bytes"), "avg_ms": ls.get("avg_ms")},
    }
    if hk("fp64") in modes:
        f64 = modes[hk("fp64")]
        out["value_fp64"] = {"value": f64["dof_iters_per_s"], "unit": "DoF-iters/s",
                             "ms_per_step": f64["ms_per_step"], "iterations": f64["iterations"],
                             "note": "the paper's precision: every step in FP64"}
    if hk("fp32") in modes and hk("fp64") in modes:
        f32, f64 = modes[hk("fp32")], modes[hk("fp64")]
        out["fp32_local_speedup_per_iteration"] = f64["ms_per_iteration"] / f32["ms_per_iteration"]
        out["fp32_local_speedup_per_solve"] = f64["ms_per_step"] / f32["ms_per_step"]
    if a.serving_requests > 0:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = serving_bench(a.serving_requests, gen, **serve_kw)
    if baseline is not None:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"], out["sparse_factor_bound"] = finish_cpu_baseline(baseline)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
