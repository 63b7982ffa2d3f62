#!/usr/bin/env python
"""Benchmark of the CG-accelerated block Cimmino path on one MI355X.

One step is one pass of the whole path over the workload:
row inner-product graph (GPU; rip_graph-partitioned workloads only) ->
partition (host C++) -> setup (permutation, transposes, factors on the GPU) ->
solve to a relative true residual of 1e-10 (GPU).  The headline `value` is
outer CG iterations per second of the solve phase (inputs resident in HBM;
for a batch, the iterations of all systems); time-to-tolerance and the other
phases are reported beside it.

The default workload is the batch of 256 2D convection-diffusion systems
(sides 48..256, 8 blocks each) in plain FP64, all systems in one batched
solve; the same run also solves the batch with FP32 projections (FP64 outer
CG) and reports both times to tolerance and their ratio, and times rip_graph
end to end on the 27-point 100^3 matrix (1e6 rows, 120M edges).

Usage: python bench.py [--steps K] [--warmup W]
                       [--workload cfg4|cfg1|cfg2|cfg3|cfg5|cfg5-rip|cfg5-band]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "outer Cimmino iters/s + time-to-1e-10 residual; % HBM roofline; mixed vs FP64"
HBM_PEAK_GBS = 8000.0

# Counter summaries of the dominant projection kernel per workload (HBM
# bytes per dispatch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this
# script, scaled by a plain copy's counts).  Each summary records the SHA-256
# of the kernel's source file; the traffic is reported only while that source
# is unchanged.
TRAFFIC_PROFILES = {
    ("cfg4", "fp64"): "profiles/k_band_sweep_f64_cd2d_batch256_K8.md",
    ("cfg4", "mixed-proj"): "profiles/k_band_sweep_f32_cd2d_batch256_K8.md",
    ("cfg2", "fp64"): "profiles/k_inner_grp_f64_cd3d_64cubed_K32.md",
    ("cfg2", "mixed-proj"): "profiles/k_inner_grp_f64v32_cd3d_64cubed_K32.md",
    ("cfg5", "mixed-proj"): "profiles/k_dense_apply_f32_st27_100cubed_K512.md",
    ("cfg5-band", "mixed-proj"): "profiles/k_band_sweep_f32_st27_100cubed_K512.md",
}


def measured_traffic(workload, precision):
    """(bytes per dispatch, profile path) from the workload's counter
    summary, or (None, reason) when there is none or its kernel changed."""
    import hashlib
    import re
    path = TRAFFIC_PROFILES.get((workload, precision))
    if path is None:
        return None, "no counter summary for this workload"
    full = os.path.join(ROOT, path)
    if not os.path.exists(full):
        return None, path + " missing"
    text = open(full).read()
    m_src = re.search(r"^source: (\S+) sha256 ([0-9a-f]{64})$", text, re.M)
    m_val = re.search(r"^traffic_bytes_per_dispatch: ([0-9.eE+-]+)$", text, re.M)
    if not (m_src and m_val):
        return None, path + " has no machine-readable traffic line"
    src = os.path.join(ROOT, m_src.group(1))
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != m_src.group(2):
        return None, "kernel source changed since " + path
    return float(m_val.group(1)), path


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg4")
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed", "mixed-proj"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=10,
                    help="outer iterations of each oracle solve in the CPU baseline sample")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32-projection solve of a batched workload")
    ap.add_argument("--method", default="cg", choices=["cg", "alg1", "block"],
                    help="cg: Algorithm 2 (default; with --nrhs, one CG per right-hand side "
                         "through bc_solve_multi); alg1: Algorithm 1 (plain block Cimmino) "
                         "with omega = 2 / (lambda_min + lambda_max) of H estimated by Lanczos "
                         "through bc_project before the timed solve; block: block CG on H for "
                         "the --nrhs right-hand sides (bc_solve_block)")
    ap.add_argument("--partitioner", default="greedy", choices=["greedy", "multilevel"],
                    help="partitioner of the rip_graph workloads (the configurations name the "
                         "greedy one)")
    ap.add_argument("--spectrum", action="store_true",
                    help="also compare the spectrum of H (Lanczos through bc_project) and the "
                         "CG iteration count for contiguous and greedy rip_graph blocks of the "
                         "workload's matrix")
    ap.add_argument("--nrhs", type=int, default=None,
                    help="right-hand sides of the single-system workload solved together by "
                         "bc_solve_multi (vector 0: the workload's f, the others A times a "
                         "seeded Gaussian vector); value then counts the outer iterations of "
                         "every right-hand side.  Without it: one bc_solve")
    ap.add_argument("--no-rip", action="store_true",
                    help="skip the rip_graph measurement on the 27-point 100^3 matrix")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only measure what plain device kernels reach against the 8 TB/s "
                         "datasheet peak (a streaming sum, a device copy, a += b) and print the "
                         "device properties; no solve")
    ap.add_argument("--compare", action="store_true",
                    help="also time plain FP64 on the same matrices (per system, one after "
                         "another, for a batch) and report the time-to-tolerance ratio")
    return ap.parse_args()


class Workload:
    """Host inputs of one bench configuration."""

    def __init__(self, name, precision=None):
        import workloads as W
        import paper_1710_07769_amd as bc
        self.name = name
        self.batched = False
        self.opts = {}
        self.tol = 1e-10
        if name == "cfg1":
            p = W.config1()
            self.problems, self.partition = [p], "contiguous"
            self.opts = {"projection": bc.BC_PROJ_DENSE_CHOL}
            self.desc = "cd2d-32 n=1024 K=4 contiguous, dense Cholesky, FP64"
        elif name == "cfg2":
            p = W.config2()
            self.problems, self.partition = [p], "greedy-rip"
            self.opts = {"projection": bc.BC_PROJ_INNER_CG}
            self.desc = "cd3d-64 n=262144 K=32 greedy-rip, inner CG, FP64"
        elif name == "cfg3":
            p = W.config3()
            self.problems, self.partition = [p], "contiguous"
            self.opts = {"projection": bc.BC_PROJ_INNER_CG, "precision": bc.BC_MIXED}
            self.desc = "powerlaw n=500000 K=64 uneven, inner CG, mixed"
        elif name == "cfg4":
            self.problems, self.partition = W.config4(), "contiguous"
            self.batched = True
            self.opts = {"precision": bc.BC_FP64}
            self.desc = ("256 x cd2d sides 48..256, K=8 each, batched, projection kind per "
                         "block by the byte model (banded FP64 Cholesky), plain FP64")
        elif name in ("cfg5", "cfg5-rip"):
            p = W.config5()
            self.problems = [p]
            self.partition = "greedy-rip" if name == "cfg5-rip" else "contiguous"
            self.opts = {"projection": bc.BC_PROJ_DENSE_CHOL, "precision": bc.BC_MIXED_PROJ}
            self.desc = ("st27-100 n=1e6 K=512 %s, dense FP64 Cholesky, FP32 triangular applies"
                         % self.partition)
        elif name == "cfg5-band":
            # the same matrix and blocks with sparse-factor projections:
            # banded FP64 Cholesky of each block after reverse Cuthill-McKee
            p = W.config5()
            self.problems, self.partition = [p], "contiguous"
            self.opts = {"projection": bc.BC_PROJ_BAND_CHOL, "precision": bc.BC_MIXED_PROJ}
            self.desc = ("st27-100 n=1e6 K=512 contiguous, banded FP64 Cholesky (RCM), FP32 "
                         "triangular applies")
        else:
            raise SystemExit("unknown workload " + name)
        if precision == "fp64":
            self.opts["precision"] = bc.BC_FP64
        elif precision == "mixed":
            self.opts["precision"] = bc.BC_MIXED
        elif precision == "mixed-proj":
            self.opts["precision"] = bc.BC_MIXED_PROJ
        if name == "cfg4" and self.opts["precision"] != bc.BC_FP64:
            self.desc = self.desc.replace("plain FP64", "FP32 applies, FP64 sparse products "
                                                        "and outer CG")
        self.precision = {bc.BC_FP64: "fp64", bc.BC_MIXED: "mixed",
                          bc.BC_MIXED_PROJ: "mixed-proj"}[self.opts.get("precision", bc.BC_FP64)]
        self.mixed = self.opts.get("precision", 0) in (bc.BC_MIXED, bc.BC_MIXED_PROJ)
        self.n = sum(q.n for q in self.problems)
        self.nnz = sum(q.A.nnz for q in self.problems)


def run_step(wl, f_dev, method="cg", partitioner="greedy", nrhs=None):
    """One pass of the whole path; returns a dict of phase times and stats.
    With nrhs given, f_dev holds nrhs right-hand sides (nrhs x n) for bc_solve_multi."""
    import torch
    import paper_1710_07769_amd as bc
    out = {"rip_ms": 0.0, "rip_spgemm_ms": 0.0, "partition_ms": 0.0}
    parts = []
    for q in wl.problems:
        if wl.partition == "greedy-rip":
            t0 = time.perf_counter()
            g = bc.rip_graph(q.n, q.A.rowptr, q.A.col, q.A.val)
            t1 = time.perf_counter()
            part = (bc.bc_partition_multilevel(g, q.K) if partitioner == "multilevel"
                    else bc.bc_partition_greedy(g, q.K))
            t2 = time.perf_counter()
            out["cutsize"], out["int_cut"] = bc.bc_partition_cut(g, part)
            out["rip_ms"] += (t1 - t0) * 1e3
            out["rip_spgemm_ms"] += bc.rip_graph_timing()["spgemm_ms"]
            out["partition_ms"] += (t2 - t1) * 1e3
            out["rip_edges"] = int(g.col.size)
        else:
            part = q.part()
        parts.append(part)
    t0 = time.perf_counter()
    # several right-hand sides run on the sliced-ELL copies of A, built here
    # whatever their padding
    opts = bc.make_opts(**(dict(wl.opts, spmv_lanes=-1) if nrhs is not None else wl.opts))
    if wl.batched:
        ctx = bc.bc_setup_batched([(q.n, q.A.rowptr, q.A.col, q.A.val, q.K, pt)
                                   for q, pt in zip(wl.problems, parts)], opts)
    else:
        q = wl.problems[0]
        ctx = bc.bc_setup(q.n, q.A.rowptr, q.A.col, q.A.val, q.K, parts[0], opts)
    torch.cuda.synchronize()
    out["setup_ms"] = (time.perf_counter() - t0) * 1e3
    out["lanes"] = bc.bc_schedule(ctx)
    kind, bw = bc.bc_block_info(ctx)
    out["block_kinds"] = {"dense": int((kind == bc.KIND_DENSE).sum()),
                          "inner_cg": int((kind == bc.KIND_INNER).sum()),
                          "banded": int((kind == bc.KIND_BAND).sum())}
    if (kind == bc.KIND_BAND).any():
        out["block_kinds"]["max_half_bandwidth"] = int(bw.max())
    try:
        x = torch.empty_like(f_dev)
        if method == "alg1":
            # relaxation parameter from the spectrum of H (outside the timed solve)
            from paper_1710_07769_amd.spectrum import spectrum_of
            t0 = time.perf_counter()
            spec = spectrum_of(ctx, wl.n, steps=40, seed=0)
            out["lanczos_ms"] = (time.perf_counter() - t0) * 1e3
            out["spectrum"] = {"lambda_min": spec.lambda_min, "lambda_max": spec.lambda_max,
                               "omega": spec.omega_opt, "lanczos_steps": spec.steps}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = bc.bc_cimmino(ctx, f_dev, None, spec.omega_opt, wl.tol, 100000, x)
        elif method == "block":
            t0 = time.perf_counter()
            sts = bc.bc_solve_block(ctx, nrhs, f_dev, None, wl.tol, 10000, x)
        elif nrhs is not None:
            t0 = time.perf_counter()
            sts = bc.bc_solve_multi(ctx, nrhs, f_dev, None, wl.tol, 10000, x)
        elif wl.batched:
            t0 = time.perf_counter()
            sts = bc.bc_solve_batched(ctx, f_dev, None, wl.tol, 10000, x)
        else:
            t0 = time.perf_counter()
            sts = [bc.bc_solve(ctx, f_dev, None, wl.tol, 10000, x)]
        torch.cuda.synchronize()
        out["solve_ms"] = (time.perf_counter() - t0) * 1e3
    finally:
        bc.bc_destroy(ctx)
    out["iterations"] = sum(s.iterations for s in sts)
    out["sys_iters"] = [int(s.iterations) for s in sts]
    out["max_iterations"] = max(s.iterations for s in sts)
    out["status"] = max(abs(s.status) for s in sts)
    out["rel_residual"] = max(s.rel_residual for s in sts)
    out["t_proj_ms"] = sts[0].t_proj_ms
    out["proj_launches"] = sts[0].proj_launches
    out["proj_bytes"] = sts[0].proj_bytes
    out["inner_iterations"] = sts[0].inner_iterations
    out["x"] = x
    return out


def spectrum_study(wl, f_dev, steps=60):
    """Contiguous (uniform) against greedy and multilevel rip_graph blocks of the same matrix
    (Section 2, the paper's spectrum study): extreme Ritz values of H after
    `steps` Lanczos steps through bc_project, kappa, the share of Ritz values
    within 0.1 of 1, and the CG iterations and time to the workload's tol."""
    import torch
    import paper_1710_07769_amd as bc
    import workloads as W
    from paper_1710_07769_amd.spectrum import spectrum_of
    q = wl.problems[0]
    out = {}
    g = bc.rip_graph(q.n, q.A.rowptr, q.A.col, q.A.val)
    for name in ("contiguous", "greedy-rip", "multilevel-rip"):
        if name == "contiguous":
            part = W.blocks_to_part(W.contiguous_blocks(q.n, q.K))
        elif name == "greedy-rip":
            part = bc.bc_partition_greedy(g, q.K)
        else:
            part = bc.bc_partition_multilevel(g, q.K)
        ctx = bc.bc_setup(q.n, q.A.rowptr, q.A.col, q.A.val, q.K, part, bc.make_opts(**wl.opts))
        try:
            sp = spectrum_of(ctx, q.n, steps=steps, seed=0)
            x = torch.empty_like(f_dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = bc.bc_solve(ctx, f_dev, None, wl.tol, 10000, x)
            torch.cuda.synchronize()
            out[name] = {"cutsize": bc.bc_partition_cut(g, part)[0],
                         "lambda_min": sp.lambda_min, "lambda_max": sp.lambda_max,
                         "kappa": sp.kappa, "lanczos_steps": sp.steps,
                         "ritz_within_0.1_of_1": float(np.mean(np.abs(sp.ritz - 1.0) <= 0.1)),
                         "cg_iterations": st.iterations,
                         "time_to_tol_ms": (time.perf_counter() - t0) * 1e3}
        finally:
            bc.bc_destroy(ctx)
        print("[bench] spectrum %s: %s" % (name, out[name]), file=sys.stderr, flush=True)
    return out


def rip_graph_bench(reps=3):
    """rip_graph end to end on the 27-point 100^3 matrix (n = 1e6, 120M
    edges): host CSR in, pinned host graph out.  Reported with the time of
    the two sparse-product passes (HIP events), edges/s, and the passes'
    bytes per second against two byte counts: compulsory (each pass reads A
    and the compacted A^T once; the count pass writes the row counts, the
    emit pass reads the row offsets and writes the graph) and gathered (each
    product reads its column entry of A^T: index and value)."""
    import paper_1710_07769_amd as bc
    import workloads as W
    q = W.config5()
    n, nnz = q.n, q.A.nnz
    ccount = np.bincount(q.A.col, minlength=n)
    t = int(np.sqrt(n))
    products = int(np.minimum(ccount, t)[q.A.col].sum())
    wall, spg, tot = [], [], []
    ne = 0
    for _ in range(reps):
        t0 = time.perf_counter()
        g = bc.rip_graph(n, q.A.rowptr, q.A.col, q.A.val)
        wall.append((time.perf_counter() - t0) * 1e3)
        tm = bc.rip_graph_timing()
        spg.append(tm["spgemm_ms"])
        tot.append(tm["total_ms"])
        ne = int(g.col.size)
        del g
    a_bytes = (n + 1) * 4 + nnz * 12          # rowptr, col, value
    at_bytes = (n + 1) * 4 + int(np.minimum(ccount, t).sum()) * 12
    compulsory = 2 * (a_bytes + at_bytes) + n * 4 + (n + 1) * 8 + ne * 20
    gathered = 2 * (a_bytes + products * 12) + n * 4 + (n + 1) * 8 + ne * 20
    sp_s = min(spg) / 1e3
    out = {"matrix": "27-point stencil 100^3, n=%d nnz=%d" % (n, nnz), "edges": ne,
           "products_per_pass": products,
           "end_to_end_ms": min(wall), "library_total_ms": min(tot), "spgemm_ms": min(spg),
           "edges_per_s_end_to_end": ne / (min(wall) / 1e3),
           "edges_per_s_spgemm": ne / sp_s,
           "spgemm_gbs_compulsory": compulsory / sp_s / 1e9,
           "spgemm_gbs_gathered": gathered / sp_s / 1e9,
           "compulsory_bytes": compulsory, "gathered_bytes": gathered,
           "reps": reps, "times": "best of the repetitions"}
    print("[bench] rip_graph st27-100: %s" % out, file=sys.stderr, flush=True)
    return out


def _oracle_sample_worker(args):
    """One oracle solve of the CPU baseline (a process of its own): the
    oracle's projection setup, then `iters` outer iterations of Algorithm 2
    (tol = 0), or of Algorithm 1 with relaxation `omega`.  The iteration
    phase starts at a barrier shared by all workers so that the sample's
    wall time covers iterations running side by side."""
    q, part, iters, omega, barrier = args
    from oracle import BlockProjections, block_cimmino_cg, block_cimmino_plain
    A = q.A.to_scipy()
    t0 = time.perf_counter()
    B = BlockProjections(A, part, q.K)
    t1 = time.perf_counter()
    if barrier is not None:
        barrier.wait()
    t2 = time.perf_counter()
    if omega is None:
        block_cimmino_cg(A, q.f, part, q.K, tol=0.0, maxit=iters, proj=B)
    else:
        block_cimmino_plain(A, q.f, part, q.K, omega=omega, tol=0.0, maxit=iters, proj=B)
    t3 = time.perf_counter()
    return {"name": q.name, "setup_s": t1 - t0, "start": t2, "end": t3, "iters": iters}


def _pool_init():
    # one thread per worker process: the workers are the parallelism
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"


def cpu_baseline(wl, iters, omega=None, sys_iters=None):
    """The oracle timed on the host cores on a bounded sample of the workload.

    A batch: one oracle solve per worker process, one worker per host core
    (at most 16), on systems spread evenly over the batch's sizes, all
    iterating at once.  Each sampled system's time per outer iteration
    (measured with all workers running) stands for the batch's systems
    nearest to it in size; the batch's CPU time is then the sum, over its
    systems, of the outer iterations the GPU solve took (`sys_iters`) times
    that per-iteration time, spread over the cores, and value = the batch's
    outer iterations over that time.  One system: the oracle's own solve,
    its BLAS on every host core.  Each solve is the oracle's projection setup
    (reported separately) and then its first `iters` outer iterations."""
    import multiprocessing as mp
    from oracle import rip_graph, greedy_partition
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    if wl.batched:
        cores = min(cores, len(wl.problems))
        order = np.argsort([q.n for q in wl.problems], kind="stable")
        pick = [int(order[int(round(i * (len(order) - 1) / max(cores - 1, 1)))])
                for i in range(cores)]
        qs = [wl.problems[i] for i in pick]
        ctx = mp.get_context("spawn")
        with ctx.Manager() as mgr:
            barrier = mgr.Barrier(len(qs))
            with ctx.Pool(len(qs), initializer=_pool_init) as pool:
                res = pool.map(_oracle_sample_worker,
                               [(q, q.part(), iters, omega, barrier) for q in qs])
        wall = max(r["end"] for r in res) - min(r["start"] for r in res)
        per_it = np.array([(r["end"] - r["start"]) / r["iters"] for r in res])
        ns = np.array([q.n for q in qs], dtype=float)
        its = np.asarray(sys_iters if sys_iters is not None else [iters] * len(wl.problems),
                         dtype=float)
        near = [int(np.argmin(np.abs(ns - q.n))) for q in wl.problems]
        cpu_s = float(np.sum(its * per_it[near])) / len(qs)
        sides = sorted(int(round(np.sqrt(q.n))) for q in qs)
        return {"value": float(its.sum()) / cpu_s, "unit": "outer iters/s", "cores": len(qs),
                "kind": "oracle",
                "sample": "%d of the %d systems (grid sides %s), one oracle process per host "
                          "core (1 BLAS thread each): projection setup (%.1f s mean), then %d "
                          "outer CG iterations each, all started together (%.1f s until the "
                          "last finished); scaled to the whole batch: each system's outer "
                          "iterations in the GPU solve (%d in all) at the per-iteration time of "
                          "the sampled system nearest in size, over %d cores = %.0f s; %d host "
                          "cores visible"
                          % (len(qs), len(wl.problems), ",".join(map(str, sides)),
                             float(np.mean([r["setup_s"] for r in res])), iters, wall,
                             int(its.sum()), len(qs), cpu_s, len(os.sched_getaffinity(0)))}
    q = wl.problems[0]
    part = greedy_partition(rip_graph(q.A), q.K) if wl.partition == "greedy-rip" else q.part()
    r = _oracle_sample_worker((q, part, iters, omega, None))
    try:
        from threadpoolctl import threadpool_info
        blas = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # threadpoolctl missing: report the process's own view
        blas = 1
    return {"value": iters / (r["end"] - r["start"]), "unit": "outer iters/s", "cores": blas,
            "kind": "oracle",
            "sample": "%s: oracle projection setup (%.1f s, seminormal equations with SuperLU / "
                      "LAPACK per block) then its first %d %s iterations (%.1f s); BLAS on %d "
                      "threads (SuperLU itself is sequential); %d host cores visible"
                      % (q.name, r["setup_s"], iters, "outer CG" if omega is None else
                         "Algorithm 1", r["end"] - r["start"], blas,
                         len(os.sched_getaffinity(0)))}


def mixed_batched(wl, f_dev, reps=3):
    """The same batch solved with FP32 projections (FP64 outer CG): setup
    once, one untimed solve, then `reps` timed solves (median)."""
    import torch
    import paper_1710_07769_amd as bc
    opts = dict(wl.opts, precision=bc.BC_MIXED_PROJ)
    ctx = bc.bc_setup_batched([(q.n, q.A.rowptr, q.A.col, q.A.val, q.K, q.part())
                               for q in wl.problems], bc.make_opts(**opts))
    try:
        x = torch.empty_like(f_dev)
        times, its = [], []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = bc.bc_solve_batched(ctx, f_dev, None, wl.tol, 10000, x)
            torch.cuda.synchronize()
            if r > 0:
                times.append((time.perf_counter() - t0) * 1e3)
            its.append(int(max(st.iterations for st in sts)))
            print("[bench] FP32 projections, batched: %.1f ms, %d iterations (slowest system)"
                  % ((time.perf_counter() - t0) * 1e3, its[-1]), file=sys.stderr, flush=True)
        res = max(st.rel_residual for st in sts)
        proj_ms = sts[0].t_proj_ms
        launches = sts[0].proj_launches
        pbytes = sts[0].proj_bytes
    finally:
        bc.bc_destroy(ctx)
    return {"time_to_tol_ms": float(np.median(times)), "iterations_max": its[-1],
            "rel_residual": res,
            "projection_avg_launch_ms": proj_ms / max(launches, 1),
            "projection_bytes_per_launch": pbytes / max(launches, 1)}


def fp64_comparison(wl, f_dev, t_config_ms):
    """Plain FP64 GPU solves of the same systems and partitions: a batch is
    solved system by system (one context and one bc_solve each)."""
    import torch
    import paper_1710_07769_amd as bc
    opts = dict(wl.opts)
    opts["precision"] = bc.BC_FP64
    t_solve = 0.0
    iters = []
    off = 0
    for q in wl.problems:
        part = q.part() if wl.partition == "contiguous" else None
        if part is None:
            g = bc.rip_graph(q.n, q.A.rowptr, q.A.col, q.A.val)
            part = bc.bc_partition_greedy(g, q.K)
        ctx = bc.bc_setup(q.n, q.A.rowptr, q.A.col, q.A.val, q.K, part, bc.make_opts(**opts))
        try:
            fq = f_dev[off:off + q.n].contiguous()
            x = torch.empty_like(fq)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = bc.bc_solve(ctx, fq, None, wl.tol, 10000, x)
            torch.cuda.synchronize()
            t_solve += time.perf_counter() - t0
            iters.append(st.iterations)
        finally:
            bc.bc_destroy(ctx)
        off += q.n
        if len(iters) % 16 == 0:
            print("[bench] plain FP64: %d/%d systems, %.1f ms so far"
                  % (len(iters), len(wl.problems), t_solve * 1e3), file=sys.stderr, flush=True)
    print("[bench] plain FP64 per system: %.1f ms total" % (t_solve * 1e3), file=sys.stderr,
          flush=True)
    extra = {}
    if wl.batched:
        ctx = bc.bc_setup_batched([(q.n, q.A.rowptr, q.A.col, q.A.val, q.K, q.part())
                                   for q in wl.problems], bc.make_opts(**opts))
        try:
            x = torch.empty_like(f_dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = bc.bc_solve_batched(ctx, f_dev, None, wl.tol, 10000, x)
            torch.cuda.synchronize()
            extra["fp64_batched_time_to_tol_ms"] = (time.perf_counter() - t0) * 1e3
            extra["fp64_batched_iterations_max"] = int(max(st.iterations for st in sts))
        finally:
            bc.bc_destroy(ctx)
        print("[bench] FP64 batched: %.1f ms" % extra["fp64_batched_time_to_tol_ms"],
              file=sys.stderr, flush=True)
    return {**extra, "fp64_time_to_tol_ms": t_solve * 1e3,
            "speedup_vs_fp64": (t_solve * 1e3) / t_config_ms if t_config_ms > 0 else None,
            "fp64_iterations_total": int(sum(iters)),
            "fp64_iterations_max": int(max(iters)),
            "mode": "one bc_solve per system, one after another" if wl.batched else "bc_solve"}


def hbm_probe():
    """Bandwidth that plain device kernels reach on this GPU: torch's
    streaming sum (reads), device copy (read + write) and a += b (two reads,
    one write), 1 and 4 GiB per operand, median of 10 event-timed runs."""
    import json
    import torch
    p = torch.cuda.get_device_properties(0)
    out = {"device": p.name, "arch": getattr(p, "gcnArchName", ""),
           "compute_units": p.multi_processor_count,
           "memory_GiB": round(p.total_memory / 2**30, 1),
           "l2_MiB_per_xcd": getattr(p, "L2_cache_size", 0) / 2**20,
           "datasheet_hbm_GBs": HBM_PEAK_GBS, "rates_GBs": {}}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def med(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(10):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[5]

    for gib in (1, 4):
        n = (gib << 30) // 8
        a = torch.empty(n, dtype=torch.float64, device="cuda")
        b = torch.ones(n, dtype=torch.float64, device="cuda")
        nb = gib * 2**30
        r = out["rates_GBs"]
        r["sum_%dGiB" % gib] = round(nb / med(lambda: b.sum()) / 1e6)
        r["copy_%dGiB" % gib] = round(2 * nb / med(lambda: a.copy_(b)) / 1e6)
        r["add_%dGiB" % gib] = round(3 * nb / med(lambda: a.add_(b)) / 1e6)
        del a, b
    print(json.dumps(out))


def main():
    args = parse()
    if args.hbm_probe:
        hbm_probe()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1710_07769_amd as bc  # noqa: F401  (fails loudly if the library is missing)
    dev = torch.device("cuda:0")
    wl = Workload(args.workload, args.precision)
    f = torch.from_numpy(np.concatenate([q.f for q in wl.problems])).to(dev)
    print("[bench] workload %s: %s; n=%d nnz=%d" % (wl.name, wl.desc, wl.n, wl.nnz),
          file=sys.stderr, flush=True)
    if args.method == "alg1" and wl.batched:
        raise SystemExit("--method alg1 takes a single-system workload")
    xstar = np.concatenate([q.xstar for q in wl.problems])
    if args.method == "block" and args.nrhs is None:
        raise SystemExit("--method block needs --nrhs")
    if args.nrhs is not None:
        if wl.batched or args.method == "alg1" or args.nrhs < 1:
            raise SystemExit("--nrhs takes a single-system workload, --method cg or block and "
                             "nrhs >= 1")
        import workloads as W
        q = wl.problems[0]
        F, Xs = W.multi_rhs(q.A, args.nrhs, seed=1000)
        F[0], Xs[0] = q.f, q.xstar
        f = torch.from_numpy(np.ascontiguousarray(F)).to(dev)
        xstar = Xs.reshape(-1)
    for w in range(args.warmup):
        r = run_step(wl, f, args.method, args.partitioner, args.nrhs)
        print("[bench] warmup %d: iters=%d solve=%.1f ms" % (w, r["iterations"], r["solve_ms"]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    runs = []
    for k in range(args.steps):
        r = run_step(wl, f, args.method, args.partitioner, args.nrhs)
        runs.append(r)
        print("[bench] step %d: iters=%d solve=%.1f ms setup=%.1f ms rip=%.1f ms part=%.1f ms"
              % (k, r["iterations"], r["solve_ms"], r["setup_ms"], r["rip_ms"],
                 r["partition_ms"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    ms_per_step = (T1 - T0) * 1e3 / max(args.steps, 1)
    iters = sum(r["iterations"] for r in runs)
    solve_s = sum(r["solve_ms"] for r in runs) / 1e3
    value = iters / solve_s if solve_s > 0 else 0.0
    proj_ms = sum(r["t_proj_ms"] for r in runs)
    launches = sum(r["proj_launches"] for r in runs)
    pbytes = sum(r["proj_bytes"] for r in runs)
    achieved = pbytes / (proj_ms / 1e3) / 1e9 if proj_ms > 0 else 0.0
    xs = runs[-1]["x"].cpu().numpy().reshape(-1)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "outer iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if wl.mixed else "f64",
        "data": "synthetic",
        "config": {"workload": wl.desc + ("; Algorithm 1 (plain block Cimmino)"
                                          if args.method == "alg1" else "")
                   + ("; multilevel partitioner" if args.partitioner == "multilevel"
                      and wl.partition == "greedy-rip" else "")
                   + ("; %d right-hand sides solved together (%s)"
                      % (args.nrhs, "bc_solve_block, block CG" if args.method == "block"
                         else "bc_solve_multi")
                      if args.nrhs is not None else ""),
                   "n": wl.n, "nnz": wl.nnz,
                   "K": [q.K for q in wl.problems][0] if not wl.batched else 8,
                   "systems": len(wl.problems), "partition": wl.partition, "tol": wl.tol},
        "iterations": runs[-1]["iterations"],
        "max_iterations_per_system": runs[-1]["max_iterations"],
        "time_to_tol_ms": float(np.mean([r["solve_ms"] for r in runs])),
        "setup_ms": float(np.mean([r["setup_ms"] for r in runs])),
        "rip_graph_ms": float(np.mean([r["rip_ms"] for r in runs])),
        "rip_spgemm_ms": float(np.mean([r["rip_spgemm_ms"] for r in runs])),
        "partition_ms": float(np.mean([r["partition_ms"] for r in runs])),
        "rel_residual": max(r["rel_residual"] for r in runs),
        "rel_error_vs_xstar": float(np.linalg.norm(xs - xstar) / np.linalg.norm(xstar)),
        "inner_iterations_per_solve": runs[-1]["inner_iterations"],
        "block_kinds": runs[-1]["block_kinds"],
        "spmv_lanes_per_row": {"A": runs[-1]["lanes"][0], "AT": runs[-1]["lanes"][1]},
        "roofline": {"bound": "hbm", "kernel": "block projections (%s)" % ", ".join(
                         name for name, key in (("dense triangular sweeps", "dense"),
                                                ("inner CG", "inner_cg"),
                                                ("banded triangular sweeps", "banded"))
                         if runs[-1]["block_kinds"][key] > 0),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "avg_launch_ms": proj_ms / max(launches, 1),
                     "bytes_per_launch": pbytes / max(launches, 1),
                     "timing": "wall-clock stamp kernels on the library stream around each "
                               "projection launch (the solve replays captured graphs, inside "
                               "which events cannot be timed)",
                     "traffic": None},
    }
    traffic, tsrc = (measured_traffic(wl.name, wl.precision) if args.nrhs is None
                     and args.method == "cg" else (None, "not profiled"))
    line["roofline"]["traffic"] = traffic
    line["roofline"]["traffic_source"] = tsrc
    if "cutsize" in runs[-1]:
        line["partition_cutsize"] = runs[-1]["cutsize"]
    if args.nrhs is not None:
        line["nrhs"] = args.nrhs
        line["rhs_solves_per_s"] = args.nrhs / (line["time_to_tol_ms"] / 1e3)
    if args.method == "alg1":
        line["spectrum"] = runs[-1]["spectrum"]
        line["lanczos_ms"] = runs[-1]["lanczos_ms"]
    if args.spectrum:
        if wl.batched:
            raise SystemExit("--spectrum takes a single-system workload")
        line["spectrum_study"] = spectrum_study(wl, f)
    if args.compare:
        line["fp64_comparison"] = fp64_comparison(wl, f, line["time_to_tol_ms"])
    if wl.batched and not args.no_mixed and wl.precision == "fp64" and args.method == "cg":
        # the precision pattern on the same matrices, batched against batched
        mb = mixed_batched(wl, f)
        mb["speedup_vs_fp64_batched"] = line["time_to_tol_ms"] / mb["time_to_tol_ms"]
        mb["mode"] = ("bc_solve_batched with FP32 copies of the banded factors applied in FP64 "
                      "arithmetic (FP64 factorization, sparse products and outer CG)")
        line["mixed_batched"] = mb
    if not args.no_rip:
        line["rip_graph_st27_100cubed"] = rip_graph_bench()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(
            wl, args.cpu_iters, line["spectrum"]["omega"] if args.method == "alg1" else None,
            runs[-1]["sys_iters"] if wl.batched else None)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
