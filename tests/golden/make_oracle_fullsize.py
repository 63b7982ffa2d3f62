"""Writes tests/golden/oracle_fullsize.json: the FP64 oracle's results on the
full-size synthetic workloads, for the sampled full-size parity tests.

Only oracle/ and workloads/ are used (no GPU code).  For each workload the
oracle runs Algorithm 2 to a relative true residual of 1e-10 with the
workload's partition and records the iteration count, the final relative
residual, and the solution at 2000 seeded sample indices (the GPU side
compares its iterate at the same iteration count on those entries).

Run from the repository root:  python tests/golden/make_oracle_fullsize.py
(tens of minutes of single-threaded CPU; config 2, config 4's largest
systems and the greedy partition of config 5's 120M-edge graph dominate).
Arguments select entries (cfg2 cfg3 cfg4 cfg5 cfg5-rip, and cfg2-ml for the
hash of the oracle's multilevel partition of config 2's row inner-product
graph); the others in the file are kept.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import (block_cimmino_cg, rip_graph, greedy_partition,  # noqa: E402
                    multilevel_partition, BlockProjections)

NSAMPLE = 2000
TAIL = 32   # iterations of residual history kept before the stop
OUT = os.path.join(ROOT, "tests", "golden", "oracle_fullsize.json")


def run(name, A, f, part, K, tol=1e-10):
    t0 = time.time()
    M = A.to_scipy()
    B = BlockProjections(M, part, K)
    t1 = time.time()
    res = block_cimmino_cg(M, f, part, K, tol=tol, proj=B)
    t2 = time.time()
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(A.n, size=min(NSAMPLE, A.n), replace=False))
    print("%s: iterations %d rel_res %.3e setup %.1f s solve %.1f s"
          % (name, res.iterations, res.rel_residual, t1 - t0, t2 - t1), flush=True)
    # the relative true residuals of the last iterations (the checks of a
    # stop decided at a different iteration read them)
    t1_hist = max(0, res.iterations - TAIL + 1)
    hist = {str(t): float(res.history[t]) for t in range(t1_hist, res.iterations + 1)}
    return {"n": int(A.n), "K": int(K), "tol": tol, "iterations": int(res.iterations),
            "status": int(res.status), "rel_residual": float(res.rel_residual),
            "history_tail": hist,
            "sample_index": idx.tolist(), "sample_x": res.x[idx].tolist(),
            "x_norm2": float(np.linalg.norm(res.x)),
            "oracle_setup_s": t1 - t0, "oracle_solve_s": t2 - t1}


def part_hash(part):
    return int(np.sum(part.astype(np.int64) * np.arange(1, part.size + 1, dtype=np.int64))
               % (2**61 - 1))


def rip_graph_chunked(A, chunk=16384):
    """The oracle's row inner-product graph built in row chunks (the same
    steps as oracle.rip_rows over consecutive row ranges, the prescaled and
    sparsified matrix prepared once), for graphs too large to build whole."""
    from oracle import ripgraph as R
    n, rows, col, val = R._prepared(A, True, True)
    cptr, crow, cval = R._column_lists(n, rows, col, val)
    rp, cols, costs, wgts = [np.zeros(1, dtype=np.int64)], [], [], []
    lo = np.searchsorted(rows, np.arange(0, n + chunk, chunk))
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        a, b = lo[c0 // chunk], lo[c0 // chunk + 1] if c1 < n else rows.size
        i, j, k, prod = R._products(rows[a:b], col[a:b], val[a:b], cptr, crow, cval)
        g = R._assemble(c1 - c0, np.arange(c0, c1, dtype=np.int64), i, j, k, prod, 1 << 20)
        rp.append(g.rowptr[1:] + rp[-1][-1])
        cols.append(g.col)
        costs.append(g.cost)
        wgts.append(g.wgt)
    return R.RipGraph(n, np.concatenate(rp), np.concatenate(cols), np.concatenate(costs),
                      np.concatenate(wgts))


def main():
    which = sys.argv[1:] or ["cfg2", "cfg3", "cfg4", "cfg5", "cfg5-rip"]
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    if "cfg2" in which:
        p = workloads.config2()
        part = greedy_partition(rip_graph(p.A), p.K)
        out["cfg2"] = run("cfg2", p.A, p.f, part, p.K)
        out["cfg2"]["partition_sha"] = part_hash(part)
    if "cfg2-ml" in which:
        p = workloads.config2()
        part = multilevel_partition(rip_graph(p.A), p.K)
        out.setdefault("cfg2", {})["partition_ml_sha"] = int(
            np.sum(part.astype(np.int64) * np.arange(1, p.n + 1, dtype=np.int64)) % (2**61 - 1))
        print("cfg2 multilevel partition hash", out["cfg2"]["partition_ml_sha"], flush=True)
    if "cfg3" in which:
        p = workloads.config3()
        out["cfg3"] = run("cfg3", p.A, p.f, p.part(), p.K)
    if "cfg5" in which:
        p = workloads.config5()
        out["cfg5"] = run("cfg5", p.A, p.f, p.part(), p.K)
    if "cfg5-rip" in which:
        # the greedy partition of the 27-point 100^3 matrix's row inner-product
        # graph (120M edges) and the FP64 solve on it
        p = workloads.config5()
        t0 = time.time()
        g = rip_graph_chunked(p.A)
        t1 = time.time()
        part = greedy_partition(g, p.K)
        t2 = time.time()
        print("cfg5-rip: graph %d edges in %.0f s, greedy partition in %.0f s"
              % (g.col.size, t1 - t0, t2 - t1), flush=True)
        out["cfg5_rip"] = run("cfg5-rip", p.A, p.f, part, p.K)
        out["cfg5_rip"]["partition_sha"] = part_hash(part)
        out["cfg5_rip"]["edges"] = int(g.col.size)
    if "cfg4" in which:
        probs = workloads.config4()
        sides = [int(round(np.sqrt(q.n))) for q in probs]
        # the three smallest systems, one of side about 128, and the three
        # largest (the slowest to converge, which set the batch's time)
        order = np.argsort(sides, kind="stable")
        pick = [int(i) for i in order[:3]]
        mid = int(np.argmin([abs(s - 128) for s in sides]))
        for k in [mid] + [int(i) for i in order[-3:]]:
            if k not in pick:
                pick.append(k)
        out.setdefault("cfg4", {})
        for k in pick:
            q = probs[k]
            out["cfg4"][str(k)] = run("cfg4[%d] side %d" % (k, sides[k]), q.A, q.f, q.part(), q.K)
    json.dump(out, open(OUT, "w"))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
