"""Writes tests/golden/oracle_fullsize.json: the FP64 oracle's results on the
full-size synthetic workloads, for the sampled full-size parity tests.

Only oracle/ and workloads/ are used (no GPU code).  For each workload the
oracle runs Algorithm 2 to a relative true residual of 1e-10 with the
workload's partition and records the iteration count, the final relative
residual, and the solution at 2000 seeded sample indices (the GPU side
compares its iterate at the same iteration count on those entries).

Run from the repository root:  python tests/golden/make_oracle_fullsize.py
(several minutes of single-threaded CPU; config 2 dominates).  With the
argument cfg2-ml it only adds the hash of the oracle's multilevel partition of
config 2's row inner-product graph (about 30 s).
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
    return {"n": int(A.n), "K": int(K), "tol": tol, "iterations": int(res.iterations),
            "status": int(res.status), "rel_residual": float(res.rel_residual),
            "sample_index": idx.tolist(), "sample_x": res.x[idx].tolist(),
            "x_norm2": float(np.linalg.norm(res.x)),
            "oracle_setup_s": t1 - t0, "oracle_solve_s": t2 - t1}


def main():
    which = sys.argv[1:] or ["cfg2", "cfg3", "cfg4", "cfg5"]
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    if "cfg2" in which:
        p = workloads.config2()
        part = greedy_partition(rip_graph(p.A), p.K)
        out["cfg2"] = run("cfg2", p.A, p.f, part, p.K)
        out["cfg2"]["partition_sha"] = int(np.sum(part.astype(np.int64) *
                                                  np.arange(1, p.n + 1, dtype=np.int64)) % (2**61 - 1))
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
    if "cfg4" in which:
        probs = workloads.config4()
        sides = [int(round(np.sqrt(q.n))) for q in probs]
        # the three smallest systems and one of side about 128 (oracle time grows fast)
        order = np.argsort(sides, kind="stable")
        pick = [int(i) for i in order[:3]]
        mid = int(np.argmin([abs(s - 128) for s in sides]))
        if mid not in pick:
            pick.append(mid)
        out["cfg4"] = {}
        for k in pick:
            q = probs[k]
            out["cfg4"][str(k)] = run("cfg4[%d] side %d" % (k, sides[k]), q.A, q.f, q.part(), q.K)
    json.dump(out, open(OUT, "w"))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
