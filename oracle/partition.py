"""K-way partitioning of G_RIP and partition quality (oracle; test infrastructure).

The paper partitions G_RIP with METIS (k-way, 10% imbalance, unit vertex
weights; Sections 2.3 and 3.1) to minimise the cutsize, which equals the sum
of inter-block row inner products interIP (Section 2.2).  METIS is a
third-party randomised tool; this project replaces it with a deterministic
greedy partitioner on the integer weights, specified here and implemented a
second time, independently, in the GPU library's host code:

1. Balance cap (eq. (partbal) with epsilon = 0.1 and unit weights):
   W_max = max(floor(1.1 n / K), ceil(n / K)).
2. Growth.  For k = 0 .. K-2, with R unassigned vertices left, part k is
   grown to exactly ceil(R / (K - k)) vertices.  It starts from the
   lowest-index unassigned vertex; each further vertex is the unassigned
   vertex with the largest total integer weight to the vertices already in
   part k (ties to the lower index); if no unassigned vertex touches part k,
   the lowest-index unassigned vertex is taken.  Part K-1 takes the rest.
3. Refinement.  Two passes over the vertices in ascending order.  Vertex v in
   part a (with more than one vertex) moves to the part q != a with the
   largest gain conn(v, q) - conn(v, a) > 0 among parts that v touches and
   that stay within W_max after the move (ties to the lower part id).
"""
from __future__ import annotations

import heapq
import itertools
import math

import numpy as np


def part_max_weight(n: int, K: int) -> int:
    return max(int(math.floor(1.1 * n / K)), -(-n // K))


def greedy_partition(g, K: int, passes: int = 2) -> np.ndarray:
    """Deterministic greedy K-way partition of a graph in CSR form
    (``n``, ``rowptr``, ``col``, integer ``wgt``); returns int32 part[n]."""
    n = g.n
    if not (1 <= K <= n):
        raise ValueError("need 1 <= K <= n")
    rowptr = np.asarray(g.rowptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    wgt = np.asarray(g.wgt, dtype=np.int64)
    part = np.full(n, -1, dtype=np.int64)
    conn = np.zeros(n, dtype=np.int64)
    lowest = 0
    remaining = n
    for k in range(K - 1):
        target = -(-remaining // (K - k))
        heap = []
        touched = []
        for _ in range(target):
            v = -1
            while heap:
                negc, u = heapq.heappop(heap)
                if part[u] == -1 and conn[u] == -negc:
                    v = u
                    break
            if v == -1:
                while part[lowest] != -1:
                    lowest += 1
                v = lowest
            part[v] = k
            remaining -= 1
            for e in range(rowptr[v], rowptr[v + 1]):
                u = col[e]
                if part[u] == -1:
                    if conn[u] == 0:
                        touched.append(u)
                    conn[u] += wgt[e]
                    heapq.heappush(heap, (-int(conn[u]), int(u)))
        for u in touched:
            conn[u] = 0
    part[part == -1] = K - 1

    wmax = part_max_weight(n, K)
    W = np.bincount(part, minlength=K).astype(np.int64)
    for _ in range(passes):
        for v in range(n):
            a = part[v]
            if W[a] <= 1:
                continue
            to = {}
            for e in range(rowptr[v], rowptr[v + 1]):
                q = int(part[col[e]])
                to[q] = to.get(q, 0) + int(wgt[e])
            inside = to.get(int(a), 0)
            best_q, best_gain = -1, 0
            for q in sorted(to):
                if q == a or W[q] + 1 > wmax:
                    continue
                gain = to[q] - inside
                if gain > best_gain:
                    best_q, best_gain = q, gain
            if best_q >= 0:
                part[v] = best_q
                W[a] -= 1
                W[best_q] += 1
    return part.astype(np.int32)


def _edges_upper(g):
    rowptr = np.asarray(g.rowptr, dtype=np.int64)
    i = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rowptr))
    j = np.asarray(g.col, dtype=np.int64)
    up = i < j
    return i[up], j[up], up


def cutsize(g, part) -> float:
    """Sum of the costs of the cut edges, each undirected edge once (eq. (partcut))."""
    i, j, up = _edges_upper(g)
    cut = part[i] != part[j]
    return float(np.sum(np.asarray(g.cost)[up][cut]))


def int_cut(g, part) -> int:
    """Sum of the integer weights of the cut edges, each undirected edge once."""
    i, j, up = _edges_upper(g)
    cut = part[i] != part[j]
    return int(np.sum(np.asarray(g.wgt, dtype=np.int64)[up][cut]))


def ip_matrix(g, part, K) -> np.ndarray:
    """ip_km = sum of |c_ij| over rows i in block k and j in block m, k != m
    (Section 2.2); the diagonal is left at zero."""
    rowptr = np.asarray(g.rowptr, dtype=np.int64)
    i = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rowptr))
    j = np.asarray(g.col, dtype=np.int64)
    IP = np.zeros((K, K))
    np.add.at(IP, (part[i], part[j]), np.asarray(g.cost))
    np.fill_diagonal(IP, 0.0)
    return IP


def imbalance(part, K) -> float:
    W = np.bincount(part, minlength=K)
    return float(W.max() / (len(part) / K) - 1.0)


def brute_force_min_cut(g, K: int) -> int:
    """Minimum integer cut over all K-way partitions with nonempty parts within
    the W_max cap (tiny graphs only)."""
    n = g.n
    wmax = part_max_weight(n, K)
    best = None
    for labels in itertools.product(range(K), repeat=n - 1):
        part = np.array((0,) + labels, dtype=np.int64)  # vertex 0 fixed in part 0 (symmetry)
        W = np.bincount(part, minlength=K)
        if W.min() == 0 or W.max() > wmax:
            continue
        c = int_cut(g, part)
        if best is None or c < best:
            best = c
    return best
