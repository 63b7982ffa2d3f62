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


class _Graph:
    """A level of the multilevel scheme: CSR with integer edge and vertex weights."""

    def __init__(self, n, rowptr, col, wgt, vw):
        self.n, self.rowptr, self.col, self.wgt, self.vw = n, rowptr, col, wgt, vw


def _grow_weighted(G: _Graph, K: int) -> np.ndarray:
    """Growth of greedy_partition by vertex weight: part k grows until it
    weighs ceil(remaining weight / parts left), keeping one vertex for each
    later part; largest connection first (ties to the lower index), else the
    lowest-index unassigned vertex; part K-1 takes the rest."""
    n = G.n
    part = np.full(n, -1, dtype=np.int64)
    conn = np.zeros(n, dtype=np.int64)
    lowest = 0
    rem_w = int(G.vw.sum())
    rem_v = n
    for k in range(K - 1):
        target = -(-rem_w // (K - k))
        heap, touched, wk = [], [], 0
        while wk < target and rem_v > K - 1 - k:
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
            wk += int(G.vw[v])
            rem_v -= 1
            for e in range(G.rowptr[v], G.rowptr[v + 1]):
                u = int(G.col[e])
                if part[u] == -1:
                    if conn[u] == 0:
                        touched.append(u)
                    conn[u] += int(G.wgt[e])
                    heapq.heappush(heap, (-int(conn[u]), u))
        rem_w -= wk
        for u in touched:
            conn[u] = 0
    part[part == -1] = K - 1
    return part


FM_STALL = 64


def _fm_conn(G: _Graph, part, v):
    """conn(v, q): total edge weight from v to part q, for the parts v touches."""
    to = {}
    for e in range(G.rowptr[v], G.rowptr[v + 1]):
        q = int(part[G.col[e]])
        to[q] = to.get(q, 0) + int(G.wgt[e])
    return to


def _fm_key(to, a):
    """The largest conn(v, q) - conn(v, a) over touched parts q != a, the
    part of v (None when v touches no other part)."""
    inside = to.get(a, 0)
    gains = [to[q] - inside for q in to if q != a]
    return max(gains) if gains else None


def _refine_fm(G: _Graph, K: int, wmax: int, passes: int, part: np.ndarray,
               stall_limit: int = FM_STALL, trace=None) -> None:
    """Fiduccia-Mattheyses refinement with vertex weights (in place).

    Each pass: every vertex unlocked; a max-priority queue of (key, vertex)
    (larger key first, ties to the lower vertex) over the vertices that touch
    another part.  A popped entry is skipped when its vertex is locked or its
    key is no longer current.  Otherwise the vertex moves to the touched part
    q != a of largest gain conn(v,q) - conn(v,a) (ties to the lower q) among
    those that stay within W_max, provided part a keeps some weight; with no
    such part the entry is dropped and the vertex stays unlocked.  A move may
    have a negative gain.  The mover is locked, the move logged with the
    running sum of gains, and every unlocked neighbour (adjacency order) is
    pushed again with its new key.  The pass ends when the queue is empty or
    FM_STALL moves in a row have not raised the best running sum; the moves
    after the best prefix (the shortest one on ties) are undone in reverse
    order.  Passes stop early after one whose best running sum is 0.
    ``trace``, if a list, receives (pass, vertex, from, to, gain) for every
    move made, undone or not."""
    W = np.zeros(K, dtype=np.int64)
    np.add.at(W, part, G.vw)
    for pass_no in range(passes):
        locked = np.zeros(G.n, dtype=bool)
        conn = [_fm_conn(G, part, v) for v in range(G.n)]
        heap = []
        for v in range(G.n):
            key = _fm_key(conn[v], int(part[v]))
            if key is not None:
                heap.append((-key, v))
        heapq.heapify(heap)
        log = []
        cum = best = 0
        best_len = 0
        stall = 0
        while heap and stall < stall_limit:
            negk, v = heapq.heappop(heap)
            if locked[v]:
                continue
            a = int(part[v])
            to = conn[v]
            key = _fm_key(to, a)
            if key is None or key != -negk:
                continue
            if W[a] <= G.vw[v]:
                continue
            inside = to.get(a, 0)
            q_best, g_best = -1, None
            for q in sorted(to):
                if q == a or W[q] + G.vw[v] > wmax:
                    continue
                gain = to[q] - inside
                if g_best is None or gain > g_best:
                    q_best, g_best = q, gain
            if q_best < 0:
                continue
            part[v] = q_best
            W[a] -= G.vw[v]
            W[q_best] += G.vw[v]
            locked[v] = True
            log.append((v, a))
            if trace is not None:
                trace.append((pass_no, v, a, q_best, g_best))
            cum += g_best
            if cum > best:
                best, best_len, stall = cum, len(log), 0
            else:
                stall += 1
            # the neighbours' connections follow the move; then each
            # unlocked neighbour is queued with its new key
            nbrs = range(G.rowptr[v], G.rowptr[v + 1])
            for e in nbrs:
                cu, w = conn[int(G.col[e])], int(G.wgt[e])
                cu[a] -= w
                if cu[a] == 0:
                    del cu[a]
                cu[q_best] = cu.get(q_best, 0) + w
            for e in nbrs:
                u = int(G.col[e])
                if not locked[u]:
                    ku = _fm_key(conn[u], int(part[u]))
                    if ku is not None:
                        heapq.heappush(heap, (-ku, u))
        for v, a in reversed(log[best_len:]):
            q = int(part[v])
            part[v] = a
            W[q] -= G.vw[v]
            W[a] += G.vw[v]
        if best == 0:
            break


def _coarsen(G: _Graph, maxvw: int):
    """Heavy-edge matching in ascending vertex order (heaviest edge to an
    unmatched neighbour within the vertex-weight cap, ties to the lower
    index), then contraction: coarse vertices in ascending order of their
    lower fine vertex, parallel edges summed, internal edges dropped.
    Returns the coarse graph and the fine-to-coarse map."""
    n = G.n
    match = [-1] * n
    for v in range(n):
        if match[v] != -1:
            continue
        best, bw = -1, 0
        for e in range(G.rowptr[v], G.rowptr[v + 1]):
            u = int(G.col[e])
            if match[u] != -1 or G.vw[v] + G.vw[u] > maxvw:
                continue
            w = int(G.wgt[e])
            if w > bw or (w == bw and best >= 0 and u < best):
                best, bw = u, w
        if best >= 0:
            match[v], match[best] = best, v
        else:
            match[v] = v
    cmap = [-1] * n
    first = []
    for v in range(n):
        if cmap[v] == -1:
            cmap[v] = cmap[match[v]] = len(first)
            first.append(v)
    nc = len(first)
    vw = np.zeros(nc, dtype=np.int64)
    rowptr, col, wgt = [0], [], []
    for c, a in enumerate(first):
        members = [a] if match[a] == a else [a, match[a]]
        vw[c] = sum(int(G.vw[x]) for x in members)
        acc = {}
        for x in members:
            for e in range(G.rowptr[x], G.rowptr[x + 1]):
                d = cmap[int(G.col[e])]
                if d != c:
                    acc[d] = acc.get(d, 0) + int(G.wgt[e])
        for d in sorted(acc):
            col.append(d)
            wgt.append(acc[d])
        rowptr.append(len(col))
    C = _Graph(nc, np.array(rowptr, dtype=np.int64), np.array(col, dtype=np.int64),
               np.array(wgt, dtype=np.int64), vw)
    return C, np.array(cmap, dtype=np.int64)


def multilevel_partition(g, K: int, passes: int = 2) -> np.ndarray:
    """Deterministic multilevel K-way partition (heavy-edge coarsening while
    the graph has more than 30 K vertices, weighted greedy growth on the
    coarsest graph, at most ``passes`` FM passes at every level on the way
    back, see _refine_fm);
    returns int32 part[n].  The same specification as the library's host
    implementation, written independently."""
    n = g.n
    if not (1 <= K <= n):
        raise ValueError("need 1 <= K <= n")
    wmax = part_max_weight(n, K)
    coarse_to = max(30 * K, K)
    maxvw = max(1, -(-n // (20 * K)))
    levels = [_Graph(n, np.asarray(g.rowptr, dtype=np.int64), np.asarray(g.col, dtype=np.int64),
                     np.asarray(g.wgt, dtype=np.int64), np.ones(n, dtype=np.int64))]
    maps = []
    while levels[-1].n > coarse_to and len(levels) < 30:
        C, cmap = _coarsen(levels[-1], maxvw)
        if C.n > 0.9 * levels[-1].n:
            break
        levels.append(C)
        maps.append(cmap)
    part = _grow_weighted(levels[-1], K)
    _refine_fm(levels[-1], K, wmax, passes, part)
    for lvl in range(len(levels) - 2, -1, -1):
        part = part[maps[lvl]]
        _refine_fm(levels[lvl], K, wmax, passes, part)
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
