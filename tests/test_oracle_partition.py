"""Pins of the oracle's partitioner and partition-quality measures.

P9:  cutsize(Pi) = sum_{k<m} ip_km = half the sum of |c_ij| over off-block
     entries (Section 2.2), and the paper's interIP arithmetic.
P10: on tiny graphs the greedy cut is never below the brute-force optimum.
Closed forms: K equal disjoint cliques are separated with zero cut; on a
path the parts are contiguous segments.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from workloads import Csr
from oracle import (rip_graph, greedy_partition, cutsize, int_cut, ip_matrix, imbalance,
                    brute_force_min_cut, part_max_weight)
from oracle.ripgraph import RipGraph


def graph_from_dense(W):
    W = np.asarray(W, dtype=np.int64)
    n = W.shape[0]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, wg = [], []
    for i in range(n):
        nz = np.flatnonzero(W[i])
        nz = nz[nz != i]
        cols.extend(nz.tolist())
        wg.extend(W[i, nz].tolist())
        rowptr[i + 1] = len(cols)
    wg = np.array(wg, dtype=np.int64)
    return RipGraph(n, rowptr, np.array(cols, dtype=np.int32), wg.astype(np.float64), wg)


def test_interip_arithmetic(golden):
    gv = golden["interIP_sample"]
    assert sum(gv["straightforward_ip"]) == gv["straightforward_total"]
    assert sum(gv["good_ip"]) == gv["good_total"]


@pytest.mark.parametrize("seed", [0, 1])
def test_cutsize_equals_interip(seed):
    rng = np.random.default_rng(seed)
    n, K = 50, 4
    M = sp.random(n, n, density=0.08, random_state=rng,
                  data_rvs=lambda k: rng.integers(1, 6, k).astype(float)).tocsr() + sp.eye(n)
    A = Csr.from_scipy(M)
    g = rip_graph(A, prescale=False, sparsify=False)
    part = rng.integers(0, K, n)
    IP = ip_matrix(g, part, K)
    assert np.allclose(IP, IP.T)
    upper = sum(IP[k, m] for k in range(K) for m in range(k + 1, K))
    D = A.to_scipy().toarray()
    C = np.abs(D @ D.T)
    off = part[:, None] != part[None, :]
    assert cutsize(g, part) == pytest.approx(upper, rel=1e-14)
    assert cutsize(g, part) == pytest.approx(0.5 * C[off].sum(), rel=1e-14)
    assert int_cut(g, part) == int(round(0.5 * C[off].sum())) * 2 ** 20


@pytest.mark.parametrize("seed,n,K", [(0, 8, 2), (1, 9, 3), (2, 10, 2), (3, 9, 3)])
def test_greedy_not_below_brute_force(seed, n, K):
    rng = np.random.default_rng(seed)
    W = np.triu(rng.integers(0, 4, (n, n)) * (rng.random((n, n)) < 0.5), 1)
    W = W + W.T
    g = graph_from_dense(W)
    part = greedy_partition(g, K)
    assert set(part.tolist()) == set(range(K))
    assert np.bincount(part, minlength=K).max() <= part_max_weight(n, K)
    best = brute_force_min_cut(g, K)
    assert int_cut(g, part) >= best


def test_disjoint_cliques_zero_cut():
    K, s = 4, 5
    W = np.zeros((K * s, K * s), dtype=np.int64)
    rng = np.random.default_rng(5)
    perm = rng.permutation(K * s)
    for k in range(K):
        idx = perm[k * s:(k + 1) * s]
        W[np.ix_(idx, idx)] = 3
    np.fill_diagonal(W, 0)
    g = graph_from_dense(W)
    part = greedy_partition(g, K)
    assert int_cut(g, part) == 0
    assert np.all(np.bincount(part) == s)


def test_path_gives_contiguous_segments():
    n, K = 20, 4
    W = np.zeros((n, n), dtype=np.int64)
    for i in range(n - 1):
        W[i, i + 1] = W[i + 1, i] = 1
    part = greedy_partition(graph_from_dense(W), K)
    assert np.array_equal(part, np.repeat(np.arange(K), 5))


def test_greedy_on_stencil_graph_is_balanced_and_beats_contiguous():
    p = workloads.small_config2(N=10, K=4)
    g = rip_graph(p.A)
    part = greedy_partition(g, p.K)
    assert imbalance(part, p.K) <= 0.1 + 1e-12
    assert set(part.tolist()) == set(range(p.K))
    contiguous = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, p.K))
    assert cutsize(g, part) <= cutsize(g, contiguous) * 1.05
    assert np.array_equal(part, greedy_partition(g, p.K))  # deterministic


def _path(n):
    W = np.zeros((n, n), dtype=np.int64)
    for i in range(n - 1):
        W[i, i + 1] = W[i + 1, i] = 1
    return graph_from_dense(W)


def test_hand_computed_partitions():
    # path of 10, K = 4: growth sizes ceil(10/4)=3, ceil(7/3)=3, ceil(4/2)=2, rest 2;
    # every boundary move has gain 0, so refinement keeps the segments
    assert greedy_partition(_path(10), 4).tolist() == [0, 0, 0, 1, 1, 1, 2, 2, 3, 3]
    # path of 9, K = 2: vertex 4 has gain 0 towards part 1 (which has room): no move
    assert greedy_partition(_path(9), 2).tolist() == [0] * 5 + [1] * 4
    # 3x3 grid graph, unit weights, K = 3: ties go to the lowest index, so parts are rows
    W = np.zeros((9, 9), dtype=np.int64)
    for r in range(3):
        for c in range(3):
            v = 3 * r + c
            if c < 2:
                W[v, v + 1] = W[v + 1, v] = 1
            if r < 2:
                W[v, v + 3] = W[v + 3, v] = 1
    assert greedy_partition(graph_from_dense(W), 3).tolist() == [0, 0, 0, 1, 1, 1, 2, 2, 2]


def test_refinement_moves_positive_gain():
    """Hand-traced: growth (K = 3, caps ceil(10/3) = 4, then 3, rest 3) gives
    part 0 = {0, 9, 1, 4} (9 has weight 4 to 0; 1 then has 8; 4 and 6 tie at 6
    and 4 wins), part 1 = {2, 3, 8} (2 touches nothing unassigned, 3 is the
    lowest unassigned, then 8), part 2 = {5, 6, 7}.  Refinement (W_max = 4):
    vertex 2 would gain 3 towards part 0 but part 0 is full; vertex 5 gains 5
    towards part 1 and moves; vertex 6 would gain 5 towards part 0 (full)."""
    W = np.array([[0, 3, 0, 1, 1, 0, 0, 0, 1, 4],
                  [3, 0, 3, 0, 5, 0, 3, 0, 0, 5],
                  [0, 3, 0, 0, 0, 0, 0, 0, 0, 0],
                  [1, 0, 0, 0, 0, 0, 0, 0, 2, 0],
                  [1, 5, 0, 0, 0, 0, 3, 0, 0, 0],
                  [0, 0, 0, 0, 0, 0, 0, 0, 5, 0],
                  [0, 3, 0, 0, 3, 0, 0, 4, 0, 3],
                  [0, 0, 0, 0, 0, 0, 4, 0, 3, 2],
                  [1, 0, 0, 2, 0, 5, 0, 3, 0, 0],
                  [4, 5, 0, 0, 0, 0, 3, 2, 0, 0]])
    g = graph_from_dense(W)
    assert greedy_partition(g, 3, passes=0).tolist() == [0, 0, 1, 1, 0, 2, 2, 2, 1, 0]
    assert greedy_partition(g, 3).tolist() == [0, 0, 1, 1, 0, 1, 2, 2, 1, 0]


# ------------------------------------------------------------- multilevel

from oracle import multilevel_partition  # noqa: E402
from oracle.partition import _coarsen, _Graph, _refine_fm  # noqa: E402


@pytest.mark.parametrize("seed,n,K", [(0, 8, 2), (1, 9, 3), (3, 12, 3)])
def test_multilevel_small_graph_is_greedy_and_not_below_brute_force(seed, n, K):
    # n <= 30 K: no coarsening; the weighted growth with unit weights is the
    # greedy growth, and W_max = n / K leaves no room for a move, so neither
    # refinement moves a vertex and the two partitioners coincide
    rng = np.random.default_rng(seed)
    W = np.triu(rng.integers(0, 4, (n, n)) * (rng.random((n, n)) < 0.5), 1)
    g = graph_from_dense(W + W.T)
    part = multilevel_partition(g, K)
    assert np.array_equal(part, greedy_partition(g, K))
    assert int_cut(g, part) >= brute_force_min_cut(g, K)


def test_multilevel_separates_disjoint_cliques_through_coarsening():
    K, s = 3, 60   # n = 180 > 30 K: two or more coarsening levels
    W = np.zeros((K * s, K * s), dtype=np.int64)
    perm = np.random.default_rng(9).permutation(K * s)
    for k in range(K):
        idx = perm[k * s:(k + 1) * s]
        W[np.ix_(idx, idx)] = 2
    np.fill_diagonal(W, 0)
    g = graph_from_dense(W)
    part = multilevel_partition(g, K)
    assert int_cut(g, part) == 0
    assert np.all(np.bincount(part, minlength=K) == s)


def test_multilevel_on_a_path_gives_contiguous_segments():
    n, K = 200, 4
    W = np.zeros((n, n), dtype=np.int64)
    for i in range(n - 1):
        W[i, i + 1] = W[i + 1, i] = 1
    g = graph_from_dense(W)
    part = multilevel_partition(g, K)
    assert np.all(np.diff(part) >= 0) and set(part.tolist()) == set(range(K))
    assert np.bincount(part).max() <= part_max_weight(n, K)
    assert int_cut(g, part) == K - 1


def test_coarsening_invariants():
    p = workloads.small_config2(N=10, K=4)
    g = rip_graph(p.A)
    G = _Graph(g.n, np.asarray(g.rowptr, dtype=np.int64), np.asarray(g.col, dtype=np.int64),
               np.asarray(g.wgt, dtype=np.int64), np.ones(g.n, dtype=np.int64))
    C, cmap = _coarsen(G, maxvw=3)
    assert C.vw.sum() == g.n and C.vw.max() <= 3 and C.n < g.n
    # edge weight is conserved except on the contracted (internal) edges
    i = np.repeat(np.arange(g.n), np.diff(G.rowptr))
    internal = cmap[i] == cmap[G.col]
    assert C.wgt.sum() == G.wgt.sum() - G.wgt[internal].sum()
    # the coarse graph is symmetric with positive weights and no loops
    M = sp.csr_matrix((C.wgt, C.col, C.rowptr), shape=(C.n, C.n))
    assert (M != M.T).nnz == 0 and M.diagonal().sum() == 0 and C.wgt.min() >= 1


def test_multilevel_on_stencil_graph_is_balanced():
    p = workloads.small_config2(N=12, K=6)
    g = rip_graph(p.A)
    part = multilevel_partition(g, p.K)
    assert set(part.tolist()) == set(range(p.K))
    assert np.bincount(part, minlength=p.K).max() <= part_max_weight(p.n, p.K)
    contiguous = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, p.K))
    print("cut greedy %.3f multilevel %.3f contiguous %.3f"
          % (cutsize(g, greedy_partition(g, p.K)), cutsize(g, part), cutsize(g, contiguous)))
    assert cutsize(g, part) <= cutsize(g, contiguous)


def _weighted_graph(n, edges, vw=None, order=None):
    """_Graph from undirected (i, j, w) edges; ``order`` may give a vertex's
    adjacency in a chosen order (default ascending)."""
    adj = {v: {} for v in range(n)}
    for i, j, w in edges:
        adj[i][j] = w
        adj[j][i] = w
    rowptr, col, wgt = [0], [], []
    for v in range(n):
        nb = (order or {}).get(v, sorted(adj[v]))
        assert sorted(nb) == sorted(adj[v])
        col += nb
        wgt += [adj[v][u] for u in nb]
        rowptr.append(len(col))
    vw = np.ones(n, dtype=np.int64) if vw is None else np.asarray(vw, dtype=np.int64)
    return _Graph(n, np.array(rowptr, dtype=np.int64), np.array(col, dtype=np.int64),
                  np.array(wgt, dtype=np.int64), vw)


def test_coarsen_hand_traced():
    # Vertex 0 lists neighbour 2 before 1 and both edges weigh 5: the tie
    # goes to the lower index, 0-1.  Vertex 2 then takes 3 (0 and 1 are
    # matched).  Vertex 4 cannot take 5 (weights 2 + 2 > 3), and takes 7
    # (edge 4) over 8 (edge 1).  Vertex 5 takes 6; vertex 8 finds only a
    # matched neighbour and stays single.  Coarse vertices in order of their
    # lower fine vertex: {0,1} {2,3} {4,7} {5,6} {8}.  Coarse edges:
    # c0-c1 = 5 (0-2) + 2 (1-2) + 1 (1-3) = 8; c1-c2 = 4 (3-4);
    # c2-c3 = 4 (4-5) + 2 (7-6) = 6; c2-c4 = 1 (4-8); 0-1, 2-3, 4-7 and 5-6
    # are internal and dropped.
    edges = [(0, 1, 5), (0, 2, 5), (1, 2, 2), (1, 3, 1), (2, 3, 3), (3, 4, 4), (4, 5, 4),
             (4, 7, 4), (5, 6, 1), (6, 7, 2), (4, 8, 1)]
    G = _weighted_graph(9, edges, vw=[1, 1, 1, 1, 2, 2, 1, 1, 1], order={0: [2, 1]})
    C, cmap = _coarsen(G, maxvw=3)
    assert cmap.tolist() == [0, 0, 1, 1, 2, 3, 3, 2, 4]
    assert C.n == 5
    assert C.vw.tolist() == [2, 2, 3, 3, 1]
    assert C.rowptr.tolist() == [0, 1, 3, 6, 7, 8]
    assert C.col.tolist() == [1, 0, 2, 1, 3, 4, 2, 2]
    assert C.wgt.tolist() == [8, 8, 4, 4, 6, 1, 6, 1]


# Two groups: {0,1,2} tightly bound, 3 and 4 tied to each other (3) and to
# the group by 1 each, and each tied by 2 to one of 5, 6 of the group
# {5..9}.  From parts {0..4} | {5..9} no single move has a positive gain.
_FM_EDGES = [(0, 1, 5), (0, 2, 5), (1, 2, 5), (0, 3, 1), (1, 4, 1), (3, 4, 3),
             (5, 6, 5), (5, 7, 5), (6, 7, 5), (7, 8, 5), (8, 9, 5), (5, 9, 5),
             (3, 5, 2), (4, 6, 2)]


def test_fm_climbs_through_a_negative_move_and_rolls_back_hand_traced():
    # Pass 1: keys 3: 2-4 = -2, 4: -2, 5: 2-15 = -13, 6: 2-10 = -8.  Vertex
    # 3 moves first (gain -2, running sum -2); 4's key becomes 5-1 = +4 and
    # it moves (running sum +2, the best).  0 and 1 (keys -9) would bring
    # part 1 to 8 > W_max = 7 and are dropped.  Cut 4 -> 2, parts 3 | 7.
    # Pass 2: 3 moves back (-4), 4 follows (+2), 6 (-8), 5 (-3): running
    # sums -4, -2, -10, -13, never above 0; 7 and 9 would overfill part 0.
    # All four moves are undone and refinement stops.
    G = _weighted_graph(10, _FM_EDGES)
    part = np.array([0] * 5 + [1] * 5, dtype=np.int64)
    _refine_fm(G, 2, 7, 1, part)
    assert part.tolist() == [0, 0, 0, 1, 1, 1, 1, 1, 1, 1]
    part2 = np.array([0] * 5 + [1] * 5, dtype=np.int64)
    _refine_fm(G, 2, 7, 5, part2)
    assert part2.tolist() == part.tolist()
    # the positive-gain sweeps of greedy_partition would make no move here
    g = graph_from_dense(_dense(G))
    assert int_cut(g, np.array([0] * 5 + [1] * 5)) == 4 and int_cut(g, part) == 2


def test_fm_undoes_a_pass_without_gain():
    # from the pass-1 result, a single pass tries 3, 4, 6, 5 and undoes them
    G = _weighted_graph(10, _FM_EDGES)
    start = [0, 0, 0, 1, 1, 1, 1, 1, 1, 1]
    part = np.array(start, dtype=np.int64)
    _refine_fm(G, 2, 7, 1, part)
    assert part.tolist() == start


def test_fm_three_parts_tie_and_undo_after_the_best_prefix_hand_traced():
    # Parts {0,1,2} {3,4,5} {6,7,8}, W_max = 4.  Pass 1: vertex 0 gains 1
    # towards part 1 and towards part 2; the tie goes to part 1 (best sum 1
    # after one move).  6, 1 and 2 would overfill part 1 and are dropped; 5
    # moves to part 0 (-4), then 4 (0); 3 would overfill part 0.  The two
    # moves after the best prefix are undone: cut 5 -> 4.  Pass 2: 0 moves
    # on to part 2 (gain 0 beats -1 towards part 0), 2 moves to part 1 (-4);
    # 1 may not empty part 0.  No gain: both are undone.
    edges = [(1, 2, 5), (0, 1, 1), (3, 4, 5), (4, 5, 5), (0, 3, 2), (6, 7, 5), (7, 8, 5),
             (0, 6, 2), (2, 5, 1)]
    G = _weighted_graph(9, edges)
    want = [1, 0, 0, 1, 1, 1, 2, 2, 2]
    for passes in (1, 2, 3):
        part = np.array([0, 0, 0, 1, 1, 1, 2, 2, 2], dtype=np.int64)
        _refine_fm(G, 3, 4, passes, part)
        assert part.tolist() == want, passes
    g = graph_from_dense(_dense(G))
    assert int_cut(g, np.array([0, 0, 0, 1, 1, 1, 2, 2, 2])) == 5
    assert int_cut(g, np.array(want)) == 4


def test_fm_move_order_guards_and_stall_hand_traced():
    # Parts {0,1} | {2..5}, W_max = 10.  Keys: 0: 4-1 = 3, 2: 5-2 = 3,
    # 1: 3-1 = 2, 4: 2-5 = -3.  Pass 1: 0 moves (+3; tie with 2 to the lower
    # vertex).  1's key rises to 4 but moving it would empty part 0; the
    # entries (3, 2) and (2, 1) are stale (keys now -5 and 4).  4 moves (-3),
    # which raises 5 to +5 (moves, best sum 5 after three moves) and 1 to 0
    # (moves, running sum 5, not above the best, undone).  Pass 2: 1 (0) and
    # 4 (-3) move, 5 may not empty part 0, and both moves are undone.
    edges = [(0, 1, 1), (0, 2, 4), (1, 2, 1), (2, 3, 2), (1, 4, 2), (4, 5, 5)]
    G = _weighted_graph(6, edges)
    part = np.array([0, 0, 1, 1, 1, 1], dtype=np.int64)
    trace = []
    _refine_fm(G, 2, 10, 4, part, trace=trace)
    assert trace == [(0, 0, 0, 1, 3), (0, 4, 1, 0, -3), (0, 5, 1, 0, 5), (0, 1, 0, 1, 0),
                     (1, 1, 0, 1, 0), (1, 4, 0, 1, -3)]
    assert part.tolist() == [1, 0, 1, 1, 0, 0]
    # with a stall limit of one move, pass 1 stops after 4's move (-3) and
    # undoes it; pass 2 moves 0 back (-3, 1 may not empty part 0), undoes it
    # and stops
    part = np.array([0, 0, 1, 1, 1, 1], dtype=np.int64)
    trace = []
    _refine_fm(G, 2, 10, 4, part, stall_limit=1, trace=trace)
    assert trace == [(0, 0, 0, 1, 3), (0, 4, 1, 0, -3), (1, 0, 1, 0, -3)]
    assert part.tolist() == [1, 0, 1, 1, 1, 1]


def _dense(G):
    W = np.zeros((G.n, G.n), dtype=np.int64)
    for v in range(G.n):
        for e in range(G.rowptr[v], G.rowptr[v + 1]):
            W[v, G.col[e]] = G.wgt[e]
    return W


def test_multilevel_hand_traced_on_a_64_vertex_path():
    # n = 64 > 30 K = 60 with K = 2: one coarsening level.  The matching
    # pairs (2i, 2i+1) (cap ceil(64/40) = 2), giving a 32-vertex path of
    # weight-2 vertices.  Growth gives part 0 the coarse vertices 0..15.
    # FM (W_max = floor(1.1*64/2) = 35): coarse 15 moves across (gain 0),
    # coarse 14 would bring part 1 to 36 and is dropped, the pass gains
    # nothing and is undone.  Projected down, fine vertices 31, 30, 29 move
    # (gain 0 each), 28 would bring part 1 to 36, and the pass is undone:
    # the halves 0..31 | 32..63.
    n = 64
    g = graph_from_dense(np.eye(n, k=1, dtype=np.int64) + np.eye(n, k=-1, dtype=np.int64))
    G = _Graph(n, np.asarray(g.rowptr, dtype=np.int64), np.asarray(g.col, dtype=np.int64),
               np.asarray(g.wgt, dtype=np.int64), np.ones(n, dtype=np.int64))
    C, cmap = _coarsen(G, maxvw=2)
    assert cmap.tolist() == [v // 2 for v in range(n)]
    assert C.n == 32 and C.vw.tolist() == [2] * 32 and C.wgt.tolist() == [1] * 62
    assert multilevel_partition(g, 2).tolist() == [0] * 32 + [1] * 32
