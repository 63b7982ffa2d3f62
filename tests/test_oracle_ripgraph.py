"""Pins of the oracle's row inner-product graph (Sections 2.1 and 2.3).

P7:  the printed worked value r_2 r_4^T = 9*12 + 6*18 = 216 (Section 2.1).
P8:  the 25x25 dense-column example: nnz(A A^T) = 531 (Section 2.3); keeping
     the isqrt(25) = 5 largest entries of the dense column leaves
     5^2 + 20 = 45 nonzeros (derived from the same construction).
P11: on integer-valued matrices (exact products and sums) the graph equals the
     off-diagonal nonzeros of the dense product A @ A.T, bit for bit.
Also: prescaled costs are cosines of row angles; the summation order is
ascending column index; weights are ceil(2^20 * cost); the graph is symmetric.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import Csr
import workloads
from oracle import rip_graph, rip_rows, row_norms, sparsify_columns


def csr(M):
    return Csr.from_scipy(sp.csr_matrix(np.asarray(M, dtype=np.float64)))


def as_dense(g):
    D = np.zeros((g.n, g.n))
    for i in range(g.n):
        for e in range(g.rowptr[i], g.rowptr[i + 1]):
            D[i, g.col[e]] = g.cost[e]
    return D


def test_worked_value_216(golden):
    gv = golden["row_inner_product_r2_r4"]
    a, b = gv["row2_shared_values"], gv["row4_shared_values"]
    # rows share two columns (1 and 3); other entries in disjoint columns
    M = np.zeros((2, 6))
    M[0, [0, 1, 3]] = [5.0, a[0], a[1]]
    M[1, [1, 3, 5]] = [b[0], b[1], 7.0]
    g = rip_graph(_two_rows(M), prescale=False, sparsify=False)
    assert g.cost[0] == gv["product"] == 216.0
    assert g.wgt[0] == 216 * 2 ** 20


def _two_rows(M):
    # pad to a square CSR (the extra rows are empty and produce no edges)
    n = M.shape[1]
    full = np.zeros((n, n))
    full[:2] = M
    return csr(full)


def test_dense_column_example(golden):
    gv = golden["dense_column_example"]
    n, nz = gv["n"], gv["dense_column_nnz"]
    rng = np.random.default_rng(0)
    c = 3
    A = np.eye(n)
    rows = np.sort(np.concatenate([[c], rng.choice(np.delete(np.arange(n), c), nz - 1, replace=False)]))
    A[rows, c] = rng.uniform(0.1, 0.9, nz) * rng.choice([-1, 1], nz)
    A[c, c] = 5.0
    M = csr(A)
    assert M.nnz == n + nz - 1
    g = rip_graph(M, prescale=True, sparsify=False)
    assert g.col.size + n == gv["nnz_AAT"]
    # the dense-column rule: isqrt(25) = 5 < 23 kept entries
    assert math.isqrt(n) == gv["kept_after_sparsify"]
    gs = rip_graph(M, prescale=True, sparsify=True)
    k = gv["kept_after_sparsify"]
    assert gs.col.size + n == k * k + (n - k)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_integer_matrix_matches_dense_product(seed):
    rng = np.random.default_rng(seed)
    n = 60
    M = sp.random(n, n, density=0.06, random_state=rng,
                  data_rvs=lambda k: rng.integers(-9, 10, k).astype(float)).tocsr()
    M.eliminate_zeros()
    M = M + sp.eye(n)
    A = csr(M.toarray())
    g = rip_graph(A, prescale=False, sparsify=False)
    D = A.to_scipy().toarray()
    C = D @ D.T
    np.fill_diagonal(C, 0.0)
    G = as_dense(g)
    assert np.array_equal(G, np.abs(C))
    assert g.col.size == np.count_nonzero(C)
    assert np.array_equal(g.wgt, np.ceil(g.cost * 2 ** 20).astype(np.int64))


def test_prescaled_costs_are_cosines():
    A = csr([[3.0, 4.0, 0.0], [0.0, 4.0, 3.0], [0.0, 0.0, 2.0]])
    g = rip_graph(A, prescale=True, sparsify=False)
    D = as_dense(g)
    assert D[0, 1] == pytest.approx(16.0 / 25.0, rel=4e-16)
    assert D[1, 2] == pytest.approx(3.0 / 5.0, rel=4e-16)
    assert D[0, 2] == 0.0
    assert np.all(g.cost <= 1.0 + 4e-16)
    assert np.all(g.wgt >= 1) and np.all(g.wgt <= 2 ** 20 + 1)


def test_weights_are_ceilings():
    # ceil(y) is the integer w with w - 1 < y <= w; 2^20 * cost is exact in FP64
    p = workloads.small_config5(N=6, K=4)
    g = rip_graph(p.A)
    y = g.cost * 2.0 ** 20
    assert np.all(g.wgt >= y) and np.all(g.wgt - 1 < y)
    assert np.mean(g.wgt != np.round(y)) > 0.2   # fractional parts are common


def test_row_norm_order_and_values():
    rowptr = np.array([0, 3, 4])
    val = np.array([3.0, 4.0, 12.0, 2.0])
    assert np.array_equal(row_norms(rowptr, val), [13.0, 2.0])


def test_accumulation_is_sequential_in_column_order():
    # Products over the shared columns are added one by one in ascending column
    # order.  (1e16 + 1) - 1e16 rounds to 0: no edge.  (1e16 - 1e16) + 1 = 1: an
    # edge of cost 1, which a descending order ((1 - 1e16) + 1e16 = 0) would lose.
    A = csr([[1e16, 1.0, -1e16], [1.0, 1.0, 1.0], [0.0, 0.0, 1.0]])
    g = rip_graph(A, prescale=False, sparsify=False, alpha=1)
    assert 1 not in g.col[g.rowptr[0]:g.rowptr[1]]
    B = csr([[1e16, -1e16, 1.0], [1.0, 1.0, 1.0], [0.0, 0.0, 1.0]])
    g = rip_graph(B, prescale=False, sparsify=False, alpha=1)
    row0 = dict(zip(g.col[g.rowptr[0]:g.rowptr[1]].tolist(), g.cost[g.rowptr[0]:g.rowptr[1]]))
    assert row0[1] == 1.0
    with pytest.raises(ValueError):
        rip_graph(A, prescale=False, sparsify=False)   # 2^20 * |c_02| = 2^20 * 1e16 does not fit


def test_sparsify_keeps_largest_with_low_row_ties():
    n = 16  # isqrt = 4
    rowptr = np.arange(0, 2 * n + 1, 2)
    col = np.zeros(2 * n, dtype=np.int64)
    col[1::2] = np.arange(n)
    col[0] = 0
    # every row: entry in column 0 and its diagonal; rows 0..15 in column 0
    val = np.ones(2 * n)
    val[0::2] = [1, 5, 2, 5, 3, 5, 1, 0.5, 4, 4, 4, 0.1, 0.2, 0.3, 0.4, 0.6]
    rows_ = np.repeat(np.arange(n), 2)
    entries = np.stack([rows_, col, val], 1)
    keep = sparsify_columns(n, rowptr, col.astype(np.int64), val, 4)
    kept_rows_col0 = sorted(int(r) for r, c, v, k in zip(rows_, col, val, keep) if c == 0 and k)
    # |5| at rows 1,3,5 then the tie at 4 between rows 8,9,10 goes to row 8
    assert kept_rows_col0 == [1, 3, 5, 8]
    assert entries.shape[0] == keep.size


def test_symmetric_bitwise_and_rows_subset():
    p = workloads.small_config5(N=6, K=4)
    g = rip_graph(p.A)
    D = as_dense(g)
    assert np.array_equal(D, D.T)
    sub = np.array([0, 7, 100, 215])
    gr = rip_rows(p.A, sub)
    for t, i in enumerate(sub):
        a = slice(g.rowptr[i], g.rowptr[i + 1])
        b = slice(gr.rowptr[t], gr.rowptr[t + 1])
        assert np.array_equal(g.col[a], gr.col[b])
        assert np.array_equal(g.cost[a], gr.cost[b])
        assert np.array_equal(g.wgt[a], gr.wgt[b])


def test_stencil_graph_size():
    # 3D 7-point: rows share a column iff their grid distance <= 2 in the stencil sense
    p = workloads.small_config2(N=8, K=4)
    g = rip_graph(p.A)
    deg = np.diff(g.rowptr)
    assert deg.max() == 24  # interior vertex: 6 (dist 1) + 12 (diag) + 6 (dist 2)
    assert np.all(g.cost > 0) and np.all(g.cost <= 1.0 + 4e-16)
