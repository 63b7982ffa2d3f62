"""Row inner-product graph G_RIP(A) (oracle; test infrastructure).

Section 2.1: one vertex per row of A and an edge (v_i, v_j) wherever the row
inner product r_i r_j^T is nonzero, with cost |r_i r_j^T|.  The graph is the
off-diagonal pattern of C = A A^T with |c_ij| as costs.  Section 2.1 prescales
the rows to unit 2-norm so that a cost is the cosine of the angle between two
rows.  Section 2.3 builds C with a row-wise sparse product, first replacing
each dense column (more than sqrt(n) nonzeros) by its sqrt(n) largest entries
in absolute value, and gives METIS integer weights wgt = ceil(alpha * cost).

Readings taken where the text leaves freedom:

* row norm: sqrt of the sum of squares accumulated in ascending column order;
  the prescaled value is a / norm (both correctly rounded);
* dense-column threshold t = isqrt(n); a column is dense if it stores more
  than t entries; the kept entries are the t largest |a| after prescaling,
  ties broken by the lower row index;
* c_ij is accumulated over the shared columns k in ascending k, each product
  rounded before it is added (no fused multiply-add);
* the diagonal and exact zero sums are not edges;
* alpha = 2^20, so alpha * cost is exact and wgt depends only on the cost bits;
  a weight that would not fit below 2^62 is an error (only possible without
  prescaling, where costs are not bounded by 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class RipGraph:
    n: int
    rowptr: np.ndarray  # int64 n+1
    col: np.ndarray     # int32
    cost: np.ndarray    # float64
    wgt: np.ndarray     # int64


def _segments_sequential_sum(starts: np.ndarray, lens: np.ndarray, vals: np.ndarray) -> np.ndarray:
    """out[s] = (((0 + v[start]) + v[start+1]) + ...) in strictly sequential order."""
    out = np.zeros(starts.size)
    if starts.size == 0:
        return out
    for j in range(int(lens.max()) if lens.size else 0):
        sel = lens > j
        out[sel] = out[sel] + vals[starts[sel] + j]
    return out


def row_norms(rowptr, val) -> np.ndarray:
    """||r_i||_2 with squares summed in ascending column order."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    sq = np.asarray(val, dtype=np.float64) * np.asarray(val, dtype=np.float64)
    return np.sqrt(_segments_sequential_sum(rowptr[:-1], np.diff(rowptr), sq))


def sparsify_columns(n, rowptr, col, val, t):
    """Keep, in every column with more than t entries, its t largest |val|
    (ties to the lower row).  Returns a boolean keep-mask over the entries."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    keep = np.ones(col.size, dtype=bool)
    counts = np.bincount(col, minlength=n)
    for c in np.flatnonzero(counts > t):
        ent = np.flatnonzero(col == c)
        order = np.lexsort((rows[ent], -np.abs(val[ent])))
        keep[ent[order[t:]]] = False
    return keep


def _prepared(A, prescale, sparsify):
    n = A.n
    rowptr = np.asarray(A.rowptr, dtype=np.int64)
    col = np.asarray(A.col, dtype=np.int64)
    val = np.asarray(A.val, dtype=np.float64).copy()
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    if prescale:
        nrm = row_norms(rowptr, val)
        if np.any(nrm == 0.0):
            raise ValueError("zero row: cannot prescale")
        val = val / nrm[rows]
    if sparsify:
        keep = sparsify_columns(n, rowptr, col, val, math.isqrt(n))
        rows, col, val = rows[keep], col[keep], val[keep]
    return n, rows, col, val


def _column_lists(n, rows, col, val):
    """Entries of the (sparsified) matrix grouped by column, rows ascending."""
    order = np.lexsort((rows, col))
    cptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(col, minlength=n), out=cptr[1:])
    return cptr, rows[order], val[order]


def _products(rows_i, col_i, val_i, cptr, crow, cval):
    """All products a_ik * a_jk for the given (i, k, a_ik) entries: (i, j, k, prod)."""
    cnt = cptr[col_i + 1] - cptr[col_i]
    rep_i = np.repeat(rows_i, cnt)
    rep_k = np.repeat(col_i, cnt)
    rep_a = np.repeat(val_i, cnt)
    first = np.repeat(cptr[col_i], cnt)
    offs = np.arange(rep_i.size) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    pos = first + offs
    return rep_i, crow[pos], rep_k, rep_a * cval[pos]


def _assemble(n_rows_out, row_ids, i, j, k, prod, alpha):
    order = np.lexsort((k, j, i))
    i, j, prod = i[order], j[order], prod[order]
    newpair = np.ones(i.size, dtype=bool)
    newpair[1:] = (i[1:] != i[:-1]) | (j[1:] != j[:-1])
    starts = np.flatnonzero(newpair)
    lens = np.diff(np.append(starts, i.size))
    c = _segments_sequential_sum(starts, lens, prod)
    pi, pj = i[starts], j[starts]
    edge = (pi != pj) & (c != 0.0)
    pi, pj, c = pi[edge], pj[edge], c[edge]
    cost = np.abs(c)
    scaled = cost * float(alpha)
    if scaled.size and not (np.all(np.isfinite(scaled)) and scaled.max() < 2.0 ** 62):
        raise ValueError("alpha * cost does not fit a 62-bit integer weight")
    wgt = np.ceil(scaled).astype(np.int64)
    pos = np.searchsorted(row_ids, pi)
    rowptr = np.zeros(n_rows_out + 1, dtype=np.int64)
    np.cumsum(np.bincount(pos, minlength=n_rows_out), out=rowptr[1:])
    return RipGraph(n_rows_out, rowptr, pj.astype(np.int32), cost, wgt)


def rip_graph(A, prescale=True, sparsify=True, alpha=1 << 20) -> RipGraph:
    """Edges, costs and integer weights of G_RIP(A) (Sections 2.1 and 2.3).

    ``A`` is any object with ``n``, ``rowptr``, ``col``, ``val`` (CSR).  The
    result is a symmetric adjacency in CSR form without the diagonal."""
    n, rows, col, val = _prepared(A, prescale, sparsify)
    cptr, crow, cval = _column_lists(n, rows, col, val)
    i, j, k, prod = _products(rows, col, val, cptr, crow, cval)
    return _assemble(n, np.arange(n), i, j, k, prod, alpha)


def rip_rows(A, row_ids, prescale=True, sparsify=True, alpha=1 << 20) -> RipGraph:
    """Rows ``row_ids`` (ascending) of G_RIP(A) only: for sampled checks of
    graphs too large to build whole here."""
    row_ids = np.asarray(row_ids, dtype=np.int64)
    n, rows, col, val = _prepared(A, prescale, sparsify)
    cptr, crow, cval = _column_lists(n, rows, col, val)
    sel = np.isin(rows, row_ids)
    i, j, k, prod = _products(rows[sel], col[sel], val[sel], cptr, crow, cval)
    return _assemble(row_ids.size, row_ids, i, j, k, prod, alpha)
