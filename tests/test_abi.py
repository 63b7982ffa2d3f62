"""C-ABI checks that need no GPU: every declared symbol is exported, host-side
validation rejects malformed input with BC_ERR_INVALID, and the library's
host partitioners reproduce the oracle's greedy and multilevel partitions bit for bit."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads
from oracle import rip_graph as oracle_rip, greedy_partition, cutsize, int_cut

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

bc = pytest.importorskip("paper_1710_07769_amd")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    return sorted({n for n in names if n.startswith(("bc_", "rip_")) and not n.endswith("_t")})


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 16
    lib = C.CDLL(bc.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_defaults_and_status_strings():
    o = bc.make_opts()
    assert o.precision == bc.BC_FP64 and o.projection == bc.BC_PROJ_AUTO
    assert o.dense_max_m == 4096 and o.inner_tol == 1e-12 and o.replace_every == 20
    assert o.stop_rule == bc.BC_STOP_REL2 and o.use_graph == 1 and o.spmv_lanes == 0
    assert o.multi_gather == bc.BC_GATHER_AUTO
    for s in (0, 1, -1, -2, -3, -4, -5):
        assert bc.status_str(s) not in ("", "unknown status")


def _expect_invalid(fn):
    with pytest.raises(bc.BCError) as ei:
        fn()
    assert ei.value.status == bc.BC_ERR_INVALID


def test_setup_validation_without_device():
    p = workloads.config1()
    A = p.A
    part = p.part()
    bad_col = A.col.copy(); bad_col[3] = p.n
    _expect_invalid(lambda: bc.bc_setup(p.n, A.rowptr, bad_col, A.val, p.K, part, stream=False))
    unsorted = A.col.copy(); unsorted[[0, 1]] = unsorted[[1, 0]]
    _expect_invalid(lambda: bc.bc_setup(p.n, A.rowptr, unsorted, A.val, p.K, part, stream=False))
    nanv = A.val.copy(); nanv[5] = np.nan
    _expect_invalid(lambda: bc.bc_setup(p.n, A.rowptr, A.col, nanv, p.K, part, stream=False))
    badp = part.copy(); badp[0] = p.K
    _expect_invalid(lambda: bc.bc_setup(p.n, A.rowptr, A.col, A.val, p.K, badp, stream=False))
    _expect_invalid(lambda: bc.bc_setup(p.n, A.rowptr, A.col, A.val, p.n + 1,
                                        np.arange(p.n), stream=False))
    empty = np.zeros(p.n, dtype=np.int32)  # blocks 1..K-1 empty
    _expect_invalid(lambda: bc.bc_setup(p.n, A.rowptr, A.col, A.val, p.K, empty, stream=False))
    badrp = A.rowptr.copy(); badrp[10] = badrp[11] + 1
    _expect_invalid(lambda: bc.bc_setup(p.n, badrp, A.col, A.val, p.K, part, stream=False))
    _expect_invalid(lambda: bc.rip_graph(p.n, A.rowptr, bad_col, A.val, stream=False))
    for bad in (-1, 3):
        _expect_invalid(lambda: bc.bc_setup(p.n, A.rowptr, A.col, A.val, p.K, part,
                                            bc.make_opts(multi_gather=bad), stream=False))
    _expect_invalid(lambda: bc.bc_set_wait_limit(None, 1.0))


@pytest.mark.parametrize("maker,K", [(workloads.config1, 4), (lambda: workloads.small_config2(N=12, K=6), 6),
                                     (lambda: workloads.small_config5(N=8, K=5), 5),
                                     (lambda: workloads.small_config3(n=3000, K=7), 7)])
def test_library_partitioner_matches_oracle(maker, K):
    p = maker()
    g = oracle_rip(p.A)
    for passes in (0, 1, 2):
        ref = greedy_partition(g, K, passes=passes)
        got = bc.bc_partition_greedy(g, K, passes=passes)
        assert np.array_equal(ref, got), passes
    cs, ic = bc.bc_partition_cut(g, got)
    assert ic == int_cut(g, got)
    assert cs == pytest.approx(cutsize(g, got), rel=1e-12)


@pytest.mark.parametrize("maker,K", [(workloads.config1, 4), (lambda: workloads.small_config2(N=12, K=6), 6),
                                     (lambda: workloads.small_config5(N=8, K=5), 5),
                                     (lambda: workloads.small_config3(n=3000, K=7), 7)])
def test_library_multilevel_partitioner_matches_oracle(maker, K):
    from oracle import multilevel_partition
    p = maker()
    g = oracle_rip(p.A)
    for passes in (0, 2):
        ref = multilevel_partition(g, K, passes=passes)
        got = bc.bc_partition_multilevel(g, K, passes=passes)
        assert np.array_equal(ref, got), passes


def test_library_multilevel_on_a_64_vertex_path():
    # one coarsening level (pairs), growth of 16 weight-2 coarse vertices,
    # FM passes that gain nothing at either level: the halves (the oracle's
    # hand-traced case)
    n = 64
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = []
    for v in range(n):
        col += [u for u in (v - 1, v + 1) if 0 <= u < n]
        rowptr[v + 1] = len(col)
    wgt = np.ones(len(col), dtype=np.int64)
    from oracle.ripgraph import RipGraph
    g = RipGraph(n, rowptr, np.array(col, dtype=np.int32), wgt.astype(np.float64), wgt)
    assert bc.bc_partition_multilevel(g, 2).tolist() == [0] * 32 + [1] * 32


def test_partitioner_rejects_bad_graphs():
    g = oracle_rip(workloads.config1().A)
    with pytest.raises(bc.BCError):
        bc.bc_partition_greedy(g, 0)
    with pytest.raises(bc.BCError):
        bc.bc_partition_greedy(g, g.n + 1)
    g.wgt = g.wgt.copy(); g.wgt[0] = 0
    with pytest.raises(bc.BCError):
        bc.bc_partition_greedy(g, 4)
