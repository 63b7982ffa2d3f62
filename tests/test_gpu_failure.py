"""Failure paths on the GPU, each forced through the C ABI with every kernel
exiting normally.

* Bounded device waits: bc_set_wait_limit(ctx, 0) makes every wait of the
  inner-CG workgroups (barriers in global memory) and of the row-owned dense
  sweep (waves waiting for published rows) give up at its first check.  The
  call then returns BC_ERR_DEVICE, and after the limit is restored the same
  context gives the bits of a fresh context (the wait-error word is the
  context's own and is cleared at every call; the inner-CG barrier epochs
  restart from zero after a failed call).
* Breakdown of Algorithm 2 (p.psi <= 0): two identical rows in different
  blocks make H singular; with a right-hand side inconsistent in those rows
  and in one eigenspace of H, the first step reaches r = 0 exactly while
  f - A x stays nonzero, so the next step has p = 0 and p.psi = 0.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_1710_07769_amd as bc
import workloads
from workloads import Csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def banner(msg):
    print("\n[case] " + msg, flush=True)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def _gives_up_then_recovers(dev, A, part, K, **opts):
    v = to_dev(np.random.default_rng(7).standard_normal(A.n), dev)
    f = to_dev(A.to_scipy() @ np.ones(A.n), dev)
    fresh = bc.BlockCimmino(A, part, K, **opts)
    solver = bc.BlockCimmino(A, part, K, **opts)
    try:
        ref_hv = fresh.project(v).cpu().numpy()
        ref_x, ref_st = fresh.solve(f, tol=1e-10)
        bc.bc_set_wait_limit(solver.ctx, 0.0)
        with pytest.raises(bc.BCError) as e:
            solver.project(v)
        assert e.value.status == bc.BC_ERR_DEVICE
        with pytest.raises(bc.BCError) as e:
            solver.solve(f, tol=1e-10)
        assert e.value.status == bc.BC_ERR_DEVICE
        torch.cuda.synchronize()
        # the same context, limit restored: a clean call, bit for bit the
        # fresh context's results
        bc.bc_set_wait_limit(solver.ctx, 2.0)
        hv = solver.project(v).cpu().numpy()
        assert np.array_equal(hv, ref_hv)
        x, st = solver.solve(f, tol=1e-10)
        assert st.status == bc.BC_OK and st.iterations == ref_st.iterations
        assert np.array_equal(x.cpu().numpy(), ref_x.cpu().numpy())
    finally:
        solver.close()
        fresh.close()


def test_wait_limit_inner_cg_groups(dev):
    banner("inner CG with 4 workgroups per block: every barrier gives up, then the context "
           "recovers")
    p = workloads.small_config2(N=16, K=4)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, p.K))
    _gives_up_then_recovers(dev, p.A, part, p.K, projection=bc.BC_PROJ_INNER_CG, inner_groups=4)


def test_wait_limit_dense_row_owned_sweep(dev):
    banner("dense blocks of 2456 rows (row-owned sweep): every row wait gives up, then the "
           "context recovers")
    p = workloads.small_config5(N=17, K=2)
    _gives_up_then_recovers(dev, p.A, p.part(), p.K, projection=bc.BC_PROJ_DENSE_CHOL)


def test_wait_limit_rejects_bad_values(dev):
    p = workloads.config1()
    solver = bc.BlockCimmino(p.A, p.part(), p.K)
    try:
        for bad in (-1.0, float("nan"), float("inf")):
            with pytest.raises(bc.BCError) as e:
                bc.bc_set_wait_limit(solver.ctx, bad)
            assert e.value.status == bc.BC_ERR_INVALID
    finally:
        solver.close()


def test_breakdown_duplicate_rows_in_different_blocks(dev):
    banner("rows 0 and 1 identical, in different blocks: H singular, r = 0 after one step, "
           "then p.psi = 0")
    # rows of a 4x4 Hadamard matrix (norm 2, mutually orthogonal) with row 1
    # a copy of row 0: every block's rows are orthogonal, so the scaled block
    # Gram matrices are I and every step below is exact in FP64
    M = np.array([[1, 1, 1, 1], [1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1]], dtype=np.float64)
    A = Csr.from_scipy(sp.csr_matrix(M))
    part = np.array([0, 1, 0, 1], dtype=np.int32)
    # f inconsistent in the duplicated rows, xi = sum_i A_i^+ f_i = (1,1,1,1)
    # lies in the eigenspace of H for eigenvalue 2: alpha = 1/2, x = 1/2,
    # r = 0, while f - A x = (-1, 1, 0, 0)
    f = to_dev(np.array([1.0, 3.0, 0.0, 0.0]), dev)
    for proj in (bc.BC_PROJ_DENSE_CHOL, bc.BC_PROJ_BAND_CHOL):
        solver = bc.BlockCimmino(A, part, 2, projection=proj)
        try:
            x, st = solver.solve(f, tol=1e-10, maxit=100)
            assert st.status == bc.BC_ERR_BREAKDOWN, st.status
            assert st.iterations == 1
            assert np.array_equal(x.cpu().numpy(), np.full(4, 0.5))
        finally:
            solver.close()
