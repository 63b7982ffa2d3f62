"""Block CG on H for several right-hand sides (``bc_solve_block``) on the GPU
against the oracle's ``block_cimmino_block_cg`` (needs an MI355X).

Bars (FP64 factors): per column the oracle's iteration count (a difference of
one only as a near-tie of the stop decision) and, at a fixed iteration count
with tol = 0, the iterate within 1e-8 relative; repeated right-hand sides give
identical columns and a zero right-hand side stops at iteration 0.  With FP32
applies: every column reaches the tolerance on its true residual.
"""
import numpy as np
import pytest

import paper_1710_07769_amd as bc
import workloads
from oracle import BlockProjections, block_cimmino_block_cg, block_cimmino_cg
from _bars import counts_match

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def banner(msg):
    print("\n[case] " + msg, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def st27(N, K):
    p = workloads.small_config5(N=N, K=K)
    return p, workloads.blocks_to_part(workloads.contiguous_blocks(p.n, K))


def block_residual_at(A, F, part, K, B, tol, j):
    """The oracle's relative true residual of column j after t block
    iterations (its run to tol stopped at t)."""
    return lambda t: block_cimmino_block_cg(A, F.T, part, K, tol=tol, maxit=t,
                                            proj=B).rel_residual[j]


def check_vs_oracle(dev, p, part, K, F, tol=1e-10, fixed=(1, 3, 6), **opts):
    A = p.A.to_scipy()
    B = BlockProjections(A, part, K)
    ref = block_cimmino_block_cg(A, F.T, part, K, tol=tol, proj=B)
    solver = bc.BlockCimmino(p.A, part, K, spmv_lanes=-1, **opts)
    try:
        Fd = torch.from_numpy(np.ascontiguousarray(F)).to(dev)
        X, sts = solver.solve_block(Fd, tol=tol, maxit=2000)
        X = X.cpu().numpy()
        for j, st in enumerate(sts):
            print("rhs %d: iterations gpu=%d oracle=%d status %d rel_res=%.2e"
                  % (j, st.iterations, ref.iterations[j], st.status, st.rel_residual))
            assert st.status == bc.BC_OK and st.rel_residual <= tol * (1 + 1e-6)
            # iterates are compared at fixed counts below
            counts_match(st.iterations, int(ref.iterations[j]),
                         block_residual_at(A, F, part, K, B, tol, j), tol, "rhs %d" % j)
        for k in fixed:
            refk = block_cimmino_block_cg(A, F.T, part, K, tol=0.0, maxit=k, proj=B)
            Xk, stk = solver.solve_block(Fd, tol=0.0, maxit=k)
            Xk = Xk.cpu().numpy()
            err = max(rel(Xk[j], refk.X[:, j]) for j in range(F.shape[0]))
            print("after %d iterations: max rel err vs oracle %.3e" % (k, err))
            assert all(s.iterations == k and s.status == bc.BC_NOT_CONVERGED for s in stk)
            assert err <= 1e-8
        return X, sts, ref
    finally:
        solver.close()


def test_block_cg_dense_fp64(dev):
    banner("bc_solve_block st27-10 K=6 dense FP64, 4 right-hand sides")
    p, part = st27(10, 6)
    F, _ = workloads.multi_rhs(p.A, 4, 21)
    X, sts, ref = check_vs_oracle(dev, p, part, 6, F, projection=bc.BC_PROJ_DENSE_CHOL)
    # one Krylov space for all: no more iterations than CG for each alone
    cg = max(block_cimmino_cg(p.A.to_scipy(), F[j], part, 6, tol=1e-10).iterations
             for j in range(4))
    print("block iterations %d, CG per right-hand side up to %d"
          % (max(s.iterations for s in sts), cg))
    assert max(s.iterations for s in sts) <= cg


def test_block_cg_one_rhs_is_cg(dev):
    banner("bc_solve_block with one right-hand side against bc_solve (Algorithm 2)")
    p, part = st27(10, 6)
    solver = bc.BlockCimmino(p.A, part, 6, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        f = torch.from_numpy(p.f).to(dev)
        x1, st1 = solver.solve(f, tol=1e-10)
        X, sts = solver.solve_block(f.reshape(1, -1).contiguous(), tol=1e-10)
        print("iterations block=%d cg=%d" % (sts[0].iterations, st1.iterations))
        ref = block_cimmino_cg(p.A.to_scipy(), p.f, part, 6, tol=1e-10)
        if counts_match(sts[0].iterations, st1.iterations, lambda t: ref.history[t], 1e-10):
            assert rel(X[0].cpu().numpy(), x1.cpu().numpy()) <= 1e-8
    finally:
        solver.close()


def test_block_cg_banded(dev):
    banner("bc_solve_block st27-8 K=8 banded FP64, 3 right-hand sides")
    p, part = st27(8, 8)
    F, _ = workloads.multi_rhs(p.A, 3, 22)
    check_vs_oracle(dev, p, part, 8, F, fixed=(2, 4), projection=bc.BC_PROJ_BAND_CHOL)


def test_block_cg_inner_cg(dev):
    banner("bc_solve_block cd3d-12 K=4 inner CG FP64, 2 right-hand sides")
    p = workloads.small_config2(N=12, K=4)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, 4))
    F, _ = workloads.multi_rhs(p.A, 2, 23)
    check_vs_oracle(dev, p, part, 4, F, fixed=(2, 5), projection=bc.BC_PROJ_INNER_CG)


def test_block_cg_dependent_and_zero(dev):
    banner("bc_solve_block: repeated, dependent and zero right-hand sides")
    p, part = st27(8, 4)
    F, _ = workloads.multi_rhs(p.A, 5, 24)
    F[1] = F[0]
    F[3] = 2.0 * F[0] - F[2]
    F[4] = 0.0
    A = p.A.to_scipy()
    ref = block_cimmino_block_cg(A, F.T, part, 4, tol=1e-10)
    solver = bc.BlockCimmino(p.A, part, 4, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        X, sts = solver.solve_block(torch.from_numpy(F).to(dev), tol=1e-10)
        X = X.cpu().numpy()
        print("iterations", [s.iterations for s in sts], "oracle", list(ref.iterations))
        assert sts[4].iterations == 0 and sts[4].status == bc.BC_OK and not X[4].any()
        assert all(s.status == bc.BC_OK and s.rel_residual <= 1e-10 * (1 + 1e-6) for s in sts)
        assert np.array_equal(X[0], X[1])
        B = BlockProjections(A, part, 4)
        for j in range(4):
            if counts_match(sts[j].iterations, int(ref.iterations[j]),
                            block_residual_at(A, F, part, 4, B, 1e-10, j), 1e-10, "rhs %d" % j):
                assert rel(X[j], ref.X[:, j]) <= 1e-7
    finally:
        solver.close()


def test_block_cg_fp32_applies_and_x0(dev):
    banner("bc_solve_block st27-10 K=6 FP32 dense applies, 6 right-hand sides; exact start")
    p, part = st27(10, 6)
    F, Xs = workloads.multi_rhs(p.A, 6, 25)
    solver = bc.BlockCimmino(p.A, part, 6, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL,
                             precision=bc.BC_MIXED_PROJ)
    try:
        Fd = torch.from_numpy(F).to(dev)
        X, sts = solver.solve_block(Fd, tol=1e-10)
        print("iterations", [s.iterations for s in sts])
        assert all(s.status == bc.BC_OK and s.rel_residual <= 1e-10 * (1 + 1e-6) for s in sts)
        for j in range(6):
            assert rel(X[j].cpu().numpy(), Xs[j]) <= 1e-6
        X2, sts2 = solver.solve_block(Fd, X0=torch.from_numpy(Xs).to(dev), tol=1e-10)
        assert all(s.iterations == 0 for s in sts2)
    finally:
        solver.close()


def test_block_cg_fp32_products(dev):
    banner("bc_solve_block st27-10 K=6 FP32 sparse products and dense applies, 5 right-hand "
           "sides")
    p, part = st27(10, 6)
    F, Xs = workloads.multi_rhs(p.A, 5, 27)
    solver = bc.BlockCimmino(p.A, part, 6, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL,
                             precision=bc.BC_MIXED)
    try:
        X, sts = solver.solve_block(torch.from_numpy(F).to(dev), tol=1e-10)
        print("iterations", [s.iterations for s in sts],
              "replacements", [s.replacements for s in sts])
        assert all(s.status == bc.BC_OK and s.rel_residual <= 1e-10 * (1 + 1e-6) for s in sts)
        for j in range(5):
            assert rel(X[j].cpu().numpy(), Xs[j]) <= 1e-6
    finally:
        solver.close()


def test_block_cg_sixteen_columns(dev):
    banner("bc_solve_block st27-8 K=4 dense FP64, 16 right-hand sides (32-column Gram lists); "
           "maxit = 0")
    p, part = st27(8, 4)
    F, _ = workloads.multi_rhs(p.A, 16, 28)
    X, sts, ref = check_vs_oracle(dev, p, part, 4, F, fixed=(1, 3),
                                  projection=bc.BC_PROJ_DENSE_CHOL)
    print("block iterations", [s.iterations for s in sts])
    solver = bc.BlockCimmino(p.A, part, 4, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        Fd = torch.from_numpy(F).to(dev)
        X0 = torch.zeros_like(Fd)
        X0[3] = 1.0
        X1, st1 = solver.solve_block(Fd, X0=X0, tol=1e-10, maxit=0)
        assert all(s.iterations == 0 and s.status == bc.BC_NOT_CONVERGED for s in st1)
        assert torch.equal(X1, X0)
    finally:
        solver.close()


def test_block_cg_rejects_bad_calls(dev):
    banner("bc_solve_block argument errors")
    p, part = st27(6, 3)
    solver = bc.BlockCimmino(p.A, part, 3, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        F = torch.zeros(17, p.n, dtype=torch.float64, device=dev)
        with pytest.raises(bc.BCError):
            solver.solve_block(F)
    finally:
        solver.close()


def test_block_cg_fullsize_st27_100cubed(dev):
    banner("bc_solve_block st27-100 n=1e6 K=512 FP32 dense applies, 8 right-hand sides")
    p = workloads.config5()
    F, Xs = workloads.multi_rhs(p.A, 8, 26)
    solver = bc.BlockCimmino(p.A, p.part(), p.K, spmv_lanes=-1,
                             projection=bc.BC_PROJ_DENSE_CHOL, precision=bc.BC_MIXED_PROJ)
    try:
        Fd = torch.from_numpy(F).to(dev)
        X, sts = solver.solve_block(Fd, tol=1e-10, maxit=500)
        Xm, stm = solver.solve_multi(Fd, tol=1e-10, maxit=500)
        print("block iterations", [s.iterations for s in sts], "t %.1f ms" % sts[0].t_solve_ms)
        print("independent CG iterations", [s.iterations for s in stm],
              "t %.1f ms" % stm[0].t_solve_ms)
        assert all(s.status == bc.BC_OK and s.rel_residual <= 1e-10 * (1 + 1e-6) for s in sts)
        assert max(s.iterations for s in sts) <= max(s.iterations for s in stm)
        X = X.cpu().numpy()
        for j in range(8):
            assert rel(X[j], Xs[j]) <= 1e-6
    finally:
        solver.close()
