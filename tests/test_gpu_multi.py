"""Several right-hand sides of one system (``bc_solve_multi``) on the GPU
(needs an MI355X).

Bars:
* each right-hand side of a multi solve ends with the iteration count, status
  and iterate bits of a ``bc_solve_multi`` of that right-hand side alone
  (the sliced-ELL products and the matrix-core dense sweeps give every vector
  the same bits whatever else its chunk holds); this holds for dense FP64 and
  FP32-apply factors, banded factors and inner-CG blocks, for chunks that
  leave a ragged tail and for right-hand sides that stop at different
  iterations.  Where a wide chunk takes the row-owned dense sweep (blocks
  large enough that its LDS fits one workgroup per CU) and a narrow one the
  lockstep sweep, the two sum in different orders: then the bits agree
  between solves whose chunks take the same sweep, and the rest is held to
  the tolerance bars below;
* against ``bc_solve`` of the same right-hand side (sliced-ELL products forced
  with spmv_lanes = -1 on both): banded and inner-CG blocks take the same
  kernels, so the bits agree (inner CG with several workgroups per block in
  ``bc_solve`` but enough vectors x blocks to fill the CUs runs the
  one-workgroup kernel for all vectors at once: then the bits agree with a
  one-workgroup context and the iterates with ``bc_solve`` to 1e-9);
  dense blocks use the one-vector sweeps there,
  so the iteration count agrees within one (FP64) or two (FP32 applies) and
  the iterates within 1e-9 (FP64) or 1e-6 (FP32 applies) relative;
* against the oracle (Algorithm 2 per right-hand side, FP64): the iteration
  count (a difference of one only as a near-tie of the stop decision) and, at
  the oracle's count, the iterate within 1e-8 relative (FP64 factors).
"""
import numpy as np
import pytest

import paper_1710_07769_amd as bc
import workloads
from _bars import counts_match
from oracle import backward_error, block_cimmino_cg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def banner(msg):
    print("\n[case] " + msg, flush=True)



def backward_error_at(A, f, part, K, t):
    """The oracle's normwise backward error (eq. (stopping)) after t
    iterations of Algorithm 2."""
    r = block_cimmino_cg(A, f, part, K, tol=0.0, maxit=t)
    return backward_error(A, r.x, f)

def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def st27(N, K):
    p = workloads.small_config5(N=N, K=K)
    return p, workloads.blocks_to_part(workloads.contiguous_blocks(p.n, K))


def check_multi(dev, p, part, K, nrhs, seed, tol=1e-10, maxit=5000, F=None, single_exact=True,
                single_bar=(0, 0.0), **opts):
    """Multi solve against one-vector multi solves (same bits) and against one
    bc_solve per right-hand side (same bits when single_exact, else within
    single_bar = (iterations, relative error)).  Returns (F, X, stats)."""
    if F is None:
        F, _ = workloads.multi_rhs(p.A, nrhs, seed)
    solver = bc.BlockCimmino(p.A, part, K, spmv_lanes=-1, **opts)
    try:
        Fd = torch.from_numpy(F).to(dev)
        X, sts = solver.solve_multi(Fd, tol=tol, maxit=maxit)
        X = X.cpu().numpy()
        assert len(sts) == nrhs
        for j in range(nrhs):
            x1, st1 = solver.solve_multi(Fd[j:j + 1].contiguous(), tol=tol, maxit=maxit)
            x1 = x1.cpu().numpy()[0]
            xs, sts_ = solver.solve(Fd[j].contiguous(), tol=tol, maxit=maxit)
            xs = xs.cpu().numpy()
            print("rhs %d: iterations multi=%d alone=%d bc_solve=%d status %d/%d/%d rel_res=%.2e "
                  "rel_diff_vs_bc_solve=%.2e"
                  % (j, sts[j].iterations, st1[0].iterations, sts_.iterations, sts[j].status,
                     st1[0].status, sts_.status, sts[j].rel_residual, rel(X[j], xs)))
            assert sts[j].iterations == st1[0].iterations
            assert sts[j].status == st1[0].status
            assert np.array_equal(X[j], x1), "rhs %d: max diff %.3e" % (j, np.abs(X[j] - x1).max())
            assert sts[j].rel_residual == st1[0].rel_residual
            assert sts[j].status == sts_.status
            if single_exact:
                assert sts[j].iterations == sts_.iterations
                assert np.array_equal(X[j], xs)
            else:
                assert abs(sts[j].iterations - sts_.iterations) <= single_bar[0]
                assert rel(X[j], xs) <= single_bar[1]
        return F, X, sts
    finally:
        solver.close()


FP64_DENSE = dict(single_exact=False, single_bar=(1, 1e-9))
FP32_DENSE = dict(single_exact=False, single_bar=(2, 1e-6))


def test_multi_dense_fp64_matches_single_and_oracle(dev):
    banner("bc_solve_multi st27-10 K=6 dense FP64, 5 right-hand sides")
    p, part = st27(10, 6)
    F, X, sts = check_multi(dev, p, part, 6, 5, seed=11, projection=bc.BC_PROJ_DENSE_CHOL,
                            **FP64_DENSE)
    A = p.A.to_scipy()
    for j in (0, 3):
        ref = block_cimmino_cg(A, F[j], part, 6, tol=1e-10)
        print("rhs %d: oracle iterations %d" % (j, ref.iterations))
        assert sts[j].status == bc.BC_OK
        counts_match(sts[j].iterations, ref.iterations, lambda t: ref.history[t], 1e-10)
    # at the oracle's count, the iterates agree
    solver = bc.BlockCimmino(p.A, part, 6, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        ref0 = block_cimmino_cg(A, F[0], part, 6, tol=1e-10)
        Xd, sts2 = solver.solve_multi(torch.from_numpy(F).to(dev), tol=0.0, maxit=ref0.iterations)
        Xd = Xd.cpu().numpy()
        for j in (0, 3):
            refj = block_cimmino_cg(A, F[j], part, 6, tol=0.0, maxit=ref0.iterations)
            assert sts2[j].iterations == ref0.iterations
            err = rel(Xd[j], refj.x)
            print("rhs %d at %d iterations: rel_err vs oracle %.3e" % (j, ref0.iterations, err))
            assert err <= 1e-8
    finally:
        solver.close()


@pytest.mark.parametrize("nrhs", [1, 2, 9, 17])
def test_multi_dense_fp32_applies_ragged_chunks(dev, nrhs):
    banner("bc_solve_multi st27-10 K=6 FP32 dense applies, %d right-hand sides" % nrhs)
    p, part = st27(10, 6)
    check_multi(dev, p, part, 6, nrhs, seed=12, projection=bc.BC_PROJ_DENSE_CHOL,
                precision=bc.BC_MIXED_PROJ, **FP32_DENSE)


@pytest.mark.parametrize("nrhs", [3, 12])
def test_multi_dense_fp64_chunks(dev, nrhs):
    banner("bc_solve_multi st27-10 K=6 FP64 dense, %d right-hand sides" % nrhs)
    p, part = st27(10, 6)
    check_multi(dev, p, part, 6, nrhs, seed=18, projection=bc.BC_PROJ_DENSE_CHOL, **FP64_DENSE)


def test_multi_dense_row_owned_sweep(dev):
    banner("bc_solve_multi st27-14 K=2 FP32 dense applies (1372-row blocks), 16 right-hand "
           "sides: chunks of 16 take the row-owned sweep")
    p, part = st27(14, 2)
    F, _ = workloads.multi_rhs(p.A, 16, 33)
    solver = bc.BlockCimmino(p.A, part, 2, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL,
                             precision=bc.BC_MIXED_PROJ)
    try:
        Fd = torch.from_numpy(F).to(dev)
        X, sts = solver.solve_multi(Fd, tol=1e-10, maxit=3000)
        # 9 vectors also take a chunk of 16 (same sweep): the same bits
        X9, sts9 = solver.solve_multi(Fd[:9].contiguous(), tol=1e-10, maxit=3000)
        assert torch.equal(X9, X[:9])
        assert [s.iterations for s in sts9] == [s.iterations for s in sts[:9]]
        A = p.A.to_scipy()
        for j in (0, 15):
            xs, st1 = solver.solve(Fd[j].contiguous(), tol=1e-10, maxit=3000)
            ref = block_cimmino_cg(A, F[j], part, 2, tol=1e-10)
            print("rhs %d: iterations multi=%d bc_solve=%d oracle(FP64)=%d rel_res=%.2e"
                  % (j, sts[j].iterations, st1.iterations, ref.iterations, sts[j].rel_residual))
            assert sts[j].status == bc.BC_OK and sts[j].rel_residual <= 1e-10 * (1 + 1e-6)
            assert abs(sts[j].iterations - st1.iterations) <= 2
            assert rel(X[j].cpu().numpy(), xs.cpu().numpy()) <= 1e-6
            assert rel(X[j].cpu().numpy(), ref.x) <= 1e-6
    finally:
        solver.close()


def test_multi_banded(dev):
    banner("bc_solve_multi st27-8 K=8 banded FP64, 3 right-hand sides")
    p, part = st27(8, 8)
    check_multi(dev, p, part, 8, 3, seed=13, projection=bc.BC_PROJ_BAND_CHOL)


@pytest.mark.parametrize("gather", [bc.BC_GATHER_SEPARATE, bc.BC_GATHER_INTERLEAVED])
def test_multi_gather_layouts(dev, gather):
    banner("bc_solve_multi st27-10 K=6, 11 right-hand sides (chunks of 8 + 3), FP32 sparse "
           "products, gather layout %d: dense FP32 applies, then banded" % gather)
    p, part = st27(10, 6)
    check_multi(dev, p, part, 6, 11, seed=41, multi_gather=gather, precision=bc.BC_MIXED,
                projection=bc.BC_PROJ_DENSE_CHOL, **FP32_DENSE)
    check_multi(dev, p, part, 6, 11, seed=42, multi_gather=gather,
                projection=bc.BC_PROJ_BAND_CHOL)


def test_gather_layouts_same_bits(dev):
    banner("separate against interleaved gathers: bc_solve_multi (banded, 11 right-hand "
           "sides, FP64 and FP32 products) and bc_solve_block (dense, 5)")
    p, part = st27(10, 6)
    F, _ = workloads.multi_rhs(p.A, 11, 43)
    Fd = torch.from_numpy(F).to(dev)

    def run(gather, method, nr, **opts):
        s = bc.BlockCimmino(p.A, part, 6, spmv_lanes=-1, multi_gather=gather, **opts)
        try:
            X, sts = getattr(s, method)(Fd[:nr].contiguous(), tol=1e-10, maxit=2000)
            return X.cpu().numpy(), [(t.iterations, t.status) for t in sts]
        finally:
            s.close()
    for method, nr, opts in (
            ("solve_multi", 11, dict(projection=bc.BC_PROJ_BAND_CHOL)),
            ("solve_multi", 11, dict(projection=bc.BC_PROJ_BAND_CHOL, precision=bc.BC_MIXED)),
            ("solve_block", 5, dict(projection=bc.BC_PROJ_DENSE_CHOL))):
        Xs, ss = run(bc.BC_GATHER_SEPARATE, method, nr, **opts)
        Xi, si = run(bc.BC_GATHER_INTERLEAVED, method, nr, **opts)
        print(method, opts, "iterations", [t[0] for t in ss])
        assert ss == si and all(t[1] == bc.BC_OK for t in ss)
        assert np.array_equal(Xs, Xi)


def test_multi_inner_cg(dev):
    banner("bc_solve_multi cd3d-12 K=4 inner CG FP64, 2 right-hand sides")
    p = workloads.small_config2(N=12, K=4)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, 4))
    check_multi(dev, p, part, 4, 2, seed=14, projection=bc.BC_PROJ_INNER_CG)


def test_multi_inner_cg_one_launch(dev):
    banner("bc_solve_multi cd3d-16 K=8 inner CG FP64, 32 right-hand sides: blocks x vectors "
           "fill the CUs, so all vectors run in one single-workgroup launch")
    p = workloads.small_config2(N=16, K=8)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, 8))
    F, _ = workloads.multi_rhs(p.A, 32, 44)
    Fd = torch.from_numpy(F).to(dev)
    grouped = bc.BlockCimmino(p.A, part, 8, spmv_lanes=-1, projection=bc.BC_PROJ_INNER_CG)
    single = bc.BlockCimmino(p.A, part, 8, spmv_lanes=-1, projection=bc.BC_PROJ_INNER_CG,
                             inner_groups=1)
    try:
        X, sts = grouped.solve_multi(Fd, tol=1e-10)
        X1, sts1 = single.solve_multi(Fd, tol=1e-10)
        X = X.cpu().numpy()
        # the same kernel either way: the same bits, also against bc_solve with one
        # workgroup per block
        assert np.array_equal(X, X1.cpu().numpy())
        assert [s.iterations for s in sts] == [s.iterations for s in sts1]
        for j in (0, 7, 31):
            xs, st = single.solve(Fd[j].contiguous(), tol=1e-10)
            assert st.iterations == sts[j].iterations and np.array_equal(X[j], xs.cpu().numpy())
        # against the grouped kernel one vector at a time: the same iterates up to rounding
        for j in range(32):
            xg, stg = grouped.solve(Fd[j].contiguous(), tol=1e-10)
            assert sts[j].status == bc.BC_OK and sts[j].rel_residual <= 1e-10 * (1 + 1e-6)
            hist = lambda t, j=j: block_cimmino_cg(p.A.to_scipy(), F[j], part, 8,
                                                   tol=1e-10).history[t]
            if counts_match(stg.iterations, sts[j].iterations, hist, 1e-10, "rhs %d" % j):
                assert rel(X[j], xg.cpu().numpy()) <= 1e-9
        ref = block_cimmino_cg(p.A.to_scipy(), F[5], part, 8, tol=1e-10)
        print("iterations", [s.iterations for s in sts][:8], "oracle rhs 5:", ref.iterations)
        if counts_match(sts[5].iterations, ref.iterations, lambda t: ref.history[t], 1e-10):
            assert rel(X[5], ref.x) <= 1e-8
    finally:
        grouped.close()
        single.close()


def test_multi_inner_cg_fp32_values_one_launch(dev):
    banner("bc_solve_multi cd3d-16 K=8 inner CG in FP64 arithmetic on FP32 block values, "
           "32 right-hand sides in one single-workgroup launch")
    p = workloads.small_config2(N=16, K=8)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, 8))
    F, _ = workloads.multi_rhs(p.A, 32, 45)
    Fd = torch.from_numpy(F).to(dev)
    single = bc.BlockCimmino(p.A, part, 8, spmv_lanes=-1, projection=bc.BC_PROJ_INNER_CG,
                             inner_groups=1, precision=bc.BC_MIXED_PROJ)
    try:
        X, sts = single.solve_multi(Fd, tol=1e-10)
        X = X.cpu().numpy()
        assert all(s.status == bc.BC_OK and s.rel_residual <= 1e-10 * (1 + 1e-6) for s in sts)
        assert all(s.replacements == 0 for s in sts)
        # the same kernel one vector at a time: the same bits
        for j in (0, 13, 31):
            xs, st = single.solve(Fd[j].contiguous(), tol=1e-10)
            assert st.iterations == sts[j].iterations and np.array_equal(X[j], xs.cpu().numpy())
        # the FP32 values perturb the operator, not its solution: the FP64 oracle's
        # count within 1 and its solution within 1e-9 (measured: equal counts,
        # 5e-13 to 3e-12)
        for j in (0, 5, 31):
            ref = block_cimmino_cg(p.A.to_scipy(), F[j], part, 8, tol=1e-10)
            print("rhs %d: iterations %d, oracle (FP64) %d, rel err %.2e"
                  % (j, sts[j].iterations, ref.iterations, rel(X[j], ref.x)))
            assert abs(sts[j].iterations - ref.iterations) <= 1
            assert rel(X[j], ref.x) <= 1e-9
    finally:
        single.close()


def test_multi_inner_cg_mixed_restarts(dev):
    banner("bc_solve_multi powerlaw-6000 K=4 FP32 products and inner CG (restarts every 20), "
           "3 right-hand sides")
    p = workloads.small_config3(n=6000, K=4)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, 4))
    F, X, sts = check_multi(dev, p, part, 4, 3, seed=31, projection=bc.BC_PROJ_INNER_CG,
                            precision=bc.BC_MIXED)
    assert all(s.status == bc.BC_OK and s.replacements > 0 for s in sts)


def test_multi_backward_error_stop_rule(dev):
    banner("bc_solve_multi with the paper's backward-error stop rule, st27-10 K=6, 3 right-hand "
           "sides")
    p, part = st27(10, 6)
    F, X, sts = check_multi(dev, p, part, 6, 3, seed=32, tol=1e-12,
                            projection=bc.BC_PROJ_DENSE_CHOL, stop_rule=bc.BC_STOP_BACKWARD_ERR,
                            **FP64_DENSE)
    A = p.A.to_scipy()
    for j in range(3):
        ref = block_cimmino_cg(A, F[j], part, 6, tol=1e-12, stop="backward")
        print("rhs %d: iterations %d oracle %d backward error %.2e"
              % (j, sts[j].iterations, ref.iterations, sts[j].backward_err))
        assert sts[j].status == bc.BC_OK and sts[j].backward_err < 1e-12
        counts_match(sts[j].iterations, ref.iterations,
                     lambda t, j=j: backward_error_at(A, F[j], part, 6, t), 1e-12)


def test_multi_stops_independently(dev):
    banner("bc_solve_multi: zero, exact and ordinary right-hand sides stop on their own")
    p, part = st27(8, 4)
    F, _ = workloads.multi_rhs(p.A, 4, 15)
    F[1] = 0.0            # f = 0: converged before any iteration
    F[2] = 1e-3 * F[3]    # a scaled copy: the same iterations as F[3]
    F = np.ascontiguousarray(F)
    _, X, sts = check_multi(dev, p, part, 4, 4, seed=0, F=F, projection=bc.BC_PROJ_DENSE_CHOL,
                            **FP64_DENSE)
    assert sts[1].iterations == 0 and sts[1].status == bc.BC_OK
    assert float(np.abs(X[1]).max()) == 0.0
    assert sts[0].iterations > 0 and sts[3].iterations > 0


def test_multi_maxit_and_x0(dev):
    banner("bc_solve_multi: maxit, tol = 0 and a starting guess")
    p, part = st27(8, 4)
    F, Xs = workloads.multi_rhs(p.A, 3, 16)
    solver = bc.BlockCimmino(p.A, part, 4, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        Fd = torch.from_numpy(F).to(dev)
        X, sts = solver.solve_multi(Fd, tol=0.0, maxit=4)
        assert all(s.iterations == 4 and s.status == bc.BC_NOT_CONVERGED for s in sts)
        X0 = torch.from_numpy(np.ascontiguousarray(Xs)).to(dev)
        X2, sts2 = solver.solve_multi(Fd, X0=X0, tol=1e-10)
        assert all(s.iterations == 0 and s.status == bc.BC_OK for s in sts2)
        assert np.array_equal(X2.cpu().numpy(), Xs)
        # a different nrhs on the same context re-sizes the per-vector state
        X3, sts3 = solver.solve_multi(Fd[:2].contiguous(), tol=0.0, maxit=4)
        assert np.array_equal(X3.cpu().numpy(), X.cpu().numpy()[:2])
        for j in range(3):
            x1, st1 = solver.solve_multi(Fd[j:j + 1].contiguous(), tol=0.0, maxit=4)
            assert np.array_equal(x1.cpu().numpy()[0], X.cpu().numpy()[j])
    finally:
        solver.close()


def test_multi_rejects_bad_calls(dev):
    banner("bc_solve_multi argument errors")
    cases = [st27(6, 3) + (3,), st27(8, 4) + (4,)]
    batched = bc.BlockCimminoBatched([(p.A, part, K) for p, part, K in cases],
                                     projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        n = batched.n
        f = torch.zeros(2 * n, dtype=torch.float64, device=dev)
        x = torch.empty_like(f)
        with pytest.raises(bc.BCError):
            bc.bc_solve_multi(batched.ctx, 2, f, None, 1e-10, 10, x)
    finally:
        batched.close()
    p, part = st27(6, 3)
    solver = bc.BlockCimmino(p.A, part, 3, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        f = torch.zeros(p.n, dtype=torch.float64, device=dev)
        x = torch.empty_like(f)
        with pytest.raises(ValueError):
            bc.bc_solve_multi(solver.ctx, 0, f, None, 1e-10, 10, x)
        with pytest.raises(ValueError):
            bc.bc_solve_multi(solver.ctx, 2, f, None, 1e-10, 10, x)
        # the C entry point itself refuses nrhs < 1
        import ctypes
        rc = bc._lib.bc_solve_multi(solver.ctx, 0, ctypes.c_void_p(f.data_ptr()), None, 1e-10, 10,
                                    ctypes.c_void_p(x.data_ptr()), None)
        assert rc == bc.BC_ERR_INVALID
        # and more vectors than 65535 chunks of 4 (checked before any buffer is read)
        rc = bc._lib.bc_solve_multi(solver.ctx, 65535 * 4 + 1, ctypes.c_void_p(f.data_ptr()),
                                    None, 1e-10, 10, ctypes.c_void_p(x.data_ptr()), None)
        assert rc == bc.BC_ERR_INVALID
    finally:
        solver.close()


def test_multi_fullsize_st27_100cubed(dev):
    banner("bc_solve_multi st27-100 n=1e6 K=512 FP32 dense applies, 8 right-hand sides; "
           "2 of them alone and against bc_solve")
    p = workloads.config5()
    part = p.part()
    F, _ = workloads.multi_rhs(p.A, 8, 17)
    solver = bc.BlockCimmino(p.A, part, p.K, spmv_lanes=-1, projection=bc.BC_PROJ_DENSE_CHOL,
                             precision=bc.BC_MIXED_PROJ)
    try:
        Fd = torch.from_numpy(F).to(dev)
        X, sts = solver.solve_multi(Fd, tol=1e-10, maxit=2000)
        print("iterations", [s.iterations for s in sts], "t_solve_ms %.1f" % sts[0].t_solve_ms)
        assert all(s.status == bc.BC_OK and s.rel_residual <= 1e-10 * (1 + 1e-6) for s in sts)
        for j in (0, 7):
            x1, st1 = solver.solve_multi(Fd[j:j + 1].contiguous(), tol=1e-10, maxit=2000)
            assert st1[0].iterations == sts[j].iterations
            assert torch.equal(x1[0], X[j])
            xs, sts_ = solver.solve(Fd[j].contiguous(), tol=1e-10, maxit=2000)
            print("rhs %d: bc_solve iterations %d, rel diff %.2e"
                  % (j, sts_.iterations, rel(X[j].cpu().numpy(), xs.cpu().numpy())))
            assert abs(sts_.iterations - sts[j].iterations) <= 2
            assert rel(X[j].cpu().numpy(), xs.cpu().numpy()) <= 1e-6
    finally:
        solver.close()
