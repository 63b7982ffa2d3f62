"""GPU-vs-oracle parity through the C ABI (needs an MI355X).

Bars (floating point, from the arithmetic of each path):
* rip_graph pattern, costs and weights, partitions: bit-exact.
* bc_project, FP64 dense Cholesky: relative error <= 1e-10 against the
  oracle's QR projections (forward error ~ kappa(G_i) eps with kappa(G_i) < 1e4).
* bc_project, FP64 inner CG to 1e-13: <= 1e-9.
* bc_solve FP64: the same iteration count as the oracle (a difference of one
  is accepted only when the oracle's residual at that iteration is within
  1e-3 relative of the threshold) and, run for exactly the oracle's
  iteration count, ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-8.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_1710_07769_amd as bc
import workloads
from workloads import Csr
from oracle import (rip_graph as oracle_rip, greedy_partition, block_cimmino_cg,
                    BlockProjections, backward_error)
from _bars import counts_match

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------- rip_graph

def _dense_column_matrix(n, c, nz, seed):
    rng = np.random.default_rng(seed)
    A = sp.lil_matrix((n, n))
    A.setdiag(rng.uniform(1.0, 2.0, n))
    rows = rng.choice(n, nz, replace=False)
    A[rows, c] = rng.uniform(-1, 1, nz)
    A[c, c] = 3.0
    return Csr.from_scipy(A.tocsr())


def _dense_columns_matrix(n, cols, nz, seed):
    # several dense columns, values with repeated magnitudes (ties in the
    # sparsification order)
    rng = np.random.default_rng(seed)
    A = sp.lil_matrix((n, n))
    A.setdiag(rng.uniform(1.0, 2.0, n))
    for c in cols:
        rows = rng.choice(n, nz, replace=False)
        A[rows, c] = rng.choice([-0.5, 0.25, 0.5, 1.0], nz)
        A[c, c] = 3.0
    return Csr.from_scipy(A.tocsr())


def _int_matrix(n, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=0.05, random_state=rng,
                  data_rvs=lambda k: rng.integers(-9, 10, k).astype(float)).tocsr()
    M.eliminate_zeros()
    return Csr.from_scipy(M + sp.eye(n))


RIP_CASES = {
    "cd2d-32": lambda: workloads.config1().A,
    "cd3d-12": lambda: workloads.small_config2(N=12, K=4).A,
    "st27-10": lambda: workloads.small_config5(N=10, K=4).A,
    "powerlaw-4000": lambda: workloads.small_config3(n=4000, K=4).A,
    "dense-col-25": lambda: _dense_column_matrix(25, 3, 23, 0),
    "dense-col-2000": lambda: _dense_column_matrix(2000, 17, 600, 1),
    "int-300": lambda: _int_matrix(300, 2),
    "dense-cols-900": lambda: _dense_columns_matrix(900, [0, 5, 899, 450], 200, 3),
    "diagonal-50": lambda: Csr.from_scipy(sp.diags(np.arange(1.0, 51.0)).tocsr()),
    "single-1": lambda: Csr.from_scipy(sp.csr_matrix(np.array([[2.0]]))),
}


@pytest.mark.parametrize("name", sorted(RIP_CASES))
@pytest.mark.parametrize("prescale", [True, False])
def test_rip_graph_bitexact(dev, name, prescale):
    banner("rip_graph %s prescale=%s" % (name, prescale))
    A = RIP_CASES[name]()
    alpha = (1 << 20) if prescale else 1
    try:
        ref = oracle_rip(A, prescale=prescale, alpha=alpha)
    except ValueError:
        pytest.skip("weights overflow without prescaling")
    got = bc.rip_graph(A.n, A.rowptr, A.col, A.val, prescale=prescale, alpha=alpha)
    assert np.array_equal(got.rowptr, ref.rowptr)
    assert np.array_equal(got.col, ref.col)
    assert np.array_equal(got.cost.view(np.int64), ref.cost.view(np.int64))
    assert np.array_equal(got.wgt, ref.wgt)


def test_rip_partition_bitexact(dev):
    banner("greedy partition on the GPU row inner-product graph, cd3d-16 K=8")
    p = workloads.small_config2(N=16, K=8)
    g = bc.rip_graph(p.n, p.A.rowptr, p.A.col, p.A.val)
    part = bc.bc_partition_greedy(g, p.K)
    ref = greedy_partition(oracle_rip(p.A), p.K)
    assert np.array_equal(part, ref)


# ------------------------------------------------------------ projections

PROJ_CASES = {
    # name: (problem maker, K, opts)
    "cd2d-32-K4-dense": (workloads.config1, 4, {"projection": bc.BC_PROJ_DENSE_CHOL}),
    "st27-8-K5-dense": (lambda: workloads.small_config5(N=8, K=5), 5,
                        {"projection": bc.BC_PROJ_DENSE_CHOL}),
    "cd3d-10-K3-dense-ragged": (lambda: workloads.small_config2(N=10, K=3), 3,
                                {"projection": bc.BC_PROJ_DENSE_CHOL}),
    "cd2d-32-K4-band": (workloads.config1, 4, {"projection": bc.BC_PROJ_BAND_CHOL}),
    "cd2d-45-K7-band-ragged": (lambda: workloads.small_config4(nsys=1, smin=45, smax=45)[0], 7,
                               {"projection": bc.BC_PROJ_BAND_CHOL}),
    "cd3d-8-K3-band": (lambda: workloads.small_config2(N=8, K=3), 3,
                       {"projection": bc.BC_PROJ_BAND_CHOL}),
    "st27-6-K4-band": (lambda: workloads.small_config5(N=6, K=4), 4,
                       {"projection": bc.BC_PROJ_BAND_CHOL}),
    "cd3d-12-K4-inner": (lambda: workloads.small_config2(N=12, K=4), 4,
                         {"projection": bc.BC_PROJ_INNER_CG, "inner_tol": 1e-13}),
    "powerlaw-3000-K3-inner": (lambda: workloads.small_config3(n=3000, K=3), 3,
                               {"projection": bc.BC_PROJ_INNER_CG, "inner_tol": 1e-13}),
}


@pytest.mark.parametrize("name", sorted(PROJ_CASES))
def test_project_fp64(dev, name):
    banner("bc_project " + name)
    maker, K, opts = PROJ_CASES[name]
    p = maker()
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, K))
    B = BlockProjections(p.A.to_scipy(), part, K)
    rng = np.random.default_rng(7)
    solver = bc.BlockCimmino(p.A, part, K, **opts)
    try:
        for _ in range(2):
            v = rng.standard_normal(p.n)
            Hv = solver.project(to_dev(v, dev)).cpu().numpy()
            bar = 1e-9 if opts.get("projection") == bc.BC_PROJ_INNER_CG else 1e-10
            assert rel(Hv, B.H(v)) <= bar
    finally:
        solver.close()


# ------------------------------------------------------------------ solves

def _oracle_iters_and_x(p, part, K, tol, **kw):
    res = block_cimmino_cg(p.A.to_scipy(), p.f, part, K, tol=tol, **kw)
    return res


def _check_solve(dev, p, part, K, tol=1e-10, **opts):
    ref = _oracle_iters_and_x(p, part, K, tol)
    solver = bc.BlockCimmino(p.A, part, K, **opts)
    try:
        f = to_dev(p.f, dev)
        x, st = solver.solve(f, tol=tol, maxit=10000)
        assert st.status == bc.BC_OK
        assert st.rel_residual <= tol * (1 + 1e-6)
        counts_match(st.iterations, ref.iterations, lambda t: ref.history[t], tol)
        # same iteration count, compare iterates
        x2, st2 = solver.solve(f, tol=0.0, maxit=ref.iterations)
        assert st2.iterations == ref.iterations
        err = rel(x2.cpu().numpy(), ref.x)
        print("iters gpu=%d oracle=%d rel_err=%.3e" % (st.iterations, ref.iterations, err))
        assert err <= 1e-8
        return st, ref
    finally:
        solver.close()


def test_solve_config1(dev):
    banner("bc_solve cd2d-32 K=4 dense FP64")
    p = workloads.config1()
    _check_solve(dev, p, p.part(), p.K, projection=bc.BC_PROJ_DENSE_CHOL)


def test_solve_st27_dense(dev):
    banner("bc_solve st27-10 K=6 dense FP64")
    p = workloads.small_config5(N=10, K=6)
    _check_solve(dev, p, p.part(), p.K, projection=bc.BC_PROJ_DENSE_CHOL)


def test_solve_st27_dense_large_blocks(dev):
    banner("bc_solve st27-17 K=2 dense FP64, blocks of 2456 rows (row-owned sweep: one "
           "workgroup per CU)")
    p = workloads.small_config5(N=17, K=2)
    _check_solve(dev, p, p.part(), p.K, projection=bc.BC_PROJ_DENSE_CHOL)


@pytest.mark.parametrize("case", ["cd2d-32-K4", "cd2d-70-K8", "st27-8-K8"])
def test_solve_band(dev, case):
    banner("bc_solve %s banded Cholesky FP64" % case)
    if case == "cd2d-32-K4":
        p = workloads.config1()
    elif case == "cd2d-70-K8":
        p = workloads.small_config4(nsys=1, smin=70, smax=70)[0]
    else:
        p = workloads.small_config5(N=8, K=8)
    _check_solve(dev, p, p.part(), p.K, projection=bc.BC_PROJ_BAND_CHOL)


def test_auto_picks_band_for_slabs(dev):
    banner("BC_PROJ_AUTO on cd2d-96 K=8: every block banded, half-bandwidth ~ 2 * 12 lines")
    p = workloads.small_config4(nsys=1, smin=96, smax=96)[0]
    solver = bc.BlockCimmino(p.A, p.part(), p.K)
    try:
        kind, bw = solver.block_info()
        assert np.all(kind == bc.KIND_BAND)
        assert np.all((bw >= 12) & (bw <= 2 * 12 + 4))
    finally:
        solver.close()


def test_band_rejects_wide_blocks(dev):
    banner("BC_PROJ_BAND_CHOL on st27-10 K=1: no band within 127, BC_ERR_INVALID")
    p = workloads.small_config5(N=10, K=1)
    with pytest.raises(bc.BCError) as ei:
        bc.BlockCimmino(p.A, np.zeros(p.n, dtype=np.int32), 1, projection=bc.BC_PROJ_BAND_CHOL)
    assert ei.value.status == bc.BC_ERR_INVALID


def test_band_singular_block_detected(dev):
    banner("duplicate row inside a banded block: singular block")
    A = workloads.cd2d(6).to_scipy().tolil()
    A[1] = A[0]
    A = Csr.from_scipy(A.tocsr())
    part = np.zeros(A.n, dtype=np.int32)
    part[18:] = 1
    with pytest.raises(bc.BCError) as ei:
        bc.BlockCimmino(A, part, 2, projection=bc.BC_PROJ_BAND_CHOL)
    assert ei.value.status == bc.BC_ERR_SINGULAR_BLOCK


def test_solve_inner_cg_rip_partition(dev):
    banner("bc_solve cd3d-12 K=4 greedy-rip, inner CG FP64")
    p = workloads.small_config2(N=12, K=4)
    g = bc.rip_graph(p.n, p.A.rowptr, p.A.col, p.A.val)
    part = bc.bc_partition_greedy(g, p.K)
    _check_solve(dev, p, part, p.K, projection=bc.BC_PROJ_INNER_CG, inner_tol=1e-14)


@pytest.mark.parametrize("groups", [2, 4])
def test_solve_inner_cg_groups(dev, groups):
    banner("bc_solve cd3d-16 K=4 inner CG, %d workgroups per block" % groups)
    p = workloads.small_config2(N=16, K=4)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, p.K))
    _check_solve(dev, p, part, p.K, projection=bc.BC_PROJ_INNER_CG, inner_tol=1e-14,
                 inner_groups=groups)


def test_solve_batched(dev):
    banner("bc_solve_batched 6 systems cd2d sides 8..40, K=8")
    probs = workloads.small_config4()
    solver = bc.BlockCimminoBatched([(q.A, q.part(), q.K) for q in probs])
    try:
        f = to_dev(np.concatenate([q.f for q in probs]), dev)
        x, sts = solver.solve(f, tol=1e-10)
        xs = np.split(x.cpu().numpy(), np.cumsum([q.n for q in probs])[:-1])
        for q, st, xg in zip(probs, sts, xs):
            ref = block_cimmino_cg(q.A.to_scipy(), q.f, q.part(), q.K, tol=1e-10)
            assert st.status == bc.BC_OK
            assert st.rel_residual <= 1e-10 * (1 + 1e-6)
            # iterates compared only at equal counts
            if counts_match(st.iterations, ref.iterations, lambda t: ref.history[t], 1e-10):
                assert rel(xg, ref.x) <= 1e-8
    finally:
        solver.close()


def test_solve_deterministic(dev):
    banner("determinism: two solves give identical bits")
    p = workloads.small_config2(N=12, K=4)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, p.K))
    solver = bc.BlockCimmino(p.A, part, p.K, projection=bc.BC_PROJ_INNER_CG)
    try:
        f = to_dev(p.f, dev)
        x1, s1 = solver.solve(f)
        x2, s2 = solver.solve(f)
        assert s1.iterations == s2.iterations
        assert torch.equal(x1, x2)
    finally:
        solver.close()


# ----------------------------------------------------------------- edge cases

def test_single_block_one_iteration(dev):
    banner("K=1: H = I, one iteration")
    p = workloads.small_config5(N=8, K=1)
    part = np.zeros(p.n, dtype=np.int32)
    solver = bc.BlockCimmino(p.A, part, 1)
    try:
        x, st = solver.solve(to_dev(p.f, dev))
        assert st.iterations == 1 and st.status == bc.BC_OK
        assert rel(x.cpu().numpy(), p.xstar) <= 1e-10
    finally:
        solver.close()


def test_orthogonal_blocks_one_iteration(dev):
    banner("block-diagonal A aligned with the partition: one iteration")
    mats = [workloads.cd2d(s) for s in (5, 7, 6)]
    A = Csr.from_scipy(sp.block_diag([m.to_scipy() for m in mats], format="csr"))
    part = np.repeat(np.arange(3), [25, 49, 36]).astype(np.int32)
    xs = np.random.default_rng(3).standard_normal(A.n)
    f = A.to_scipy() @ xs
    solver = bc.BlockCimmino(A, part, 3)
    try:
        x, st = solver.solve(to_dev(f, dev))
        assert st.iterations == 1
        assert rel(x.cpu().numpy(), xs) <= 1e-10
    finally:
        solver.close()


def test_one_row_blocks(dev):
    banner("K = n: 1x1 blocks (plain Cimmino rows)")
    p = workloads.small_config2(N=4, K=64)
    part = np.arange(p.n, dtype=np.int32)
    _check_solve(dev, p, part, p.n)


def test_singular_block_detected(dev):
    banner("duplicate row inside a block: singular block")
    A = workloads.cd2d(6).to_scipy().tolil()
    A[1] = A[0]
    A = Csr.from_scipy(A.tocsr())
    part = np.zeros(A.n, dtype=np.int32)
    part[18:] = 1
    with pytest.raises(bc.BCError) as ei:
        bc.BlockCimmino(A, part, 2)
    assert ei.value.status == bc.BC_ERR_SINGULAR_BLOCK


def test_maxit_zero_rhs_and_exact_start(dev):
    banner("maxit reached, zero right-hand side, exact start")
    p = workloads.config1()
    solver = bc.BlockCimmino(p.A, p.part(), p.K)
    try:
        f = to_dev(p.f, dev)
        x, st = solver.solve(f, maxit=3)
        assert st.status == bc.BC_NOT_CONVERGED and st.iterations == 3
        ref = block_cimmino_cg(p.A.to_scipy(), p.f, p.part(), p.K, tol=0, maxit=3)
        assert rel(x.cpu().numpy(), ref.x) <= 1e-10
        x, st = solver.solve(torch.zeros_like(f))
        assert st.iterations == 0 and st.status == bc.BC_OK
        assert torch.count_nonzero(x) == 0
        x, st = solver.solve(f, x0=to_dev(p.xstar, dev))
        assert st.iterations == 0
    finally:
        solver.close()


def test_backward_error_stop_rule(dev):
    banner("paper stop rule: normwise backward error < 1e-10")
    p = workloads.config1()
    ref = block_cimmino_cg(p.A.to_scipy(), p.f, p.part(), p.K, tol=1e-10, stop="backward")
    solver = bc.BlockCimmino(p.A, p.part(), p.K, stop_rule=bc.BC_STOP_BACKWARD_ERR)
    try:
        x, st = solver.solve(to_dev(p.f, dev), tol=1e-10)
        assert st.status == bc.BC_OK
        A = p.A.to_scipy()

        def gamma_at(t):
            r = block_cimmino_cg(A, p.f, p.part(), p.K, tol=0.0, maxit=t)
            return backward_error(A, r.x, p.f)
        counts_match(st.iterations, ref.iterations, gamma_at, 1e-10)
        assert st.backward_err < 1e-10
    finally:
        solver.close()


def test_mixed_precision_reaches_tolerance(dev):
    banner("mixed precision cd2d-32 K=4 dense FP32 applies, FP64 outer")
    p = workloads.config1()
    ref = block_cimmino_cg(p.A.to_scipy(), p.f, p.part(), p.K, tol=1e-10)
    solver = bc.BlockCimmino(p.A, p.part(), p.K, precision=bc.BC_MIXED,
                             projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        x, st = solver.solve(to_dev(p.f, dev), tol=1e-10, maxit=2000)
        err = rel(x.cpu().numpy(), ref.x)
        print("mixed: iters=%d (oracle %d) rel_res=%.2e err_vs_oracle=%.2e"
              % (st.iterations, ref.iterations, st.rel_residual, err))
        assert st.status == bc.BC_OK and st.rel_residual <= 1e-10 * (1 + 1e-6)
        assert err <= 1e-6
    finally:
        solver.close()


MIXED_CASES = {
    # name: (problem maker, K, opts)
    "powerlaw-6000-K4-mixed-inner": (lambda: workloads.small_config3(n=6000, K=4), 4,
                                     {"projection": bc.BC_PROJ_INNER_CG, "precision": bc.BC_MIXED}),
    "st27-10-K6-fp32-dense-applies": (lambda: workloads.small_config5(N=10, K=6), 6,
                                      {"projection": bc.BC_PROJ_DENSE_CHOL,
                                       "precision": bc.BC_MIXED_PROJ}),
    "cd3d-12-K4-inner-fp32-values": (lambda: workloads.small_config2(N=12, K=4), 4,
                                     {"projection": bc.BC_PROJ_INNER_CG,
                                      "precision": bc.BC_MIXED_PROJ}),
    "cd2d-90-K8-fp32-band": (lambda: workloads.small_config4(nsys=1, smin=90, smax=90)[0], 8,
                             {"projection": bc.BC_PROJ_BAND_CHOL, "precision": bc.BC_MIXED}),
}


@pytest.mark.parametrize("name", sorted(MIXED_CASES))
def test_mixed_precision_modes(dev, name):
    banner("mixed precision " + name)
    maker, K, opts = MIXED_CASES[name]
    p = maker()
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, K))
    ref = block_cimmino_cg(p.A.to_scipy(), p.f, part, K, tol=1e-10)
    solver = bc.BlockCimmino(p.A, part, K, **opts)
    try:
        x, st = solver.solve(to_dev(p.f, dev), tol=1e-10, maxit=3000)
        err = rel(x.cpu().numpy(), ref.x)
        print("%s: iters=%d (oracle %d) rel_res=%.2e err_vs_oracle=%.2e replacements=%d"
              % (name, st.iterations, ref.iterations, st.rel_residual, err, st.replacements))
        assert st.status == bc.BC_OK
        assert st.rel_residual <= 1e-10 * (1 + 1e-6)
        assert err <= 1e-6
    finally:
        solver.close()


def test_batched_mixed(dev):
    banner("bc_solve_batched 6 systems, mixed precision")
    probs = workloads.small_config4()
    solver = bc.BlockCimminoBatched([(q.A, q.part(), q.K) for q in probs], precision=bc.BC_MIXED)
    try:
        f = to_dev(np.concatenate([q.f for q in probs]), dev)
        x, sts = solver.solve(f, tol=1e-10, maxit=3000)
        xs = np.split(x.cpu().numpy(), np.cumsum([q.n for q in probs])[:-1])
        for q, st, xg in zip(probs, sts, xs):
            assert st.status == bc.BC_OK and st.rel_residual <= 1e-10 * (1 + 1e-6)
            assert rel(xg, q.xstar) <= 1e-6
    finally:
        solver.close()


def test_batched_band_mixed(dev):
    banner("bc_solve_batched 5 systems cd2d sides 40..130, K=8, banded FP32 applies, FP64 outer")
    probs = workloads.small_config4(nsys=5, smin=40, smax=130)
    solver = bc.BlockCimminoBatched([(q.A, q.part(), q.K) for q in probs],
                                    precision=bc.BC_MIXED_PROJ, projection=bc.BC_PROJ_BAND_CHOL)
    try:
        f = to_dev(np.concatenate([q.f for q in probs]), dev)
        x, sts = solver.solve(f, tol=1e-10, maxit=5000)
        xs = np.split(x.cpu().numpy(), np.cumsum([q.n for q in probs])[:-1])
        for q, st, xg in zip(probs, sts, xs):
            print("%s: iters=%d rel_res=%.2e err=%.2e" % (q.name, st.iterations, st.rel_residual,
                                                         rel(xg, q.xstar)))
            assert st.status == bc.BC_OK and st.rel_residual <= 1e-10 * (1 + 1e-6)
            assert rel(xg, q.xstar) <= 1e-6
    finally:
        solver.close()


# ------------------------------------------------- graphs and autotuning

@pytest.mark.parametrize("case", ["band-fp64", "dense-fp32"])
def test_graph_replays_match_stream_launches(dev, case):
    banner("captured iteration groups vs plain launches (%s), three solves each" % case)
    p = workloads.small_config4(nsys=1, smin=60, smax=60)[0]
    if case == "band-fp64":
        opts = {"projection": bc.BC_PROJ_BAND_CHOL}
    else:
        opts = {"projection": bc.BC_PROJ_DENSE_CHOL, "precision": bc.BC_MIXED_PROJ}
    eager = bc.BlockCimmino(p.A, p.part(), p.K, use_graph=0, **opts)
    graph = bc.BlockCimmino(p.A, p.part(), p.K, use_graph=1, **opts)
    try:
        rng = np.random.default_rng(11)
        for k in range(3):
            f = to_dev(p.f if k == 0 else rng.standard_normal(p.n), dev)
            x1, s1 = eager.solve(f, tol=1e-10)
            x2, s2 = graph.solve(f, tol=1e-10)
            torch.cuda.synchronize()
            assert s1.status == bc.BC_OK and s2.status == bc.BC_OK
            assert s1.iterations == s2.iterations
            assert torch.equal(x1, x2), "replay %d differs" % k
    finally:
        eager.close()
        graph.close()


def test_graph_batched_mixed_matches_stream_launches(dev):
    banner("captured iteration groups, batched banded FP32 projections, vs plain launches")
    probs = workloads.small_config4(nsys=4, smin=30, smax=90)
    mats = [(q.A, q.part(), q.K) for q in probs]
    opts = {"projection": bc.BC_PROJ_BAND_CHOL, "precision": bc.BC_MIXED_PROJ}
    eager = bc.BlockCimminoBatched(mats, use_graph=0, **opts)
    graph = bc.BlockCimminoBatched(mats, use_graph=1, **opts)
    try:
        f = to_dev(np.concatenate([q.f for q in probs]), dev)
        for _ in range(2):
            x1, s1 = eager.solve(f, tol=1e-10, maxit=5000)
            x2, s2 = graph.solve(f, tol=1e-10, maxit=5000)
            assert [s.iterations for s in s1] == [s.iterations for s in s2]
            assert all(s.status == bc.BC_OK for s in s2)
            assert torch.equal(x1, x2)
    finally:
        eager.close()
        graph.close()


def test_autotuned_lanes_are_reproducible(dev):
    banner("sparse-product lane autotuning: valid choice, same result when fixed explicitly")
    p = workloads.small_config2(N=16, K=4)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, p.K))
    tuned = bc.BlockCimmino(p.A, part, p.K, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        la, lt = bc.bc_schedule(tuned.ctx)
        assert la in (-1, 1, 2, 4, 8, 16, 32, 64) and lt in (-1, 1, 2, 4, 8, 16, 32, 64)
        again = bc.BlockCimmino(p.A, part, p.K, projection=bc.BC_PROJ_DENSE_CHOL)
        assert bc.bc_schedule(again.ctx) == (la, lt)
        again.close()
        f = to_dev(p.f, dev)
        x1, s1 = tuned.solve(f)
        if la == lt:
            fixed = bc.BlockCimmino(p.A, part, p.K, projection=bc.BC_PROJ_DENSE_CHOL,
                                    spmv_lanes=la)
            x2, s2 = fixed.solve(f)
            fixed.close()
            assert s1.iterations == s2.iterations and torch.equal(x1, x2)
    finally:
        tuned.close()


SELL_CASES = {
    # name: (systems, K per system, extra options)
    "cd3d-10-ragged-fp64": (lambda: [workloads.small_config2(N=10, K=3)], 3, {}),
    "cd3d-10-ragged-fp32": (lambda: [workloads.small_config2(N=10, K=3)], 3,
                            {"precision": bc.BC_MIXED}),
    "powerlaw-3000-padded": (lambda: [workloads.small_config3(n=3000, K=3)], 3, {}),
    "batch6-cd2d-ragged": (lambda: workloads.small_config4(nsys=6, smin=8, smax=40), 4, {}),
}


@pytest.mark.parametrize("name", sorted(SELL_CASES))
def test_sliced_ell_products_match_csr(dev, name):
    banner("sliced-ELL sparse products = one-lane CSR products (bitwise), solves agree: " + name)
    maker, K, extra = SELL_CASES[name]
    probs = maker()
    systems = [(q.A, workloads.blocks_to_part(workloads.contiguous_blocks(q.n, K)), K)
               for q in probs]
    opts = dict(projection=bc.BC_PROJ_DENSE_CHOL, **extra)

    def make(lanes):
        if len(systems) == 1:
            A, part, _ = systems[0]
            return bc.BlockCimmino(A, part, K, spmv_lanes=lanes, **opts)
        return bc.BlockCimminoBatched(systems, spmv_lanes=lanes, **opts)

    sell, csr = make(-1), make(1)
    try:
        assert bc.bc_schedule(sell.ctx) == (-1, -1) and bc.bc_schedule(csr.ctx) == (1, 1)
        n = sum(q.n for q in probs)
        rng = np.random.default_rng(11)
        for _ in range(2):
            v = to_dev(rng.standard_normal(n), dev)
            assert torch.equal(sell.project(v), csr.project(v))
        f = to_dev(np.concatenate([q.f for q in probs]), dev)
        x1, s1 = sell.solve(f, tol=1e-10, maxit=3000)
        x2, s2 = csr.solve(f, tol=1e-10, maxit=3000)
        s1 = s1 if isinstance(s1, list) else [s1]
        s2 = s2 if isinstance(s2, list) else [s2]
        # the tile reductions (p.psi, ||s||^2) associate differently (one row
        # per thread here, several rows per thread in the CSR kernels), so
        # the solves agree to rounding, not bit for bit
        assert all(a.status == bc.BC_OK and a.rel_residual <= 1e-10 * (1 + 1e-6) for a in s1)
        same = True
        for q, a, b in zip(probs, s1, s2):
            hist = lambda t, q=q: block_cimmino_cg(q.A.to_scipy(), q.f, q.part(), q.K,
                                                   tol=1e-10).history[t]
            same = counts_match(a.iterations, b.iterations, hist, 1e-10, q.name) and same
        if same:
            assert rel(x1.cpu().numpy(), x2.cpu().numpy()) <= 1e-9
    finally:
        sell.close()
        csr.close()
