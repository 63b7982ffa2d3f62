"""Algorithm 1 (plain block Cimmino, ``bc_cimmino``) and the Lanczos spectrum
tool on the GPU, against the oracle (needs an MI355X).

Bars: the oracle's iteration count (a difference of one only as a near-tie of
the stop decision) and, at equal count, the iterate within 1e-10 relative (FP64
dense projections); K = 1 gives H = I, one step with omega = 1 solves the system;
the extreme Ritz values of H from products by ``bc_project`` within 1e-9 of
numpy's eigenvalues of the oracle's dense H.
"""
import numpy as np
import pytest

import paper_1710_07769_amd as bc
import workloads
from _bars import counts_match
from oracle import BlockProjections, block_cimmino_plain
from paper_1710_07769_amd.spectrum import spectrum_of

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


def st27(N, K):
    p = workloads.small_config5(N=N, K=K)
    return p, workloads.blocks_to_part(workloads.contiguous_blocks(p.n, K))


def check_against_oracle(dev, solver, p, part, K, omega, tol=1e-10):
    A = p.A.to_scipy()
    B = BlockProjections(A, part, K)
    ref = block_cimmino_plain(A, p.f, part, K, omega=omega, tol=tol, maxit=5000, proj=B)
    f = to_dev(p.f, dev)
    x, sts = solver.cimmino(f, omega, tol=tol, maxit=5000)
    st = sts[0]
    print("omega %.3f: iterations gpu=%d oracle=%d rel_res=%.2e"
          % (omega, st.iterations, ref.iterations, st.rel_residual))
    assert st.status == bc.BC_OK and st.rel_residual <= tol * (1 + 1e-6)
    counts_match(st.iterations, ref.iterations, lambda t: ref.history[t], tol)
    # equal count: both run exactly the oracle's number of updates
    x2, sts2 = solver.cimmino(f, omega, tol=0.0, maxit=ref.iterations)
    assert sts2[0].iterations == ref.iterations and sts2[0].status == bc.BC_NOT_CONVERGED
    assert rel(x2.cpu().numpy(), ref.x) <= 1e-10


@pytest.mark.parametrize("omega", [1.0, 0.8, 1.2])
def test_alg1_st27_dense(dev, omega):
    banner("Algorithm 1, 27-point 10^3, K=6, dense projections, omega=%.1f" % omega)
    p, part = st27(10, 6)
    solver = bc.BlockCimmino(p.A, part, 6, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        check_against_oracle(dev, solver, p, part, 6, omega)
    finally:
        solver.close()


def test_alg1_st27_banded(dev):
    banner("Algorithm 1, 27-point 8^3, K=4, banded projections, omega=1")
    p, part = st27(8, 4)
    solver = bc.BlockCimmino(p.A, part, 4, projection=bc.BC_PROJ_BAND_CHOL)
    try:
        check_against_oracle(dev, solver, p, part, 4, 1.0)
    finally:
        solver.close()


def test_alg1_batched_systems_stop_independently(dev):
    banner("Algorithm 1 on 3 batched 27-point systems (6^3 K=3, 8^3 K=4, 10^3 K=6)")
    cases = [st27(6, 3) + (3,), st27(8, 4) + (4,), st27(10, 6) + (6,)]
    solver = bc.BlockCimminoBatched([(p.A, part, K) for p, part, K in cases],
                                    projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        f = to_dev(np.concatenate([p.f for p, _, _ in cases]), dev)
        x, sts = solver.cimmino(f, 1.0, tol=1e-10, maxit=5000)
        xs = np.split(x.cpu().numpy(), np.cumsum([p.n for p, _, _ in cases])[:-1])
        for (p, part, K), st, xk in zip(cases, sts, xs):
            ref = block_cimmino_plain(p.A.to_scipy(), p.f, part, K, omega=1.0, tol=1e-10,
                                      maxit=5000)
            print("n=%d: iterations gpu=%d oracle=%d" % (p.n, st.iterations, ref.iterations))
            assert st.status == bc.BC_OK
            if counts_match(st.iterations, ref.iterations, lambda t: ref.history[t], 1e-10):
                assert rel(xk, ref.x) <= 1e-8
    finally:
        solver.close()


def test_alg1_single_block_is_one_step(dev):
    banner("Algorithm 1 with K=1 (H = I): one step with omega = 1 gives A^{-1} f")
    p = workloads.small_config5(N=8, K=1)
    part = np.zeros(p.n, dtype=np.int32)
    solver = bc.BlockCimmino(p.A, part, 1, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        f = to_dev(p.f, dev)
        x, sts = solver.cimmino(f, 1.0, tol=1e-10)
        assert sts[0].status == bc.BC_OK and sts[0].iterations == 1
        assert rel(x.cpu().numpy(), p.xstar) <= 1e-10
        # maxit = 0: no update, x = x0 = 0, not converged
        x0, st0 = solver.cimmino(f, 1.0, tol=1e-10, maxit=0)
        assert st0[0].status == bc.BC_NOT_CONVERGED and st0[0].iterations == 0
        assert float(x0.abs().max()) == 0.0
        with pytest.raises(bc.BCError):
            solver.cimmino(f, 0.0)
    finally:
        solver.close()


def test_lanczos_spectrum_through_bc_project(dev):
    banner("Lanczos on H through bc_project: extreme Ritz values = oracle eigenvalues")
    p, part = st27(10, 6)
    ev = np.linalg.eigvalsh(BlockProjections(p.A.to_scipy(), part, 6).dense_H())
    solver = bc.BlockCimmino(p.A, part, 6, projection=bc.BC_PROJ_DENSE_CHOL)
    try:
        sp = spectrum_of(solver.ctx, p.n, steps=150, seed=4)
        print("lambda gpu [%.12f, %.12f] oracle [%.12f, %.12f]"
              % (sp.lambda_min, sp.lambda_max, ev[0], ev[-1]))
        assert abs(sp.lambda_min - ev[0]) <= 1e-9 and abs(sp.lambda_max - ev[-1]) <= 1e-9
    finally:
        solver.close()
