"""bc_solve_noalloc through the C ABI: the same results as bc_solve, bit for
bit, on two calls in a row that share the static scratch, the second on a
smaller system (and a third, on a batch, that the scratch still holds);
a context whose vectors exceed the scratch is refused with BC_ERR_INVALID."""
import numpy as np
import pytest

import paper_1710_07769_amd as bc
import workloads

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


def _same_as_solve(dev, probs, **opts):
    batched = len(probs) > 1
    if batched:
        solver = bc.BlockCimminoBatched([(q.A, q.part(), q.K) for q in probs], **opts)
    else:
        q = probs[0]
        solver = bc.BlockCimmino(q.A, q.part(), q.K, **opts)
    try:
        f = to_dev(np.concatenate([q.f for q in probs]), dev)
        x_ref = torch.empty_like(f)
        ref = (bc.bc_solve_batched if batched else
               (lambda *a: [bc.bc_solve(*a)]))(solver.ctx, f, None, 1e-10, 10000, x_ref)
        x = torch.full_like(f, np.nan)
        sts = bc.bc_solve_noalloc(solver.ctx, f, None, 1e-10, 10000, x)
        torch.cuda.synchronize()
        assert len(sts) == len(ref)
        for a, b in zip(sts, ref):
            assert a.status == b.status == bc.BC_OK
            assert a.iterations == b.iterations
            assert a.rel_residual == b.rel_residual
        assert np.array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
        return sts
    finally:
        solver.close()


def test_noalloc_two_calls_second_smaller(dev):
    banner("bc_solve_noalloc: cd3d-16 K=4 inner CG (4096 rows), then cd2d-32 K=4 dense "
           "(1024 rows), then a batch of 6 banded systems")
    p = workloads.small_config2(N=16, K=4)
    p.part = lambda p=p: workloads.blocks_to_part(workloads.contiguous_blocks(p.n, p.K))
    _same_as_solve(dev, [p], projection=bc.BC_PROJ_INNER_CG, inner_groups=4)
    _same_as_solve(dev, [workloads.config1()], projection=bc.BC_PROJ_DENSE_CHOL)
    _same_as_solve(dev, workloads.small_config4(), projection=bc.BC_PROJ_BAND_CHOL)


def test_noalloc_refuses_systems_beyond_the_scratch(dev):
    banner("bc_solve_noalloc: 7 vectors of 5e6 rows exceed the 256 MiB scratch")
    n = 5_000_000
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    val = np.ones(n)
    K = 80  # blocks of 62,500 rows: banded (half-bandwidth 0)
    part = (np.arange(n) // (n // K)).astype(np.int32)
    ctx = bc.bc_setup(n, rowptr, col, val, K, part, bc.make_opts())
    try:
        f = torch.ones(n, dtype=torch.float64, device=dev)
        x = torch.empty_like(f)
        with pytest.raises(bc.BCError) as e:
            bc.bc_solve_noalloc(ctx, f, None, 1e-10, 100, x)
        assert e.value.status == bc.BC_ERR_INVALID
        st = bc.bc_solve(ctx, f, None, 1e-10, 100, x)  # the context itself still works
        assert st.status == bc.BC_OK
    finally:
        bc.bc_destroy(ctx)
