"""Pins of the oracle's block CG on H for several right-hand sides.

* With one right-hand side it is Algorithm 2: the same iterates at every
  step and the same iteration count.
* The defining property of block CG: after k steps each column x_j is the
  minimizer of the H-norm error ||x - x*_j||_H over x0_j plus the block Krylov
  space span{R0, H R0, ..., H^{k-1} R0} (all columns of R0 = Xi - H X0).  This
  is checked against that minimizer computed directly from an orthonormal
  basis of the space (a wrong sign or index in alpha or beta, or a lost
  H-conjugacy, breaks it).
* Finite termination: the block Krylov space grows by s dimensions per step,
  so the iteration ends within about n / s steps.
* Repeated and dependent right-hand sides (rank-deficient blocks), a zero
  right-hand side and an exact starting guess.
* The orthonormal basis routine itself.
"""
import numpy as np
import pytest

from oracle import (BlockProjections, block_cimmino_block_cg, block_cimmino_cg,
                    orthonormal_directions, OK, NOT_CONVERGED)
from tests.test_oracle_projection import rand_sparse_nonsing, rand_part


def problem(n, K, seed, s):
    A = rand_sparse_nonsing(n, 0.06, seed, dominance=1.2)
    rng = np.random.default_rng(seed + 100)
    Xs = rng.standard_normal((n, s))
    return A, A @ Xs, Xs, rand_part(n, K, seed)


def test_one_rhs_is_algorithm_2():
    A, F, _, part = problem(80, 4, 1, 1)
    B = BlockProjections(A, part, 4)
    for k in (1, 2, 5, 9):
        cg = block_cimmino_cg(A, F[:, 0], part, 4, tol=0.0, maxit=k, proj=B)
        bcg = block_cimmino_block_cg(A, F, part, 4, tol=0.0, maxit=k, proj=B)
        assert bcg.iterations[0] == k
        assert np.linalg.norm(bcg.X[:, 0] - cg.x) <= 1e-11 * np.linalg.norm(cg.x)
    cg = block_cimmino_cg(A, F[:, 0], part, 4, tol=1e-10, proj=B)
    bcg = block_cimmino_block_cg(A, F, part, 4, tol=1e-10, proj=B)
    assert bcg.status[0] == OK and bcg.iterations[0] == cg.iterations


@pytest.mark.parametrize("seed,s", [(2, 3), (3, 5)])
def test_block_krylov_minimization(seed, s):
    n, K = 60, 5
    A, F, Xs, part = problem(n, K, seed, s)
    B = BlockProjections(A, part, K)
    Hd = B.dense_H()
    X0 = np.random.default_rng(seed + 7).standard_normal((n, s)) * 0.1
    Xi = np.column_stack([B.min_norm_sum(F[:, j]) for j in range(s)])
    R0 = Xi - Hd @ X0
    for k in range(1, 5):
        res = block_cimmino_block_cg(A, F, part, K, X0=X0, tol=0.0, maxit=k, proj=B)
        assert all(res.iterations == k) and all(d == s for d in res.directions)
        # orthonormal basis of span{R0, H R0, ..., H^{k-1} R0}
        blocks = [R0]
        for _ in range(k - 1):
            blocks.append(Hd @ blocks[-1])
        V, _ = np.linalg.qr(np.column_stack(blocks))
        for j in range(s):
            # argmin over x0 + span V of ||x - x*||_H: V^T H V c = V^T (Xi_j - H x0_j)
            c = np.linalg.solve(V.T @ Hd @ V, V.T @ R0[:, j])
            xm = X0[:, j] + V @ c
            err = np.linalg.norm(res.X[:, j] - xm) / np.linalg.norm(xm)
            assert err <= 1e-8, (k, j, err)
    # and the minimizer is strictly better than the first column's own CG
    cg = block_cimmino_cg(A, F[:, 0], part, K, x0=X0[:, 0], tol=0.0, maxit=3, proj=B)
    res = block_cimmino_block_cg(A, F, part, K, X0=X0, tol=0.0, maxit=3, proj=B)

    def herr(x):
        e = x - Xs[:, 0]
        return float(np.sqrt(e @ Hd @ e))
    assert herr(res.X[:, 0]) < herr(cg.x)


def test_finite_termination():
    n, K, s = 48, 4, 6
    A, F, Xs, part = problem(n, K, 4, s)
    res = block_cimmino_block_cg(A, F, part, K, tol=1e-10)
    assert all(res.status == OK)
    assert res.iterations.max() <= n // s + 3
    assert all(res.rel_residual <= 1e-10)
    cg_max = max(block_cimmino_cg(A, F[:, j], part, K, tol=1e-10).iterations for j in range(s))
    assert res.iterations.max() < cg_max


def test_dependent_and_zero_right_hand_sides():
    n, K = 70, 5
    A, F, Xs, part = problem(n, K, 5, 5)
    F[:, 1] = F[:, 0]                    # repeated
    F[:, 3] = 2.0 * F[:, 0] - F[:, 2]    # dependent
    F[:, 4] = 0.0                        # zero
    res = block_cimmino_block_cg(A, F, part, K, tol=1e-10)
    assert res.status[4] == OK and res.iterations[4] == 0 and not res.X[:, 4].any()
    assert all(res.status == OK) and all(res.rel_residual <= 1e-10)
    assert np.array_equal(res.X[:, 0], res.X[:, 1])
    assert max(res.directions) <= 3      # at most 3 independent columns
    xd = np.linalg.solve(A.toarray(), F)
    for j in range(4):
        assert np.linalg.norm(res.X[:, j] - xd[:, j]) <= 1e-7 * np.linalg.norm(xd[:, j])


def test_exact_start_and_maxit():
    n, K = 50, 3
    A, F, Xs, part = problem(n, K, 6, 3)
    res = block_cimmino_block_cg(A, F, part, K, X0=Xs, tol=1e-10)
    assert all(res.status == OK) and all(res.iterations == 0)
    res = block_cimmino_block_cg(A, F, part, K, tol=1e-14, maxit=2)
    assert all(res.status == NOT_CONVERGED) and all(res.iterations == 2)


def test_orthonormal_directions():
    rng = np.random.default_rng(9)
    Z = rng.standard_normal((30, 5)) * np.array([1e3, 1.0, 1e-4, 5.0, 2.0])
    Z[:, 3] = 0.5 * Z[:, 0] - 2.0 * Z[:, 1]   # in the span of the first two
    T, kept = orthonormal_directions(Z)
    assert kept == [0, 1, 2, 4]
    P = Z @ T
    assert np.allclose(P.T @ P, np.eye(4), atol=1e-12)
    # the span is that of the kept columns
    Qk, _ = np.linalg.qr(Z[:, kept])
    assert np.allclose(Qk @ (Qk.T @ P), P, atol=1e-10)
    T0, kept0 = orthonormal_directions(np.zeros((10, 2)))
    assert kept0 == [] and T0.shape == (2, 0)
