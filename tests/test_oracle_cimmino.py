"""Pins of the oracle's Algorithm 2 (CG-accelerated block Cimmino).

P1: the oracle's solution agrees with a direct dense/sparse solve.
P4: K = 1 gives H = I, and so do mutually orthogonal block rows
    (A_i A_j^T = 0): CG then stops after exactly one iteration with
    x^(1) = A^{-1} f (Section 1.2: off-diagonal blocks of eq. (HQR) vanish).
P6: the H-norm of the error decreases monotonically and respects the
    Chebyshev bound 2((sqrt(k)-1)/(sqrt(k)+1))^t of Section 1.2, with
    ||y||_H = sqrt(y^T H y).
Also: the normwise backward error of eq. (stopping) on a hand-computed case,
the paper's stop rule, and Algorithm 1 (plain block Cimmino).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import (block_cimmino_cg, block_cimmino_plain, backward_error, BlockProjections,
                    OK, NOT_CONVERGED)
from tests.test_oracle_projection import rand_sparse_nonsing, rand_part


@pytest.mark.parametrize("seed,n,K", [(0, 60, 3), (1, 120, 5), (2, 200, 7)])
def test_solution_matches_direct_solve(seed, n, K):
    A = rand_sparse_nonsing(n, 0.05, seed, dominance=1.2)
    x_true = np.random.default_rng(seed).standard_normal(n)
    f = A @ x_true
    res = block_cimmino_cg(A, f, rand_part(n, K, seed), K, tol=1e-14, maxit=2000)
    assert res.status == OK
    x_ref = np.linalg.solve(A.toarray(), f)
    assert np.linalg.norm(res.x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    assert res.rel_residual <= 1e-14


def test_config1_matches_sparse_direct():
    p = workloads.config1()
    A = p.A.to_scipy()
    res = block_cimmino_cg(A, p.f, p.part(), p.K, tol=1e-10)
    assert res.status == OK and 0 < res.iterations < 1024
    x_ref = spla.spsolve(A.tocsc(), p.f)
    assert np.linalg.norm(res.x - x_ref) <= 1e-7 * np.linalg.norm(x_ref)
    assert res.rel_residual <= 1e-10
    assert res.history[-2] > 1e-10  # stopped at the first iterate below tol


def test_single_block_one_iteration():
    A = rand_sparse_nonsing(50, 0.1, 11)
    f = A @ np.random.default_rng(11).standard_normal(50)
    res = block_cimmino_cg(A, f, np.zeros(50, dtype=int), 1, tol=1e-10)
    assert res.iterations == 1 and res.status == OK
    assert np.allclose(res.x, np.linalg.solve(A.toarray(), f), rtol=0,
                       atol=1e-12 * np.linalg.norm(res.x))


def test_orthogonal_block_rows_one_iteration():
    rng = np.random.default_rng(12)
    # block-diagonal A aligned with the partition: disjoint column supports
    blocks = [rand_sparse_nonsing(m, 0.3, 20 + m) for m in (7, 11, 5, 9)]
    A = sp.block_diag(blocks, format="csr")
    n = A.shape[0]
    part = np.repeat(np.arange(4), [7, 11, 5, 9])
    perm = rng.permutation(n)               # scatter the rows: blocks are not contiguous
    A, part = A[perm], part[perm]
    f = A @ rng.standard_normal(n)
    res = block_cimmino_cg(A, f, part, 4, tol=1e-10)
    assert res.iterations == 1
    # rows of an orthogonal matrix, any partition
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    Aq = sp.csr_matrix(Q * rng.uniform(0.5, 2.0, (40, 1)))
    fq = Aq @ rng.standard_normal(40)
    res = block_cimmino_cg(Aq, fq, rand_part(40, 6, 3), 6, tol=1e-10)
    assert res.iterations == 1


def test_non_orthogonal_needs_more_iterations():
    p = workloads.config1()
    res = block_cimmino_cg(p.A.to_scipy(), p.f, p.part(), p.K, tol=1e-10)
    assert res.iterations > 1


@pytest.mark.parametrize("seed,K", [(13, 4), (14, 6)])
def test_H_norm_error_monotone_and_bounded(seed, K):
    n = 80
    A = rand_sparse_nonsing(n, 0.06, seed, dominance=0.8)
    xstar = np.random.default_rng(seed).standard_normal(n)
    f = A @ xstar
    part = rand_part(n, K, seed)
    B = BlockProjections(A, part, K, backend="qr")
    ev = np.linalg.eigvalsh(B.dense_H())
    kappa = ev.max() / ev.min()
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    res = block_cimmino_cg(A, f, part, K, tol=1e-13, proj=B, xstar=xstar)
    e = np.array(res.herr)
    assert res.status == OK and res.iterations >= 3
    assert np.all(e[1:] <= e[:-1] * (1 + 1e-9) + 1e-13 * e[0])
    t = np.arange(e.size)
    assert np.all(e <= 2 * rho ** t * e[0] * (1 + 1e-9) + 1e-12 * e[0])


def test_backward_error_closed_form():
    A = sp.csr_matrix(np.array([[2.0, -1.0], [0.5, 3.0]]))
    x = np.array([1.0, -2.0])
    f = np.array([4.5, -5.0])
    # A x - f = (4 - 4.5, -5.5 + 5) = (-0.5, -0.5); ||A||_inf = 3.5; ||x||_1 = 3; ||f||_inf = 5
    assert backward_error(A, x, f) == pytest.approx(0.5 / (3.5 * 3 + 5), rel=1e-15)


def test_paper_stop_rule_and_status():
    p = workloads.config1()
    A = p.A.to_scipy()
    res = block_cimmino_cg(A, p.f, p.part(), p.K, tol=1e-10, stop="backward")
    assert res.status == OK and res.backward_err < 1e-10
    res_rel = block_cimmino_cg(A, p.f, p.part(), p.K, tol=1e-10)
    assert res.iterations <= res_rel.iterations  # gamma is the looser measure here
    res1 = block_cimmino_cg(A, p.f, p.part(), p.K, tol=1e-10, maxit=1)
    assert res1.status == NOT_CONVERGED and res1.iterations == 1


def test_zero_rhs_and_exact_start():
    p = workloads.config1()
    A = p.A.to_scipy()
    res = block_cimmino_cg(A, np.zeros(p.n), p.part(), p.K)
    assert res.iterations == 0 and np.all(res.x == 0)
    res = block_cimmino_cg(A, p.f, p.part(), p.K, x0=p.xstar)
    assert res.iterations == 0


def test_plain_block_cimmino():
    # one block, omega = 1: a single step is the exact solution
    A = rand_sparse_nonsing(30, 0.2, 15)
    f = A @ np.ones(30)
    res = block_cimmino_plain(A, f, np.zeros(30, dtype=int), 1, omega=1.0, tol=1e-12)
    assert res.iterations == 1
    # several blocks: converges for 0 < omega < 2 / lambda_max(H), slower than CG
    p = workloads.config1()
    Am = p.A.to_scipy()
    B = BlockProjections(Am, p.part(), p.K)
    res_p = block_cimmino_plain(Am, p.f, p.part(), p.K, omega=1.0, tol=1e-6, maxit=20000, proj=B)
    res_c = block_cimmino_cg(Am, p.f, p.part(), p.K, tol=1e-6, proj=B)
    assert res_p.status == OK and res_p.iterations > res_c.iterations


@pytest.mark.parametrize("omega", [0.7, 1.3])
def test_plain_block_cimmino_error_recursion(omega):
    # eq. (iterscheme): e^(t) = (I - omega H)^t e^(0), with H = sum_i pinv(A_i) A_i
    # formed here from numpy's SVD-based pseudo-inverse of each dense block
    # (independent of the oracle's QR / seminormal-equation projections)
    n, K, t = 50, 4, 6
    A = rand_sparse_nonsing(n, 0.08, 21)
    part = rand_part(n, K, 21)
    x_true = np.random.default_rng(5).standard_normal(n)
    f = A @ x_true
    Ad = A.toarray()
    H = np.zeros((n, n))
    for i in range(K):
        Ai = Ad[part == i]
        H += np.linalg.pinv(Ai) @ Ai
    x0 = np.random.default_rng(6).standard_normal(n)
    e = x0 - x_true
    Qm = np.eye(n) - omega * H
    for _ in range(t):
        e = Qm @ e
    res = block_cimmino_plain(A, f, part, K, omega=omega, x0=x0, tol=0.0, maxit=t)
    assert res.iterations == t
    assert np.linalg.norm(res.x - (x_true + e)) <= 1e-10 * np.linalg.norm(x_true)
