"""Pins of the oracle's projections against facts the paper and linear algebra fix.

P2: each P_i is an orthogonal projector onto range(A_i^T) (Section 1: the
    sum of projections P_R(A_i^T)); it does not depend on row scaling or on
    the row order inside a block (Section 2.1, Section 2.2).
P3: H is symmetric positive definite for square nonsingular A (Section 1.1),
    trace(H) = n (trace of a projector is its rank and the ranks add up to n),
    eig(H) lies in (0, K], the spectrum equals that of D^{-1} A A^T with
    D = blockdiag(A_i A_i^T), and a column permutation of A does not change it
    (Section 1.2).
P5: for K = 2 the similar matrix of eq. (HQR) is [[I, M], [M^T, I]] with the
    singular values of M = Q_1^T Q_2 equal to cosines of principal angles, so
    eig(H) = {1 +- cos theta_j} plus ones.
P12: the seminormal-equations backend agrees with the QR backend.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle.projection import QRProjector, CSNEProjector, BlockProjections, SingularBlock


def rand_sparse_nonsing(n, density, seed, dominance=1.5):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, data_rvs=rng.standard_normal).tocsr()
    M = M + sp.diags(dominance * (np.abs(M).sum(axis=1).A1 + 1.0) * rng.choice([-1, 1], n))
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M


def rand_part(n, K, seed):
    rng = np.random.default_rng(seed)
    part = np.concatenate([np.arange(K), rng.integers(0, K, n - K)])
    rng.shuffle(part)
    return part


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_projector_invariants(seed):
    n = 40
    A = rand_sparse_nonsing(n, 0.1, seed)
    rng = np.random.default_rng(100 + seed)
    rows = np.sort(rng.choice(n, 12, replace=False))
    Ai = A[rows]
    P = QRProjector(Ai)
    Pm = np.column_stack([P.project(e) for e in np.eye(n)])
    assert np.allclose(Pm @ Pm, Pm, atol=1e-13)
    assert np.allclose(Pm, Pm.T, atol=1e-13)
    v = rng.standard_normal(n)
    assert np.allclose(Ai @ P.project(v), Ai @ v, rtol=0, atol=1e-12 * np.linalg.norm(Ai @ v))
    assert np.linalg.norm(P.project(v)) <= np.linalg.norm(v) * (1 + 1e-14)
    assert np.isclose(np.trace(Pm), 12, atol=1e-12)
    # min-norm solution: solves A_i d = r and lies in range(A_i^T)
    r = rng.standard_normal(12)
    d = P.min_norm(r)
    assert np.allclose(Ai @ d, r, atol=1e-12 * np.linalg.norm(r) * 100)
    assert np.allclose(P.project(d), d, atol=1e-12 * np.linalg.norm(d))
    # equals the textbook pseudoinverse on the dense block
    assert np.allclose(d, np.linalg.pinv(Ai.toarray()) @ r, atol=1e-11 * np.linalg.norm(d))
    # row scaling and row order inside a block leave P unchanged
    Dsc = sp.diags(rng.uniform(0.1, 10.0, 12))
    perm = rng.permutation(12)
    P2 = QRProjector((Dsc @ Ai)[perm])
    Pm2 = np.column_stack([P2.project(e) for e in np.eye(n)])
    assert np.allclose(Pm, Pm2, atol=1e-12)


def test_singular_block_detected():
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0.0], [2.0, 4.0, 0.0], [0.0, 0.0, 1.0]]))
    with pytest.raises(SingularBlock):
        QRProjector(A[:2])
    with pytest.raises(SingularBlock):
        CSNEProjector(A[:2])


@pytest.mark.parametrize("seed,K", [(3, 3), (4, 5), (5, 8)])
def test_H_spectrum_facts(seed, K):
    n = 48
    A = rand_sparse_nonsing(n, 0.08, seed)
    part = rand_part(n, K, seed)
    B = BlockProjections(A, part, K, backend="qr")
    H = B.dense_H()
    assert np.allclose(H, H.T, atol=1e-13)
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert ev.min() > 0
    assert ev.max() <= K + 1e-12
    assert np.isclose(np.trace(H), n, atol=1e-11)
    # spec(H) = spec(D^{-1} C), C = A A^T, D = blockdiag(A_i A_i^T), rows in block order
    order = np.concatenate(B.rows)
    Ap = A[order].toarray()
    C = Ap @ Ap.T
    D = np.zeros_like(C)
    off = 0
    for rows in B.rows:
        m = rows.size
        D[off:off + m, off:off + m] = C[off:off + m, off:off + m]
        off += m
    ev2 = np.sort(np.linalg.eigvals(np.linalg.solve(D, C)).real)
    assert np.allclose(ev, ev2, atol=1e-10)
    # column permutation does not change the spectrum
    cp = np.random.default_rng(seed).permutation(n)
    Bc = BlockProjections(A[:, cp], part, K, backend="qr")
    ev3 = np.linalg.eigvalsh(Bc.dense_H())
    assert np.allclose(ev, ev3, atol=1e-11)


@pytest.mark.parametrize("seed", [6, 7])
def test_two_block_spectrum_principal_angles(seed):
    n = 30
    A = rand_sparse_nonsing(n, 0.15, seed)
    part = np.zeros(n, dtype=int)
    part[np.random.default_rng(seed).choice(n, 13, replace=False)] = 1
    B = BlockProjections(A, part, 2, backend="qr")
    ev = np.sort(np.linalg.eigvalsh(B.dense_H()))
    A1 = A[B.rows[0]].toarray()
    A2 = A[B.rows[1]].toarray()
    theta = sla.subspace_angles(A1.T, A2.T)
    c = np.cos(theta)
    m1, m2 = B.rows[0].size, B.rows[1].size
    expect = np.sort(np.concatenate([1 + c, 1 - c, np.ones(abs(m1 - m2))]))
    assert np.allclose(ev, expect, atol=1e-12)


@pytest.mark.parametrize("seed", [8, 9])
def test_csne_matches_qr(seed):
    n = 120
    A = rand_sparse_nonsing(n, 0.04, seed)
    part = rand_part(n, 4, seed)
    Bq = BlockProjections(A, part, 4, backend="qr")
    Bc = BlockProjections(A, part, 4, backend="csne")
    Bs = BlockProjections(A, part, 4, backend="csne", dense_max=0)   # sparse LU path
    v = np.random.default_rng(seed).standard_normal(n)
    hq = Bq.H(v)
    assert np.linalg.norm(Bc.H(v) - hq) <= 1e-12 * np.linalg.norm(hq)
    assert np.linalg.norm(Bs.H(v) - hq) <= 1e-12 * np.linalg.norm(hq)
    assert np.linalg.norm(Bc.min_norm_sum(v) - Bq.min_norm_sum(v)) <= 1e-12 * np.linalg.norm(Bq.min_norm_sum(v))


def test_csne_correction_on_ill_conditioned_block():
    """The seminormal equations alone lose about kappa(A_i)^2 * eps; one
    correction step brings the error back to about kappa(A_i) * eps.  A block
    with kappa ~ 1e5 separates the two."""
    rng = np.random.default_rng(21)
    n, m = 30, 6
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, m)))
    Ai = U @ np.diag(np.logspace(0, -5, m)) @ V.T
    P = QRProjector(sp.csr_matrix(Ai))
    C = CSNEProjector(sp.csr_matrix(Ai))
    r = rng.standard_normal(m)
    dq, dc = P.min_norm(r), C.min_norm(r)
    assert np.linalg.norm(dc - dq) <= 1e-9 * np.linalg.norm(dq)
    # without the correction step the error is orders of magnitude larger
    y = C._gsolve(r)
    d0 = C.At @ y
    assert np.linalg.norm(d0 - dq) > 1e3 * np.linalg.norm(dc - dq)
