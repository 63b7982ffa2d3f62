"""Block Cimmino iterations (oracle; test infrastructure).

* :func:`block_cimmino_cg`    - Algorithm 2: classical CG applied to
  H x = xi with xi = sum_i A_i^+ f_i (eq. (cg); the relaxation omega appears
  on both sides and cancels).
* :func:`block_cimmino_plain` - Algorithm 1 / eq. (iterscheme):
  x <- x + omega sum_i A_i^+ (f_i - A_i x).
* :func:`backward_error`      - the normwise backward error gamma of eq.
  (stopping), used by the paper's experiments with threshold 1e-10.
* :func:`block_cimmino_block_cg` - block CG on H X = Xi for several right-hand
  sides at once, with orthonormalized search directions (the stabilized
  block-CG acceleration that Section 3.1 attributes to ABCD Solver for
  multiple right-hand sides; the paper itself uses Algorithm 2).

Conventions taken where the paper is silent:

* An iteration is one application of H inside the loop; x^(0) counts as
  iteration 0.  The stop rule is evaluated once on x^(0) and then after each
  update of x.
* The stop rule uses the true residual s = f - A x, recomputed directly from
  x each iteration.  ``stop="rel2"`` (default) stops when ||s||_2 <= tol ||f||_2;
  ``stop="backward"`` stops when gamma < tol (the paper's rule).
* CG breaks down if p^T H p is not a positive finite number.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .projection import BlockProjections

OK = 0
NOT_CONVERGED = 1
BREAKDOWN = -3


@dataclass
class CimminoResult:
    x: np.ndarray
    iterations: int
    status: int
    rel_residual: float
    backward_err: float
    history: List[float] = field(default_factory=list)   # ||f - A x_t|| / ||f|| per t
    herr: List[float] = field(default_factory=list)      # ||x_t - x*||_H per t if x* given


def backward_error(A, x: np.ndarray, f: np.ndarray) -> float:
    """gamma = ||A x - f||_inf / (||A||_inf ||x||_1 + ||f||_inf)  (eq. (stopping))."""
    A = sp.csr_matrix(A)
    normA = np.abs(A).sum(axis=1).max()
    num = np.abs(A @ x - f).max()
    den = normA * np.abs(x).sum() + np.abs(f).max()
    return float(num / den) if den > 0 else 0.0


def _stop(stop, A, x, s, f, nf, tol):
    if stop == "rel2":
        return np.linalg.norm(s) <= tol * nf
    if stop == "backward":
        return backward_error(A, x, f) < tol
    if stop == "never":
        return False
    raise ValueError(stop)


def block_cimmino_cg(A, f, part, K, x0=None, tol=1e-10, maxit=10000, stop="rel2",
                     backend="auto", proj: Optional[BlockProjections] = None,
                     xstar: Optional[np.ndarray] = None) -> CimminoResult:
    """Classical CG on H x = xi (Algorithm 2)."""
    A = sp.csr_matrix(A)
    f = np.asarray(f, dtype=np.float64)
    n = A.shape[0]
    if proj is None:
        proj = BlockProjections(A, part, K, backend)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    nf = np.linalg.norm(f)
    s = f - A @ x
    hist = [np.linalg.norm(s) / nf if nf > 0 else 0.0]
    herr = []

    def _herr():
        if xstar is not None:
            e = x - xstar
            herr.append(float(np.sqrt(max(e @ proj.H(e), 0.0))))

    _herr()

    def done(t, status):
        rel = np.linalg.norm(s) / nf if nf > 0 else 0.0
        return CimminoResult(x, t, status, float(rel), backward_error(A, x, f), hist, herr)

    if _stop(stop, A, x, s, f, nf, tol) or nf == 0.0:
        return done(0, OK)
    # initial H-residual: xi - H x0 = sum_i A_i^+ (f_i - A_i x0)
    r = proj.min_norm_sum(s)
    p = r.copy()
    rr = r @ r
    for t in range(1, maxit + 1):
        psi = proj.H(p)
        ppsi = p @ psi
        if not (np.isfinite(ppsi) and ppsi > 0.0):
            return done(t - 1, BREAKDOWN)
        alpha = rr / ppsi
        x += alpha * p
        r -= alpha * psi
        s = f - A @ x
        hist.append(np.linalg.norm(s) / nf)
        _herr()
        if _stop(stop, A, x, s, f, nf, tol):
            return done(t, OK)
        rr_new = r @ r
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    return done(maxit, NOT_CONVERGED)


def block_cimmino_plain(A, f, part, K, omega=1.0, x0=None, tol=1e-10, maxit=10000,
                        stop="rel2", backend="auto",
                        proj: Optional[BlockProjections] = None) -> CimminoResult:
    """Algorithm 1: x <- x + omega * sum_i A_i^+ (f_i - A_i x)."""
    A = sp.csr_matrix(A)
    f = np.asarray(f, dtype=np.float64)
    if proj is None:
        proj = BlockProjections(A, part, K, backend)
    x = np.zeros(A.shape[0]) if x0 is None else np.array(x0, dtype=np.float64)
    nf = np.linalg.norm(f)
    s = f - A @ x
    hist = [np.linalg.norm(s) / nf if nf > 0 else 0.0]
    for t in range(0, maxit + 1):
        if _stop(stop, A, x, s, f, nf, tol) or nf == 0.0:
            return CimminoResult(x, t, OK, hist[-1], backward_error(A, x, f), hist)
        if t == maxit:
            break
        x += omega * proj.min_norm_sum(s)
        s = f - A @ x
        hist.append(np.linalg.norm(s) / nf)
    return CimminoResult(x, maxit, NOT_CONVERGED, hist[-1], backward_error(A, x, f), hist)


def orthonormal_directions(Z: np.ndarray, drop: float = 1e-10):
    """Orthonormal basis of the columns of Z (n x a), taken in column order.

    The columns are scaled to unit 2-norm, then a Cholesky factorization of
    their Gram matrix G = Zn^T Zn is formed column by column; a column whose
    pivot (the squared norm of its part orthogonal to the columns kept before
    it) is at most ``drop`` is left out (it lies in their span to within
    sqrt(drop)).  Returns (T, kept): T is a x r with Z T = Zn[:, kept] L^{-T},
    whose columns are orthonormal (L: the r x r Cholesky factor of the kept
    part of G).  Zero columns are always left out."""
    a = Z.shape[1]
    d = np.linalg.norm(Z, axis=0)
    kept = [j for j in range(a) if d[j] > 0.0]
    Zn = Z[:, kept] / d[kept]
    G = Zn.T @ Zn
    L = np.zeros((len(kept), len(kept)))
    keep2 = []
    for q in range(len(kept)):
        r = len(keep2)
        # row of L for column q against the kept columns: L[:r,:r] l = G[keep2, q]
        l = np.zeros(r)
        for i in range(r):
            l[i] = (G[keep2[i], q] - L[i, :i] @ l[:i]) / L[i, i]
        piv = G[q, q] - l @ l
        if piv > drop:
            L[r, :r] = l
            L[r, r] = np.sqrt(piv)
            keep2.append(q)
    r = len(keep2)
    L = L[:r, :r]
    # T = diag(1/d)[:, kept][:, keep2] L^{-T}
    T = np.zeros((a, r))
    Linv_T = np.linalg.inv(L).T if r else np.zeros((0, 0))
    for i, q in enumerate(keep2):
        T[kept[q], :] = Linv_T[i, :] / d[kept[q]]
    return T, [kept[q] for q in keep2]


@dataclass
class BlockCGResult:
    X: np.ndarray               # n x s
    iterations: np.ndarray      # per column: block iterations until it stopped
    status: np.ndarray          # per column: OK, NOT_CONVERGED or BREAKDOWN
    rel_residual: np.ndarray    # per column ||f_j - A x_j|| / ||f_j||
    directions: List[int] = field(default_factory=list)  # search directions per iteration


def block_cimmino_block_cg(A, F, part, K, X0=None, tol=1e-10, maxit=10000,
                           backend="auto", proj: Optional[BlockProjections] = None,
                           drop: float = 1e-10) -> BlockCGResult:
    """Block CG on H X = Xi, Xi = [sum_i A_i^+ f_ij]_j, for the s columns of F
    (n x s).  One iteration applies H to the p <= s search directions P
    (orthonormal columns):

      Q = H P, M = P^T Q, alpha = M^{-1} P^T R  (minimizes the H-norm error
      over X + span P); X += P alpha, R -= Q alpha;
      beta = -M^{-1} Q^T R (the new directions are H-conjugate to P);
      P = orthonormal basis of R + P beta (orthonormal_directions).

    Only the columns not yet stopped take part: a column stops when its true
    residual satisfies ||f_j - A x_j||_2 <= tol ||f_j||_2 (tested on X0 and
    after each update, as in Algorithm 2) and is then left out of alpha, beta
    and the next directions.  A direction that is (numerically) in the span
    of the others is dropped, so repeated or dependent right-hand sides do
    not break the iteration.  With s = 1 this is Algorithm 2.  Breakdown: M
    not positive definite, or no direction left while columns are active."""
    A = sp.csr_matrix(A)
    F = np.asarray(F, dtype=np.float64)
    if F.ndim == 1:
        F = F[:, None]
    n, nr = F.shape
    if proj is None:
        proj = BlockProjections(A, part, K, backend)
    X = np.zeros((n, nr)) if X0 is None else np.array(X0, dtype=np.float64).reshape(n, nr)
    nf = np.linalg.norm(F, axis=0)
    S = F - A @ X
    iters = np.zeros(nr, dtype=np.int64)
    status = np.full(nr, NOT_CONVERGED, dtype=np.int64)
    act = []
    for j in range(nr):
        if nf[j] == 0.0 or np.linalg.norm(S[:, j]) <= tol * nf[j]:
            status[j] = OK
        else:
            act.append(j)
    dirs = []

    def result():
        rel = np.array([np.linalg.norm(S[:, j]) / nf[j] if nf[j] > 0 else 0.0 for j in range(nr)])
        return BlockCGResult(X, iters, status, rel, dirs)

    if not act:
        return result()
    R = np.zeros((n, nr))
    for j in act:
        R[:, j] = proj.min_norm_sum(S[:, j])
    T, _ = orthonormal_directions(R[:, act], drop)
    P = R[:, act] @ T
    for t in range(1, maxit + 1):
        if P.shape[1] == 0:
            status[act] = BREAKDOWN
            return result()
        dirs.append(P.shape[1])
        Q = np.column_stack([proj.H(P[:, k]) for k in range(P.shape[1])])
        M = P.T @ Q
        try:
            Lm = np.linalg.cholesky(M)
        except np.linalg.LinAlgError:
            status[act] = BREAKDOWN
            return result()
        alpha = np.linalg.solve(Lm.T, np.linalg.solve(Lm, P.T @ R[:, act]))
        X[:, act] += P @ alpha
        R[:, act] -= Q @ alpha
        S[:, act] = F[:, act] - A @ X[:, act]
        still = []
        for j in act:
            iters[j] = t
            if np.linalg.norm(S[:, j]) <= tol * nf[j]:
                status[j] = OK
            else:
                still.append(j)
        act = still
        if not act:
            return result()
        beta = -np.linalg.solve(Lm.T, np.linalg.solve(Lm, Q.T @ R[:, act]))
        Z = R[:, act] + P @ beta
        T, _ = orthonormal_directions(Z, drop)
        P = Z @ T
    return result()
