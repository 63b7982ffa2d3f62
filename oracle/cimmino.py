"""Block Cimmino iterations (oracle; test infrastructure).

* :func:`block_cimmino_cg`    - Algorithm 2: classical CG applied to
  H x = xi with xi = sum_i A_i^+ f_i (eq. (cg); the relaxation omega appears
  on both sides and cancels).
* :func:`block_cimmino_plain` - Algorithm 1 / eq. (iterscheme):
  x <- x + omega sum_i A_i^+ (f_i - A_i x).
* :func:`backward_error`      - the normwise backward error gamma of eq.
  (stopping), used by the paper's experiments with threshold 1e-10.

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
