"""Spectrum of H = sum_i A_i^+ A_i (eq. (H)) by the Lanczos method.

The convergence of both block Cimmino iterations is set by the eigenvalues of
H (Section 1.1): Algorithm 1 contracts the error by max |1 - omega lambda| per
step, fastest at omega = 2 / (lambda_min + lambda_max), and the CG bound of
Algorithm 2 depends on kappa = lambda_max / lambda_min and on how the
eigenvalues cluster around 1.  H is symmetric positive definite for a
nonsingular A, so a few dozen Lanczos steps give its extreme eigenvalues and
a picture of the clustering, from products H v only; here each product is one
``bc_project`` call (the library's sparse products and block projections on the
GPU), and the Lanczos recurrence itself (a few vectors of length n) runs on
the host in float64 with full reorthogonalization.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable

import numpy as np
from scipy.linalg import eigh_tridiagonal


@dataclass
class Spectrum:
    ritz: np.ndarray        # Ritz values, ascending
    residuals: np.ndarray   # |beta_k * last component of the Ritz vector|, per Ritz value
    steps: int

    @property
    def lambda_min(self) -> float:
        return float(self.ritz[0])

    @property
    def lambda_max(self) -> float:
        return float(self.ritz[-1])

    @property
    def kappa(self) -> float:
        return self.lambda_max / self.lambda_min

    @property
    def omega_opt(self) -> float:
        """Relaxation parameter of Algorithm 1 minimizing max |1 - omega lambda|."""
        return 2.0 / (self.lambda_min + self.lambda_max)


def lanczos(matvec: Callable[[np.ndarray], np.ndarray], n: int, steps: int = 60,
            seed: int = 0) -> Spectrum:
    """`steps` Lanczos steps on the symmetric operator `matvec` (host float64
    vectors of length n in and out), with full reorthogonalization; stops early
    on an invariant subspace.  Returns the Ritz values and their residual
    estimates."""
    steps = int(min(steps, n))
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(n)
    q /= np.linalg.norm(q)
    Q = np.zeros((steps + 1, n))
    Q[0] = q
    alpha = np.zeros(steps)
    beta = np.zeros(steps)
    k = 0
    for k in range(steps):
        w = np.asarray(matvec(Q[k]), dtype=np.float64)
        alpha[k] = Q[k] @ w
        w -= alpha[k] * Q[k]
        if k > 0:
            w -= beta[k - 1] * Q[k - 1]
        # full reorthogonalization (twice is enough)
        for _ in range(2):
            w -= Q[:k + 1].T @ (Q[:k + 1] @ w)
        beta[k] = np.linalg.norm(w)
        if beta[k] <= 1e-12 * max(1.0, abs(alpha[k])):
            k += 1
            break
        Q[k + 1] = w / beta[k]
    else:
        k = steps
    m = k
    if m == 1:
        return Spectrum(np.array([alpha[0]]), np.array([beta[0]]), 1)
    theta, S = eigh_tridiagonal(alpha[:m], beta[:m - 1])
    return Spectrum(theta, np.abs(beta[m - 1] * S[-1, :]), m)


def spectrum_of(ctx, n: int, steps: int = 60, seed: int = 0, device: str = "cuda") -> Spectrum:
    """Lanczos on H of a library context (single system): each product is
    one bc_project on the device."""
    import torch
    from . import bc_project
    v = torch.empty(n, dtype=torch.float64, device=device)
    hv = torch.empty_like(v)

    def matvec(x):
        v.copy_(torch.from_numpy(np.ascontiguousarray(x)))
        bc_project(ctx, v, hv)
        return hv.cpu().numpy()

    return lanczos(matvec, n, steps, seed)
