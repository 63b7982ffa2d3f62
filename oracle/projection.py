"""Block-row projections of the block Cimmino method (oracle; test infrastructure).

The method splits the rows of A into K blocks A_1..A_K (Section 1, eq.
(blockCimmino)).  Each block contributes the orthogonal projection onto the
range of A_i^T,

    P_i = A_i^+ A_i,   A_i^+ = A_i^T (A_i A_i^T)^{-1}          (Section 1),

and H = sum_i P_i (eq. (H)).  With the thin QR factorisation A_i^T = Q_i R_i
(eq. (Iterat)), P_i = Q_i Q_i^T and the minimum-norm solution of the
underdetermined system A_i delta = r is A_i^+ r = Q_i R_i^{-T} r.

Two interchangeable backends:

* :class:`QRProjector`   - the definition: dense Householder QR of the block
  restricted to its column support (columns where the block has a nonzero).
  Used on small inputs.
* :class:`CSNEProjector` - seminormal equations with one correction step:
  factor G_i = A_i A_i^T (dense Cholesky or sparse LU), y = G_i^{-1} r,
  delta = A_i^T y, then delta += A_i^T G_i^{-1} (r - A_i delta).  Used where
  the dense QR does not fit; cross-checked against the QR backend.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class SingularBlock(ValueError):
    """A_i does not have full row rank (so A is singular)."""


def _as_csr(M) -> sp.csr_matrix:
    M = sp.csr_matrix(M, dtype=np.float64)
    M.sum_duplicates()
    M.sort_indices()
    return M


class QRProjector:
    """P_i and A_i^+ from a dense Householder QR of A_i^T on its column support."""

    def __init__(self, Ai):
        Ai = _as_csr(Ai)
        self.m, self.n = Ai.shape
        self.support = np.unique(Ai.indices)
        if self.support.size < self.m:
            raise SingularBlock("block has %d rows but only %d nonzero columns"
                                % (self.m, self.support.size))
        B = Ai[:, self.support].toarray().T          # |c_i| x m_i  = A_i^T restricted
        self.Q, self.R = np.linalg.qr(B, mode="reduced")
        d = np.abs(np.diag(self.R))
        if self.m and d.min() <= self.m * np.finfo(np.float64).eps * np.abs(self.R).max():
            raise SingularBlock("rank-deficient block (min |R_jj| = %g)" % d.min())

    def project(self, v: np.ndarray) -> np.ndarray:
        """P_i v = Q_i (Q_i^T v)."""
        out = np.zeros(self.n)
        out[self.support] = self.Q @ (self.Q.T @ v[self.support])
        return out

    def min_norm(self, r: np.ndarray) -> np.ndarray:
        """A_i^+ r = Q_i R_i^{-T} r, the minimum-norm solution of A_i delta = r."""
        z = sla.solve_triangular(self.R, r, trans="T", lower=False)
        out = np.zeros(self.n)
        out[self.support] = self.Q @ z
        return out


class CSNEProjector:
    """A_i^+ by the seminormal equations on G_i = A_i A_i^T plus one correction."""

    def __init__(self, Ai, dense_max: int = 4096):
        self.A = _as_csr(Ai)
        self.At = self.A.T.tocsr()
        self.m, self.n = self.A.shape
        G = (self.A @ self.At).tocsc()
        self.dense = self.m <= dense_max
        if self.dense:
            try:
                self.chol = sla.cho_factor(G.toarray(), lower=True, check_finite=True)
            except np.linalg.LinAlgError as e:
                raise SingularBlock(str(e))
        else:
            try:
                self.lu = spla.splu(G, permc_spec="MMD_AT_PLUS_A")
            except RuntimeError as e:
                raise SingularBlock(str(e))

    def _gsolve(self, r):
        if self.dense:
            return sla.cho_solve(self.chol, r)
        return self.lu.solve(r)

    def min_norm(self, r: np.ndarray) -> np.ndarray:
        y = self._gsolve(r)
        delta = self.At @ y
        e = r - self.A @ delta
        return delta + self.At @ self._gsolve(e)

    def project(self, v: np.ndarray) -> np.ndarray:
        return self.min_norm(self.A @ v)


class BlockProjections:
    """All K blocks of a row partition.

    ``part[r]`` is the block of row r.  Block k holds the rows with
    ``part == k`` in ascending row order (the order inside a block does not
    change P_k, Section 2.2).  ``backend`` is "qr", "csne" or "auto" (QR when
    the dense block on its support has at most 2^22 entries).
    """

    def __init__(self, A, part: np.ndarray, K: int, backend: str = "auto",
                 dense_max: int = 4096):
        A = _as_csr(A)
        self.A = A
        self.n = A.shape[0]
        part = np.asarray(part)
        if part.shape != (self.n,) or part.min() < 0 or part.max() >= K:
            raise ValueError("part must map every row to [0, K)")
        self.K = K
        self.rows = [np.flatnonzero(part == k) for k in range(K)]
        if any(r.size == 0 for r in self.rows):
            raise ValueError("empty block")
        self.blocks = []
        for rows in self.rows:
            Ai = A[rows]
            use_qr = backend == "qr"
            if backend == "auto":
                ncols = np.unique(Ai.indices).size
                use_qr = ncols * rows.size <= (1 << 22)
            self.blocks.append(QRProjector(Ai) if use_qr else CSNEProjector(Ai, dense_max))

    def H(self, v: np.ndarray) -> np.ndarray:
        """H v = sum_i P_i v (eq. (H))."""
        out = np.zeros(self.n)
        for P in self.blocks:
            out += P.project(v)
        return out

    def min_norm_sum(self, s: np.ndarray) -> np.ndarray:
        """sum_i A_i^+ s_i where s_i are the entries of s on block i's rows."""
        out = np.zeros(self.n)
        for rows, P in zip(self.rows, self.blocks):
            out += P.min_norm(s[rows])
        return out

    def dense_H(self) -> np.ndarray:
        """H as a dense matrix (small n only)."""
        return np.column_stack([self.H(e) for e in np.eye(self.n)])
