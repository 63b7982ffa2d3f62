"""Seeded generators for the synthetic workloads.

Every generator draws from ``numpy.random.default_rng(seed)`` in a fixed,
documented order, so the same call returns identical bits on any host.  The
matrices are square, nonsingular and nonsymmetric, stored as CSR with sorted,
unique column indices per row (int32 indices, float64 values).

Workload recipes (the paper evaluates on SuiteSparse matrices with
5e4 <= n <= 5e6 and about 3-100 nonzeros per row, Section 3.3; these seeded
matrices stand in for that collection):

* ``cd2d``   2D 5-point upwind convection-diffusion, Dirichlet boundary.
* ``cd3d``   3D 7-point upwind convection-diffusion, Dirichlet boundary.
* ``powerlaw`` random sparse, power-law row lengths, diagonally shifted.
* ``stencil27`` 3D 27-point stencil with random nonsymmetric weights.

The right-hand side is always ``f = A @ xstar`` (Section 3.1 uses a vector of
ones for ``xstar``; some workloads use a Gaussian ``xstar``).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class Csr:
    n: int
    rowptr: np.ndarray  # int32, n+1
    col: np.ndarray     # int32, nnz
    val: np.ndarray     # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(M) -> "Csr":
        M = sp.csr_matrix(M)
        M.sum_duplicates()
        M.sort_indices()
        return Csr(M.shape[0], M.indptr.astype(np.int32), M.indices.astype(np.int32),
                   M.data.astype(np.float64))


@dataclass
class Problem:
    name: str
    A: Csr
    xstar: np.ndarray
    f: np.ndarray
    K: int
    # contiguous block boundaries (K+1 ints) when the partition is contiguous;
    # None when the partition is to be computed from the row inner-product graph
    bounds: Optional[np.ndarray]
    partition: str  # "contiguous" | "greedy-rip"
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.n

    def part(self) -> np.ndarray:
        if self.bounds is None:
            raise ValueError("partition of %s comes from the row inner-product graph" % self.name)
        return blocks_to_part(self.bounds)


def _finish(name, A, xstar, K, bounds, partition, **meta) -> Problem:
    f = A.to_scipy() @ xstar
    return Problem(name, A, xstar, np.ascontiguousarray(f, dtype=np.float64), K,
                   bounds, partition, dict(meta))


def _csr_from_dense_stencil(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray) -> Csr:
    """cols/vals/mask are (n, w) arrays with ascending columns along axis 1."""
    n = cols.shape[0]
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return Csr(n, rowptr.astype(np.int32), cols[mask].astype(np.int32),
               vals[mask].astype(np.float64))


def cd2d(N: int, b=(10.0, 10.0)) -> Csr:
    """2D 5-point upwind convection-diffusion on an N x N interior grid.

    Unknown (ix, iy) has index ix + N*iy.  The operator is scaled by h^2,
    h = 1/(N+1): diagonal 4 + h(|bx|+|by|); west -1 - h*max(bx,0);
    east -1 - h*max(-bx,0); south -1 - h*max(by,0); north -1 - h*max(-by,0).
    """
    bx, by = float(b[0]), float(b[1])
    h = 1.0 / (N + 1)
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    ix, iy = idx % N, idx // N
    offs = [-N, -1, 0, 1, N]
    vals = [-1 - h * max(by, 0.0), -1 - h * max(bx, 0.0), 4 + h * (abs(bx) + abs(by)),
            -1 - h * max(-bx, 0.0), -1 - h * max(-by, 0.0)]
    ok = [iy > 0, ix > 0, np.ones(n, bool), ix < N - 1, iy < N - 1]
    cols = np.stack([idx + o for o in offs], axis=1)
    V = np.broadcast_to(np.array(vals), (n, 5)).copy()
    M = np.stack(ok, axis=1)
    return _csr_from_dense_stencil(cols, V, M)


def cd3d(N: int, b) -> Csr:
    """3D 7-point upwind convection-diffusion on an N^3 interior grid.

    Unknown (ix, iy, iz) has index ix + N*iy + N^2*iz.  Scaled by h^2 with
    diagonal 6 + h*sum|b_d| and the same upwind rule as :func:`cd2d` per axis.
    """
    bx, by, bz = (float(t) for t in b)
    h = 1.0 / (N + 1)
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    ix, iy, iz = idx % N, (idx // N) % N, idx // (N * N)
    offs = [-N * N, -N, -1, 0, 1, N, N * N]
    vals = [-1 - h * max(bz, 0.0), -1 - h * max(by, 0.0), -1 - h * max(bx, 0.0),
            6 + h * (abs(bx) + abs(by) + abs(bz)),
            -1 - h * max(-bx, 0.0), -1 - h * max(-by, 0.0), -1 - h * max(-bz, 0.0)]
    ok = [iz > 0, iy > 0, ix > 0, np.ones(n, bool), ix < N - 1, iy < N - 1, iz < N - 1]
    cols = np.stack([idx + o for o in offs], axis=1)
    V = np.broadcast_to(np.array(vals), (n, 7)).copy()
    M = np.stack(ok, axis=1)
    return _csr_from_dense_stencil(cols, V, M)


def stencil27(N: int, rng: np.random.Generator) -> Csr:
    """3D 27-point stencil on N^3 with i.i.d. U(-1,1) off-diagonal weights.

    Draw order: one (n, 26) block of U(-1,1) in row-major order, the 26
    neighbour offsets in ascending linear offset; draws of neighbours outside
    the grid are discarded.  Diagonal = 1.1 * sum |off-diagonals of the row|.
    """
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    ix, iy, iz = idx % N, (idx // N) % N, idx // (N * N)
    offs, oks = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                offs.append(dz * N * N + dy * N + dx)
                ok = np.ones(n, bool)
                if dx == -1: ok &= ix > 0
                if dx == 1: ok &= ix < N - 1
                if dy == -1: ok &= iy > 0
                if dy == 1: ok &= iy < N - 1
                if dz == -1: ok &= iz > 0
                if dz == 1: ok &= iz < N - 1
                oks.append(ok)
    draws = rng.uniform(-1.0, 1.0, size=(n, 26))
    V = np.empty((n, 27))
    V[:, :13] = draws[:, :13]
    V[:, 14:] = draws[:, 13:]
    M = np.stack(oks, axis=1)
    V[:, 13] = 0.0
    V[~M] = 0.0
    V[:, 13] = 1.1 * np.abs(V).sum(axis=1)
    cols = np.stack([idx + o for o in offs], axis=1)
    return _csr_from_dense_stencil(cols, V, M)


def powerlaw_gamma(lmin=5, lmax=400, mean=20.0) -> float:
    """Exponent g with E[L] = mean for P(L) proportional to L^-g on [lmin, lmax]."""
    L = np.arange(lmin, lmax + 1, dtype=np.float64)
    lo, hi = 0.0, 6.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        w = L ** -mid
        if (w * L).sum() / w.sum() > mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def powerlaw(n: int, rng: np.random.Generator, lmin=5, lmax=400, mean=20.0) -> Csr:
    """Random sparse nonsymmetric matrix with power-law row lengths.

    Draw order: (1) the n row lengths L (diagonal included) from the discrete
    law P(L) ~ L^-g on [lmin, lmax], g fitted so E[L] = mean; (2) L-1 distinct
    uniform off-diagonal columns per row (drawn with replacement; duplicate
    draws are redrawn in rounds until every row is duplicate-free); (3) one
    N(0,1) value per off-diagonal entry in final CSR order.  The diagonal is
    1.1 * (row 1-norm of the off-diagonals).
    """
    g = powerlaw_gamma(lmin, lmax, mean)
    Ls = np.arange(lmin, lmax + 1)
    p = Ls.astype(np.float64) ** -g
    p /= p.sum()
    L = rng.choice(Ls, size=n, p=p).astype(np.int64)
    noff = L - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), noff)
    cols = rng.integers(0, n - 1, size=rows.size)
    cols += cols >= rows
    while True:
        order = np.lexsort((cols, rows))
        rows, cols = rows[order], cols[order]
        dup = np.zeros(rows.size, bool)
        dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        k = int(dup.sum())
        if k == 0:
            break
        c = rng.integers(0, n - 1, size=k)
        c += c >= rows[dup]
        cols[dup] = c
    offv = rng.standard_normal(rows.size)
    diag = 1.1 * np.bincount(rows, weights=np.abs(offv), minlength=n)
    allr = np.concatenate([rows, np.arange(n, dtype=np.int64)])
    allc = np.concatenate([cols, np.arange(n, dtype=np.int64)])
    allv = np.concatenate([offv, diag])
    order = np.lexsort((allc, allr))
    allr, allc, allv = allr[order], allc[order], allv[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(allr, minlength=n), out=rowptr[1:])
    return Csr(n, rowptr.astype(np.int32), allc.astype(np.int32), allv)


# ---------------------------------------------------------------- partitions

def multi_rhs(A: Csr, nrhs: int, seed: int) -> tuple:
    """nrhs right-hand sides F[j] = A @ Xstar[j] for one matrix (Section 3.5's
    sequences of systems with one coefficient matrix): Xstar[0] is the vector
    of ones of Section 3.1, the others are standard Gaussian vectors drawn
    from default_rng(seed) one after another.  Returns (F, Xstar), each
    (nrhs, n) float64, C order."""
    rng = np.random.default_rng(seed)
    X = np.empty((nrhs, A.n))
    for j in range(nrhs):
        X[j] = 1.0 if j == 0 else rng.standard_normal(A.n)
    M = A.to_scipy()
    F = np.stack([M @ X[j] for j in range(nrhs)]) if nrhs else np.empty((0, A.n))
    return np.ascontiguousarray(F), X


def contiguous_blocks(n: int, K: int) -> np.ndarray:
    """K contiguous blocks of near-equal size; the first n % K get one extra row."""
    q, r = divmod(n, K)
    sizes = np.full(K, q, dtype=np.int64)
    sizes[:r] += 1
    b = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(sizes, out=b[1:])
    return b


def uneven_blocks(n: int, K: int, spread: float, rng: np.random.Generator) -> np.ndarray:
    """K contiguous blocks of size ~ (n/K)(1+u), u ~ U(-spread, spread).

    The raw sizes are rescaled to sum to n and rounded by largest remainder
    (ties to the lower block index)."""
    u = rng.uniform(-spread, spread, size=K)
    raw = (1.0 + u) * (n / (1.0 + u).sum())
    base = np.floor(raw).astype(np.int64)
    rem = n - int(base.sum())
    frac = raw - base
    order = np.lexsort((np.arange(K), -frac))
    base[order[:rem]] += 1
    b = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(base, out=b[1:])
    return b


def blocks_to_part(bounds: np.ndarray) -> np.ndarray:
    K = len(bounds) - 1
    sizes = np.diff(bounds)
    return np.repeat(np.arange(K, dtype=np.int32), sizes)


# ----------------------------------------------------------------- workloads

def config1() -> Problem:
    """n = 1024: 2D convection-diffusion 32x32, b = (10,10), xstar = 1, K = 4 contiguous."""
    A = cd2d(32, (10.0, 10.0))
    return _finish("cd2d-32-K4", A, np.ones(A.n), 4, contiguous_blocks(A.n, 4), "contiguous")


def _cfg2(N: int, K: int, seed: int, name: str) -> Problem:
    rng = np.random.default_rng(seed)
    b = rng.uniform(-20.0, 20.0, size=3)
    A = cd3d(N, b)
    xstar = rng.standard_normal(A.n)
    return _finish(name, A, xstar, K, None, "greedy-rip", b=b.tolist())


def config2() -> Problem:
    """n = 262144: 3D convection-diffusion 64^3, b ~ U(-20,20)^3 then xstar ~ N(0,1)
    from seed 2; K = 32 from the greedy partitioner on the row inner-product graph."""
    return _cfg2(64, 32, 2, "cd3d-64-K32-rip")


def small_config2(N: int = 16, K: int = 8) -> Problem:
    return _cfg2(N, K, 2, "cd3d-%d-K%d-rip" % (N, K))


def _cfg3(n: int, K: int, seed: int, name: str) -> Problem:
    rng = np.random.default_rng(seed)
    A = powerlaw(n, rng)
    xstar = rng.standard_normal(n)
    bounds = uneven_blocks(n, K, 0.3, rng)
    return _finish(name, A, xstar, K, bounds, "contiguous")


def config3() -> Problem:
    """n = 500000 power-law rows (mean 20, max 400), seed 3, K = 64 uneven (+-30%)."""
    return _cfg3(500000, 64, 3, "powerlaw-500k-K64")


def small_config3(n: int = 20000, K: int = 4) -> Problem:
    return _cfg3(n, K, 3, "powerlaw-%d-K%d" % (n, K))


def _cfg4(sides: List[int], K: int, name: str) -> List[Problem]:
    out = []
    for k, s in enumerate(sides):
        A = cd2d(int(s), (10.0, 10.0))
        out.append(_finish("%s[%d]-cd2d-%d" % (name, k, s), A, np.ones(A.n), K,
                           contiguous_blocks(A.n, K), "contiguous"))
    return out


def config4() -> List[Problem]:
    """256 independent 2D convection-diffusion systems, sides ~ U{48..256} (seed 4),
    b = (10,10), xstar = 1, K = 8 contiguous blocks each."""
    rng = np.random.default_rng(4)
    sides = rng.integers(48, 257, size=256)
    return _cfg4(sides.tolist(), 8, "batch256")


def small_config4(nsys: int = 6, smin: int = 8, smax: int = 40) -> List[Problem]:
    rng = np.random.default_rng(4)
    sides = rng.integers(smin, smax + 1, size=nsys)
    return _cfg4(sides.tolist(), 8, "batch%d" % nsys)


def _cfg5(N: int, K: int, seed: int, name: str) -> Problem:
    rng = np.random.default_rng(seed)
    A = stencil27(N, rng)
    return _finish(name, A, np.ones(A.n), K, contiguous_blocks(A.n, K), "contiguous")


def config5() -> Problem:
    """n = 1e6: 27-point stencil on 100^3, U(-1,1) weights, seed 5, xstar = 1,
    K = 512 contiguous (the greedy row inner-product partition is the comparison)."""
    return _cfg5(100, 512, 5, "st27-100-K512")


def small_config5(N: int = 12, K: int = 4) -> Problem:
    return _cfg5(N, K, 5, "st27-%d-K%d" % (N, K))
