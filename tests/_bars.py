"""Shared parity bars of the GPU tests.

Outer iteration counts: the GPU and the oracle stop on the same rule, so
their counts must be equal; a difference of one is accepted only as a
near-tie of the stop decision, i.e. when the oracle's stopping quantity
(relative true residual, or the backward error for the paper's rule) at the
smaller of the two counts is within NEAR_TIE relative of the tolerance.
Iterates are compared only at equal counts.

Full-size FP64 runs of thousands of iterations (counts_match_long) may also
differ by up to DRIFT_COUNT of the oracle's count.  Each block projection is
accurate to about u * cond(A_i A_i^T) relative (u = 2^-53): 2e-10 for the
largest 2D blocks (cond about 8e5), which is the size of the tolerance
itself.  The GPU solves the normal equations with a banded Cholesky factor
in reverse Cuthill-McKee order, the oracle with corrected seminormal
equations, so the two apply H with different errors at that level in every
iteration, and where the residual falls only a few percent per iteration
the tolerance is crossed a few iterations apart.  Such a difference is
accepted when, after the oracle's count of iterations, the GPU iterate
agrees with the oracle's (the 1e-8 bar, checked by the caller) and the two
relative residuals differ by no more than that iterate difference explains:
| ||f - A x_g|| - ||f - A x_o|| | <= ||A (x_g - x_o)|| <= ||A||_2 ||x_g - x_o||,
with ||A||_2 <= sqrt(||A||_1 ||A||_inf) and ||x_g - x_o|| estimated from the
sampled entries (twice the estimate, for the sampling).
"""
import numpy as np

NEAR_TIE = 1e-3
DRIFT_COUNT = 0.005


def _near_tie(gpu_iters, ref_iters, quantity_at, tol):
    t = min(int(gpu_iters), int(ref_iters))
    q = float(quantity_at(t))
    return abs(q - tol) <= NEAR_TIE * tol, t, q


def counts_match(gpu_iters, ref_iters, quantity_at, tol, what=""):
    """True if the counts are equal; on a difference of one, asserts the
    near-tie (quantity_at(t) is the oracle's stopping quantity after t
    iterations, called only then) and returns False; otherwise fails."""
    d = int(gpu_iters) - int(ref_iters)
    if d == 0:
        return True
    assert abs(d) == 1, "%s iteration counts differ by %d (gpu %d, oracle %d)" % (
        what, d, gpu_iters, ref_iters)
    ok, t, q = _near_tie(gpu_iters, ref_iters, quantity_at, tol)
    assert ok, (
        "%s counts differ by one (gpu %d, oracle %d) but the oracle's stopping quantity at %d "
        "is %.6e, not within %.0e of tol %.1e" % (what, gpu_iters, ref_iters, t, q, NEAR_TIE, tol))
    return False


def residual_gap_bound(A, f, n, dx_samples):
    """Bound of the difference of two relative residuals ||f - A x|| / ||f||
    implied by the difference of the iterates, dx_samples being x_g - x_o on
    a uniform sample of the n entries (A: scipy sparse)."""
    absA = abs(A)
    norm2_bound = float(np.sqrt(absA.sum(axis=0).max() * absA.sum(axis=1).max()))
    dx = 2.0 * float(np.sqrt(n / len(dx_samples) * np.sum(np.square(dx_samples))))
    return norm2_bound * dx / float(np.linalg.norm(f))


def counts_match_long(gpu_iters, ref_iters, quantity_at, tol, gpu_quantity_at_ref, gap_bound,
                      what=""):
    """counts_match, or for a larger difference (at most DRIFT_COUNT of the
    oracle's count): the GPU's relative residual after the oracle's count of
    iterations (gpu_quantity_at_ref) within gap_bound (residual_gap_bound of
    the iterates at that count) of the oracle's.  Returns True only for
    equal counts."""
    d = int(gpu_iters) - int(ref_iters)
    if d == 0:
        return True
    if abs(d) == 1 and _near_tie(gpu_iters, ref_iters, quantity_at, tol)[0]:
        return False
    assert abs(d) <= max(1, DRIFT_COUNT * int(ref_iters)), (
        "%s iteration counts differ by %d (gpu %d, oracle %d)" % (what, d, gpu_iters, ref_iters))
    qo, qg = float(quantity_at(int(ref_iters))), float(gpu_quantity_at_ref)
    print("%s counts gpu %d oracle %d: relative residual after %d iterations gpu %.6e oracle "
          "%.6e, difference %.3e, bound from the iterates %.3e"
          % (what, gpu_iters, ref_iters, ref_iters, qg, qo, abs(qg - qo), gap_bound))
    assert abs(qg - qo) <= gap_bound, (
        "%s counts differ by %d and the residuals after %d iterations differ by %.3e, more "
        "than the iterates explain (%.3e)" % (what, d, ref_iters, abs(qg - qo), gap_bound))
    return False
