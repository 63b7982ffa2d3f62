"""Shared parity bars of the GPU tests.

Outer iteration counts: the GPU and the oracle stop on the same rule, so
their counts must be equal; a difference of one is accepted only as a
near-tie of the stop decision, i.e. when the oracle's stopping quantity
(relative true residual, or the backward error for the paper's rule) at the
smaller of the two counts is within NEAR_TIE relative of the tolerance.
Iterates are compared only at equal counts.

Full-size FP64 runs of thousands of iterations (counts_match_long) may also
differ by a few iterations when the two residual histories, compared at the
same iteration, differ by at most DRIFT relative: each block projection is
accurate to about u * cond(A_i A_i^T) relative (u = 2^-53), 2e-10 for the
largest 2D blocks (cond about 8e5), and the GPU and the oracle factor the
blocks differently (banded Cholesky in reverse Cuthill-McKee order against
sparse LU), so every one of the iterations applies H with a different error
at that level.  Near the stop such a history falls by about 2% per
iteration, so a few percent of drift moves the crossing of the tolerance by
a few iterations.  The count difference is bounded too, by DRIFT_COUNT of
the oracle's count.
"""
NEAR_TIE = 1e-3
DRIFT = 0.1
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


def counts_match_long(gpu_iters, ref_iters, quantity_at, gpu_quantity_at, tol, what=""):
    """counts_match, or for a larger difference (at most DRIFT_COUNT of the
    oracle's count) the drift bar: the GPU's stopping quantity after
    t = min(counts) iterations (gpu_quantity_at(t)) within DRIFT relative of
    the oracle's.  Returns True only for equal counts."""
    d = int(gpu_iters) - int(ref_iters)
    if d == 0:
        return True
    if abs(d) == 1 and _near_tie(gpu_iters, ref_iters, quantity_at, tol)[0]:
        return False
    assert abs(d) <= max(1, DRIFT_COUNT * int(ref_iters)), (
        "%s iteration counts differ by %d (gpu %d, oracle %d)" % (what, d, gpu_iters, ref_iters))
    t = min(int(gpu_iters), int(ref_iters))
    qo, qg = float(quantity_at(t)), float(gpu_quantity_at(t))
    drift = abs(qg - qo) / qo
    print("%s counts gpu %d oracle %d: stopping quantity after %d iterations gpu %.6e oracle "
          "%.6e (drift %.3f)" % (what, gpu_iters, ref_iters, t, qg, qo, drift))
    assert drift <= DRIFT, (
        "%s counts differ by %d and the stopping quantities after %d iterations differ by "
        "%.3f relative (gpu %.6e, oracle %.6e), above %.2f" % (what, d, t, drift, qg, qo, DRIFT))
    return False
