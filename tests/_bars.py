"""Shared parity bars of the GPU tests.

Outer iteration counts: the GPU and the oracle stop on the same rule, so
their counts must be equal; a difference of one is accepted only as a
near-tie of the stop decision, i.e. when the oracle's stopping quantity
(relative true residual, or the backward error for the paper's rule) at the
smaller of the two counts is within NEAR_TIE relative of the tolerance.
Iterates are compared only at equal counts.
"""
NEAR_TIE = 1e-3


def counts_match(gpu_iters, ref_iters, quantity_at, tol, what=""):
    """True if the counts are equal; on a difference of one, asserts the
    near-tie (quantity_at(t) is the oracle's stopping quantity after t
    iterations, called only then) and returns False; otherwise fails."""
    d = int(gpu_iters) - int(ref_iters)
    if d == 0:
        return True
    assert abs(d) == 1, "%s iteration counts differ by %d (gpu %d, oracle %d)" % (
        what, d, gpu_iters, ref_iters)
    t = min(int(gpu_iters), int(ref_iters))
    q = float(quantity_at(t))
    assert abs(q - tol) <= NEAR_TIE * tol, (
        "%s counts differ by one (gpu %d, oracle %d) but the oracle's stopping quantity at %d "
        "is %.6e, not within %.0e of tol %.1e" % (what, gpu_iters, ref_iters, t, q, NEAR_TIE, tol))
    return False
