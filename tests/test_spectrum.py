"""The Lanczos spectrum tool (host recurrence; the GPU products are tested
with the library).  Pinned against known spectra: a diagonal operator with
clustered eigenvalues, and the oracle's dense H of a small problem, whose
eigenvalues numpy computes directly."""
import numpy as np

import workloads
from oracle import BlockProjections
from paper_1710_07769_amd.spectrum import lanczos


def test_lanczos_extremes_of_a_known_spectrum():
    rng = np.random.default_rng(3)
    # most eigenvalues clustered near 1, a few outliers, as in H
    ev = np.concatenate([1.0 + 0.05 * rng.standard_normal(480), [0.03, 0.2, 1.9, 2.53]])
    sp = lanczos(lambda v: ev * v, ev.size, steps=80, seed=1)
    assert abs(sp.lambda_min - ev.min()) <= 1e-8 and abs(sp.lambda_max - ev.max()) <= 1e-8
    assert abs(sp.omega_opt - 2.0 / (ev.min() + ev.max())) <= 1e-8
    # Ritz values lie inside the spectrum
    assert sp.ritz.min() >= ev.min() - 1e-10 and sp.ritz.max() <= ev.max() + 1e-10


def test_lanczos_invariant_subspace_stops_early():
    ev = np.array([0.5] * 10 + [1.5] * 10)
    sp = lanczos(lambda v: ev * v, ev.size, steps=15, seed=0)
    assert sp.steps == 2
    assert np.allclose(np.sort(sp.ritz), [0.5, 1.5], atol=1e-12)


def test_lanczos_on_oracle_H():
    p = workloads.small_config2(N=8, K=4)
    part = workloads.blocks_to_part(workloads.contiguous_blocks(p.n, p.K))
    B = BlockProjections(p.A.to_scipy(), part, p.K)
    ev = np.linalg.eigvalsh(B.dense_H())
    sp = lanczos(B.H, p.n, steps=120, seed=2)
    assert abs(sp.lambda_min - ev[0]) <= 1e-9 * ev[-1]
    assert abs(sp.lambda_max - ev[-1]) <= 1e-9 * ev[-1]
    # eq. (H): the eigenvalues of H lie in (0, K]
    assert 0 < sp.lambda_min and sp.lambda_max <= p.K + 1e-12
