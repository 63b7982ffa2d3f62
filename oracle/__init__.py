"""FP64 CPU oracle for the CG-accelerated block Cimmino method (test infrastructure).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library
never calls it, shares no code with it, and must fail loudly when its own HIP
extension is missing instead of falling back to anything here.

Contents (each function cites the passage of the paper it follows):

* :mod:`oracle.projection` - block-row projections P_i = A_i^+ A_i by dense
  Householder QR of A_i^T (the definition, small inputs) and by the corrected
  seminormal equations (large inputs); Section 1, eqs. (iterscheme), (H),
  (Iterat).
* :mod:`oracle.cimmino`   - Algorithm 2 (classical CG on H x = xi), the
  normwise backward error of eq. (stopping), Algorithm 1 (plain block
  Cimmino with relaxation omega), and block CG on H for several right-hand
  sides (Section 3.1).
* :mod:`oracle.ripgraph`  - the row inner-product graph of Section 2.1 built
  from C = A A^T with the dense-column sparsification and integer edge
  weights of Section 2.3.
* :mod:`oracle.partition` - the deterministic greedy and multilevel K-way
  partitioners used in place of METIS, cutsize / interIP (Sections 2.2, 3.1,
  Appendix A).

Everything is float64 with plain NumPy/SciPy operations; no blocking, fusion
or reordering beyond what the definitions state.
"""
from .projection import QRProjector, CSNEProjector, BlockProjections
from .cimmino import (block_cimmino_cg, block_cimmino_plain, backward_error,
                      CimminoResult, OK, NOT_CONVERGED, BREAKDOWN,
                      block_cimmino_block_cg, orthonormal_directions, BlockCGResult)
from .ripgraph import rip_graph, rip_rows, row_norms, sparsify_columns, RipGraph
from .partition import (greedy_partition, multilevel_partition, cutsize, int_cut, ip_matrix,
                        imbalance, brute_force_min_cut, part_max_weight)

__all__ = [
    "QRProjector", "CSNEProjector", "BlockProjections",
    "block_cimmino_cg", "block_cimmino_plain", "backward_error", "CimminoResult",
    "block_cimmino_block_cg", "orthonormal_directions", "BlockCGResult",
    "OK", "NOT_CONVERGED", "BREAKDOWN",
    "rip_graph", "rip_rows", "row_norms", "sparsify_columns", "RipGraph",
    "greedy_partition", "multilevel_partition", "cutsize", "int_cut", "ip_matrix", "imbalance",
    "brute_force_min_cut", "part_max_weight",
]
