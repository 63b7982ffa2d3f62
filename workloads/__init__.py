"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This package only builds problem instances (matrices, right-hand sides,
partitions of the row set into contiguous blocks).  It contains none of the
block Cimmino arithmetic: no projections, no CG, no row inner products.
"""
from .gen import (Csr, Problem, cd2d, cd3d, powerlaw, stencil27,
                  contiguous_blocks, uneven_blocks, blocks_to_part, multi_rhs,
                  config1, config2, config3, config4, config5,
                  small_config2, small_config3, small_config4, small_config5)

__all__ = [
    "Csr", "Problem", "cd2d", "cd3d", "powerlaw", "stencil27",
    "contiguous_blocks", "uneven_blocks", "blocks_to_part", "multi_rhs",
    "config1", "config2", "config3", "config4", "config5",
    "small_config2", "small_config3", "small_config4", "small_config5",
]
