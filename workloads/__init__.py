"""Seeded synthetic inputs (geometry, block pattern, H and S) for the NOLSM path.

This package holds only input construction; it performs none of the density
matrix arithmetic and is shared by the oracle, the tests and the benchmark.
"""
from .water import Instance, water_box, water_with_slab, to_dense  # noqa: F401
from .configs import get_config, CONFIGS  # noqa: F401
