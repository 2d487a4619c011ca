"""Seeded synthetic workload generators shared by the oracle tests, the GPU tests and bench.py."""
from .generators import CSR, Problem, make, start_block, splitmix64_block, island_block, lap2d_island, lap2d, lap3d, fem3d, aniso3d, powerlaw  # noqa: F401
