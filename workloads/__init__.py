"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds random-number generation, random circuits, tensor-network construction
and path/slice choices.  It contains none of the contraction arithmetic.
"""
from . import circuits, configs, paths, rng  # noqa: F401
