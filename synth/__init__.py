"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package draws the random systems and initial conditions; it performs none
of the propagation arithmetic.
"""
from . import units, angular, systems  # noqa: F401
