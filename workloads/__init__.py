"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

Geometry/connectivity tables, codebooks, random vectors and direction sets.
No electromagnetic arithmetic lives here, so neither side borrows the other's
method code through this package.
"""
from . import codebooks, configs, mesh  # noqa: F401
