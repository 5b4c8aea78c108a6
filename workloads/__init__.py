"""Seeded synthetic input generators shared by the tests, the oracle runs and
the benchmark.  They hold no part of the transport method's arithmetic."""
from .problem import Boundary, Problem, CELL_TYPES, BC_KINDS  # noqa: F401
from . import configs, meshes, tables  # noqa: F401
