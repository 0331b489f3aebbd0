"""Seeded synthetic inputs (meshes, cross-section tables, sources, jobs).

Shared by the HIP path, the oracle and the benchmarks; contains no transport
arithmetic.
"""
from . import meshgen, xsgen, configs  # noqa: F401
