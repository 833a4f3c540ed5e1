"""Seeded synthetic inputs (meshes, animations, anchor sets, random starts).

Shared by the oracle's tests, the HIP library's tests and the benchmark.  It
holds none of the compression method's arithmetic.
"""
from . import animate, configs, learned, meshes  # noqa: F401
