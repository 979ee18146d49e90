"""Seeded synthetic inputs shared by the oracle tests, the HIP-path tests and
the benchmark.

This package describes *problems* (meshes, materials, sources, inflow); it
holds none of the transport or moment-system arithmetic.  Both the CPU oracle
and the HIP library consume what it produces, and neither side imports the
other.
"""
from .generators import *  # noqa: F401,F403
