"""Seeded synthetic inputs shaped like the paper's workloads.

This package only draws random numbers and lays them out as Dense and
Compressed levels (pos/crd/vals arrays).  It holds none of the arithmetic of
the operations: both the GPU path and the CPU oracle consume what it returns,
and neither is imported here.
"""
from .gen import *  # noqa: F401,F403
