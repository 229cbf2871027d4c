"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This package only draws random data in the shapes of the paper's workloads
(DC power-flow susceptance systems, random layered circuits, random unitaries,
batch and arrival schedules). It holds none of the HHL method's arithmetic:
no padding, eigen-decomposition, circuit construction or gate application.
"""
from .gen import *  # noqa: F401,F403
