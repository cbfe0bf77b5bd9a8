"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and
the benchmark. Holds no alignment arithmetic."""
from .gen import PairSet, make, fuzz, from_lists, to_ascii, WORKLOADS, DESCRIPTIONS  # noqa: F401
