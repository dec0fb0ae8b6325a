"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

Holds geometry (marker sets) and workload recipes only; no part of the flow
solver's arithmetic lives here.
"""
from . import configs, shapes  # noqa: F401
