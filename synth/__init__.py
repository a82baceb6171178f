"""Seeded synthetic inputs (scenes and path-vertex streams) for tests and benchmarks."""
from .workloads import WORKLOADS, Workload, ViewSpec, frame_seed, generate, get  # noqa: F401
