"""Seeded synthetic inputs (scenes and path-vertex streams) for tests and benchmarks."""
from .workloads import WORKLOADS, Workload, ViewSpec, frame_seed, generate, get  # noqa: F401
from .keys import synthetic_keys  # noqa: F401,E402
from .cloud import mixed_normals_frame  # noqa: F401,E402
