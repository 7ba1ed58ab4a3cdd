"""Seeded synthetic inputs shared by the oracle tests and the HIP path."""
from .workloads import Workload, make, custom, subset, box_map, SEEDS  # noqa: F401
