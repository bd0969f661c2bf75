"""Seeded synthetic inputs for the SMPC plan step (robot, scenes, noise, targets).

Shared by the FP64 oracle tests, the GPU tests and the benchmark.  It holds no
part of the plan step's arithmetic.
"""
from . import robot, scene, workload  # noqa: F401
