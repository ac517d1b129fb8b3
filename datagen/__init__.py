"""Seeded synthetic inputs (precision matrices, Gaussian samples) for tests and benchmarks."""
from .synth import *  # noqa: F401,F403
from .synth import workload, Workload  # noqa: F401
