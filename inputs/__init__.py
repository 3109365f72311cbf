"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds problem *data* only: permeability fields, boundary data,
well sources, saturation snapshots and the workload definitions.  It contains
none of the multiscale method's arithmetic, so both the CPU oracle and the GPU
library can be fed from it without sharing any solver code.
"""
from .fields import lognormal_grf, channelized_field
from .problems import Problem, make_problem, WORKLOADS, synthetic_saturation

__all__ = [
    "lognormal_grf",
    "channelized_field",
    "Problem",
    "make_problem",
    "WORKLOADS",
    "synthetic_saturation",
]
