"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws problem instances and starting populations.  It holds
none of the optimizer's arithmetic: no objective evaluation, no gradient, no
step of the oscillation cycle.
"""
from .gen import (
    GAUSS,
    STUDENT_T,
    Problem,
    RunConfig,
    config1,
    config2,
    config3,
    config4,
    config5,
    mixture_problem,
    uniform_population,
)

__all__ = [
    "GAUSS",
    "STUDENT_T",
    "Problem",
    "RunConfig",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5",
    "mixture_problem",
    "uniform_population",
]
