"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws problem instances and starting populations and states
the closed-form functions' domains.  It holds none of the optimizer's
arithmetic: no objective evaluation, no gradient, no step of the oscillation
cycle.
"""
from .gen import (
    ACKLEY,
    BUKIN6,
    CLOSED_FORMS,
    GAUSS,
    MICHALEWICZ,
    RASTRIGIN,
    SCHWEFEL,
    STUDENT_T,
    STYBLINSKI_TANG,
    TRID,
    Problem,
    RunConfig,
    closed_form_box,
    closed_form_problem,
    gauss4_d2,
    gauss32_d16,
    gauss128_d64,
    batch64,
    student48_d32,
    mixture_problem,
    two_peak_problem,
    uniform_population,
)

__all__ = [
    "ACKLEY",
    "BUKIN6",
    "CLOSED_FORMS",
    "GAUSS",
    "MICHALEWICZ",
    "RASTRIGIN",
    "SCHWEFEL",
    "STUDENT_T",
    "STYBLINSKI_TANG",
    "TRID",
    "Problem",
    "RunConfig",
    "closed_form_box",
    "closed_form_problem",
    "gauss4_d2",
    "gauss32_d16",
    "gauss128_d64",
    "batch64",
    "student48_d32",
    "mixture_problem",
    "two_peak_problem",
    "uniform_population",
]
