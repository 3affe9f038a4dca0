"""Seeded synthetic inputs for the RHIF solver: coefficient fields, reaction terms and
right-hand sides.

This package holds no arithmetic of the factorization itself. Both the CPU oracle and the
GPU path read the arrays it produces, so the two always see the same inputs.
"""
from .fields import (  # noqa: F401
    Problem,
    two_valued_field,
    gaussian_random_field,
    quantized_paper_field,
    make_problem,
    CONFIGS,
)
