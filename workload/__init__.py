"""Seeded synthetic inputs for the tensor-equation solver.

This package is shared by the FP64 oracle (``oracle/``) and by the GPU path's
tests and benchmark.  It holds no arithmetic of the solver itself: no mode
products, no normal operator, no Krylov step.  It only draws random tensors and
builds the problem's input matrices (spline collocation and finite-difference
factors), which the paper leaves to the application (Sec. 6 names a
spline-based variational reconstruction without fixing its basis).

Conventions: tensors are NumPy arrays in C order (mode 1 slowest, mode N
contiguous); all random numbers come from ``numpy.random.default_rng(seed)``.
"""
from .bspline import collocation_matrix, second_difference
from .problems import (
    Problem,
    make_problem,
    config_problem,
    batched_sizes,
    batched_problem,
    blob_field,
    blob_field_torch,
    factors,
    warmstart_problem,
    integer_tensor,
    CONFIGS,
)
from .scattered import (
    SCATTERED,
    ScatteredProblem,
    scattered_sites,
    scattered_problem,
    scattered_config,
    with_endpoints,
)

__all__ = [
    "collocation_matrix",
    "second_difference",
    "Problem",
    "make_problem",
    "config_problem",
    "batched_sizes",
    "batched_problem",
    "blob_field",
    "blob_field_torch",
    "factors",
    "warmstart_problem",
    "integer_tensor",
    "CONFIGS",
    "SCATTERED",
    "ScatteredProblem",
    "scattered_sites",
    "scattered_problem",
    "scattered_config",
    "with_endpoints",
]
