"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package only *generates* tensors.  It contains no part of the Tucker-ALS
method (no unfolding, Gram, eigen-solve, core or fit arithmetic): both the HIP
library and the CPU oracle receive its output as plain input data.
"""

from .stack import (  # noqa: F401
    haar_orthonormal,
    make_exact_rank,
    make_tiny,
    make_stereo_stack,
    serving_requests,
    STACK_CONFIGS,
)
