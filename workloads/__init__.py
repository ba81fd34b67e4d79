"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This package holds only data definitions (lattices, direction matrices,
array sizes, query ranges) and seeded random generators.  It contains none
of the method's arithmetic and imports neither the oracle nor the GPU path.
"""

from .configs import CONFIGS, Config, get  # noqa: F401
from .inputs import (  # noqa: F401
    coefficients, queries, targets, ray_params, ray_samples, smooth_field,
)
