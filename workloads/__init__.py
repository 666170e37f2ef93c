"""Seeded synthetic input generators shared by the tests, the oracle checks and the
benchmark.  This module only builds matrices; it holds none of the logarithm
method's arithmetic.
"""

from .matrices import (  # noqa: F401
    CONFIG_SEEDS,
    complex_matrix,
    real_representation,
    disk_matrix,
    rotscale_matrix,
    spd_batch,
    named_workload,
)
