"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package generates catalogues and density fields only. It contains none of
the estimator's arithmetic (no mass assignment, no line-of-sight moments, no
shell filtering, no triple sums): those live separately in ``oracle/`` (CPU,
FP64) and in the HIP library, which share no code.
"""
from .catalog import (  # noqa: F401
    WORKLOADS, Workload, workload, gaussian_field, lognormal_catalogue,
    quantise_grid_units, power_law_gaussian_spectrum, observer_grid_units,
)
