"""FP64 CPU oracle for the redshift-space bispectrum estimators (test infrastructure).

This package is test infrastructure, not product code: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. It shares no code with the HIP library (no kernels, headers,
tables or helpers); the only module both sides use is ``synth`` (seeded
inputs, no estimator arithmetic).

Parity status of each function is stated in its docstring; the pins that
check it against the paper and the mathematics live in ``tests/test_oracle_*``.
"""
from .bispec import *  # noqa: F401,F403
