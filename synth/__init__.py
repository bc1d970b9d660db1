"""Seeded synthetic inputs shared by the HIP path and the oracle.

This package holds no arithmetic of the performance model: only
random number generation for kernel input buffers and the parameter lists
(kernel variants) of the measurement, test, batched and serving workloads.
"""
from .inputs import (  # noqa: F401
    SEED_BASE, seed_for, uniform,
    suite_tiny, suite_instructive, suite_test, suite_batched, serving_trace,
    WG_SIZES, suite_wg,
)
