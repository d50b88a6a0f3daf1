"""Seeded synthetic PXST scans shared by the oracle tests, the GPU tests and the benchmark.

This package only *simulates an acquisition*: it draws a speckle reference, a
white-field, a smooth separable displacement field and a translation grid, and
renders Poisson frames with scipy's order-1 ``map_coordinates``.  It holds none of
the reconstruction arithmetic (no splat, no candidate search, no error figures),
and neither the oracle nor the HIP path imports anything from the other.
"""
from .scans import (  # noqa: F401
    Scan,
    ScanSpec,
    CONFIGS,
    make_scan,
    spec_for,
    served_job_specs,
    exact_scan,
    random_small_scan,
)
