"""Seeded synthetic inputs (points, radiation source I, field magnitude |E|).

This package only draws and shapes input data.  It contains none of the
photoionization method's arithmetic (no kernel, no quadrature, no selection),
so both the FP64 oracle and the HIP path can take their inputs from it.
"""
from .fields import (  # noqa: F401
    GAS_760,
    GAS_40,
    Workload,
    grid_points,
    config1,
    config2,
    config3,
    config5,
    gaussian_ball,
    sample_targets,
)
