"""Seeded synthetic inputs for the per-block BTO advection path.

This package only *describes inputs*: velocity grids sampled from analytic
flows, seed-lattice parameters, loss weights and the storage-precision rounding
of the grids.  It holds none of the method's arithmetic (no sampling, no time
stepping, no termination): both the FP64 CPU oracle and the HIP library consume
what it produces, and neither is imported from here.

Grid convention: a block of ``n = (nx, ny, nz)`` points with unit spacing, point
(i, j, k) at local coordinate (i, j, k); a velocity grid is an array of shape
``(nz, ny, nx, 3)`` (array-of-structures, x fastest), values in cells per unit
time.
"""

from .fields import (  # noqa: F401
    FieldSeries,
    double_gyre,
    abc_noise,
    turbulence_modes,
    turbulence,
    uniform_flow,
    solid_body_rotation,
    affine_time_linear,
    trilinear_polynomial,
)
from .quant import quantize, promote, STORAGE_DTYPES  # noqa: F401
from .workloads import WORKLOADS, make_workload  # noqa: F401
