"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds only input generation: cell-centred grids, the
straight-ray crosswell measurement operator H (Sec. 4.1, eq.
``equation_traveltimeintegral``: H_ij is the length of ray i inside cell j),
seeded standard-normal draws and a synthetic plume truth.  It contains none of
the filter's or the H^2 product's arithmetic (no covariance kernel, no Kalman
update, no interpolation); both the oracle and the HIP path consume what it
produces.
"""

from .grid import grid_shape, cell_centres, grid_size
from .rays import crosswell_geometry, crosswell_h, ray_lengths
from .streams import (normal_draws, plume_truth, observations, plume_observations, WORKLOADS,
                      workload, serving_streams, poisson_requests)

__all__ = [
    "grid_shape", "cell_centres", "grid_size",
    "crosswell_geometry", "crosswell_h", "ray_lengths",
    "normal_draws", "plume_truth", "observations", "plume_observations", "WORKLOADS", "workload",
    "serving_streams", "poisson_requests",
]
