"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only *draws inputs*: workload descriptions (image sizes, parameter
ranges), procedural flow grids, and free-standing particle sets used to feed a
single stage in isolation.  It contains none of the generator's own arithmetic
(no Philox, no seeding rule, no advection, no rendering), so that the CPU
oracle under ``oracle/`` and the HIP library can both consume it without
sharing any of the method's code.
"""

from .configs import WORKLOADS, Workload, get_workload  # noqa: F401
from .flows import lamb_oseen_grid, fourier_grid, uniform_grid, make_flows  # noqa: F401
from .particles import random_particles, edge_case_particles  # noqa: F401
