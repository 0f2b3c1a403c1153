"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds no arithmetic of the integration method itself: it only
builds analytic pressure fields with their exact gradients, analytic
velocity fields with their pressures, adds seeded noise (to gradients, or to
velocity by the paper's two models), and draws missing-data masks.  Everything returned is a plain
array; callers decide which solver (the HIP library or the CPU oracle) sees it.
"""

from .fields import (  # noqa: F401
    cell_centers,
    sin_cos_2d,
    quadratic,
    lamb_oseen_pair,
    lamb_oseen_vortices,
    gaussian_blobs,
    taylor_vortex,
    add_noise,
    disk_mask,
)
from .configs import (  # noqa: F401
    Workload,
    config_sin64,
    config_lamb_oseen_2d,
    config_blobs_3d,
    batched_instances,
    random_small,
)
from .velocity import (  # noqa: F401
    taylor_velocity,
    abc_velocity,
    noise_angular,
    noise_multiplicative,
)
