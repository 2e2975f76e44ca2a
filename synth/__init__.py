"""Seeded synthetic point-cloud workloads.

This package only draws random geometry (scenes, sensor poses, noise,
outliers).  It contains none of the registration method's arithmetic: no
voxel keys, neighbour search, normals, histograms or matching.  Both the
GPU path and the CPU oracle consume its outputs, so both see the same bytes.

Every generator is seeded from ``SeedSequence([2409, config, item])``.
Point clouds are returned as float32 structure-of-arrays of shape (3, n):
row 0 holds x, row 1 y, row 2 z.
"""

from .scenes import (  # noqa: F401
    rng_for,
    random_rotation,
    Params,
    params_indoor,
    params_c0,
    params_c1,
    c0_pair,
    c1_pair,
    lidar_scan,
    indoor_pair,
    lidar_pair,
    c2_batch,
    c2_sizes,
    lattice_pair,
    synthetic_descriptors,
    c4_trace,
    c4_pool,
    c4_requests,
    c3_pair,
)
