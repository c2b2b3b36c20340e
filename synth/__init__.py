"""Seeded synthetic inputs for linked ray tracing (sound-speed media, ring geometry
parameters, residual vectors, pair lists).

This module holds no part of the ray-tracing method itself: it only produces the
inputs that both the HIP path and the CPU oracle consume.  Every generator is
deterministic in its seed (numpy PCG64 ``default_rng``).
"""
from .media import (  # noqa: F401
    node_coords,
    homogeneous,
    linear_gradient,
    fisheye,
    gaussian_inclusions,
    smooth_random,
    striped_disc,
)
from .volume import (  # noqa: F401
    node_coords3,
    gaussian_inclusions3,
    fisheye3,
    linear_gradient3,
    hemisphere_elements,
)
from .configs import CONFIGS, CONFIGS3, make_config, make_config3, all_pairs, real_residual, complex_residual, c5_instances  # noqa: F401
