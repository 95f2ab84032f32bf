"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This module only draws random numbers (point clouds, weights, rigid motions,
arrival times).  It holds none of the solver's arithmetic: no centring, no
lifting, no costs, no Sinkhorn.  Both sides of every parity test receive the
same arrays from here.
"""
from .synth import (  # noqa: F401
    Problem,
    haar_rotation,
    gmm_points,
    config1_plain,
    config2_fp32,
    config3_scale,
    config4_requests,
    config5_grad,
    subsample,
    rotated_copy,
    landmark_indices,
    splitmix64_landmarks,
    splitmix64_stream,
    grad_points,
    scale_features,
    c5_subsample,
    seeded_gamma,
)
