"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This package only draws inputs: point clouds with per-point covariances, poses
and factor lists shaped like the paper's LiDAR workloads.  It contains none of
the matching-cost arithmetic (no voxel keys, no residuals, no Jacobians).
"""

from .scenes import (  # noqa: F401
    Workload,
    knn_covariances,
    normal_covariances,
    random_perturbation,
    make_single_factor,
    make_scan_workload,
    make_tiny_workload,
    make_degenerate_workload,
    DEGENERATE_COVS,
    pose_rows,
    rng_for,
    stream_scan_frames,
    drive_positions,
)
