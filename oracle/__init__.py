"""FP64 CPU oracle for VGICP matching-cost factors.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this package.  It shares no code with the HIP
library and never imports it.
"""

from .vgicp_oracle import (  # noqa: F401
    VoxelMap,
    voxel_scale,
    voxel_keys,
    voxelize,
    relative_pose,
    lookup,
    fused_covariance,
    positive_definite,
    fused_information,
    linearize_factor,
    evaluate_factor,
    overlap_factor,
    factor_admitted,
    submap_decision,
    linearize_workload,
    overlap_workload,
    build_maps,
    assemble_system,
    system_blocks,
)
