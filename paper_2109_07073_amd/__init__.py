"""VGICP matching-cost factors on MI355X (gfx950).

The GPU part of Koide et al., "Globally Consistent 3D LiDAR Mapping with
GPU-accelerated GICP Matching Cost Factors" (IEEE RA-L 2021): voxel maps,
Hessian-factor linearization, cost evaluation and the voxel overlap metric,
as hand-written HIP kernels behind the C ABI in include/vgicp.h.

`paper_2109_07073_amd.vgicp` is the ctypes binding; importing it needs the
built libvgicp.so (python -m paper_2109_07073_amd.build).
"""
