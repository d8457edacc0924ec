"""MI355X-native parametric voxelization of integer 3D line segments.

The method (Section 3, eq. (2)-(3) and Fig. 3 of arXiv 2009.09500) places the
points G_k = S + W*k, W = (E - S)/N, k = 0..N, and takes the voxel containing each
one.  Here N is the Chebyshev length max(|dx|,|dy|,|dz|) and the voxel of a point
is its coordinate rounded half up, evaluated exactly in integers, so every voxel
is bit-exact.  The voxels are emitted as per-segment int16 lists and as packed
occupancy bit-volumes by hand-written HIP kernels for gfx950 behind the C ABI in
``include/vox.h``; this package holds the thin Python binding over that ABI
(``binding``), the seeded synthetic workloads (``workloads``), the autotuner
driver and the serving loop.

Importing the package loads nothing native; ``binding.load()`` does.
"""

__all__ = ["binding", "workloads"]
