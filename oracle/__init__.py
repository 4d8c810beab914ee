"""FP64 CPU oracle for the sweeping-plane light-field method (test infrastructure only).

This package is a plain, slow, obviously-correct restatement of what the paper
"Real-time 3D Visualization of Radiance Fields on Light Field Displays"
(Kim, Sun, Stengel et al.) computes on its hot path:

* ``geometry``   reference camera, view grid and filter strength (Sec. 4.2-4.3, Eqs. 1-5, 8)
* ``decisions``  the integer decisions (depth keys, frustum cull, plane sampling indices),
                 taken in IEEE float32 exactly as the GPU kernels take them
* ``partition``  sort by depth and split into chunks (Alg. 1 steps CulledDepth,
                 FindQuantile, Sort_and_Chunk; Sec. 4.4)
* ``project``    EWA projection of 3D Gaussians into the reference camera (Sec. 4.4)
* ``splat``      per-chunk front-to-back rasterisation into premultiplied RGBA planes
* ``voxels``     sparse-voxel chunks rasterised into planes + in-place low-pass (Sec. 4.5)
* ``composite``  swizzle blending of the planes into the light-field views (Eqs. 6-7, Alg. 1)
* ``render``     conventional per-view rendering (the paper's ground-truth baseline)
* ``grad``       gradients of a multi-view L2 loss (torch-CPU float64 autograd)
* ``quantize``   UNORM8 plane storage (Sec. 5.1)
* ``sh``         spherical-harmonic colour in the planes (the SH ablation, Fig. 6)

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU path; the only common
dependency is the seeded input generator ``scenegen``.
"""
from . import geometry, decisions, partition, project, splat, composite, render, voxels, grad, quantize, sh  # noqa: F401
