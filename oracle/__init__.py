"""CPU FP64 oracle for the cone-beam operators and the algorithms built on them.

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the benchmark's CPU-baseline
leg are the only callers.  The product path never imports this package, and this package never
imports the product (it shares only the seeded input generators, which hold none of the method's
arithmetic).

Operators (plain C in ``ct_oracle.c``, loaded with ctypes):
  siddon_fwd / siddon_rays         ray-driven exact intersection projector (Siddon 1985, Section 2.1)
  siddon_segments                  its piece count per ray (voxel reads per ray)
  siddon_adj / siddon_adj_voxels   its exact transpose (scatter of the same traversal)
  interp_fwd / interp_rays         trilinear-interpolated projector (Chou 2011, Section 2.1)
  bp / bp_voxels                   voxel-driven backprojection, FDK or pseudo-matched weights
                                   (Jia 2011, Section 2.2)
Every operator takes the projections' views either as angles of a circular orbit or as an n x 12
table of per-view source, detector centre and unit detector axes (C-arm, helical; Section 2.1).
Algorithms (``algos.py``, numpy over the operators): CGLS, SART and OS-SART, TV steepest descent
(whole and split), the ROF model by Chambolle's projection,
FDK reconstruction (cosine weight, ramp filter, FDK-weighted backprojection).
"""
from .core import (Geometry, W_FDK, W_PM, bp, bp_transpose, bp_voxels, circular_views, get_threads,
                   interp_fwd, interp_ray, interp_rays, ray_endpoints, set_threads, siddon_adj,
                   siddon_adj_voxels, siddon_fwd, siddon_ray, siddon_rays, siddon_segments, load)
from .algos import (cgls, div3, fdk, fdk_filter, grad3, os_sart, ramp_taps, rof_chambolle, rof_chambolle_split, sart,
                    tv_grad, tv_value, tv_steps, tv_steps_split)

__all__ = [
    "Geometry", "W_FDK", "W_PM", "bp", "bp_transpose", "bp_voxels", "circular_views", "get_threads",
    "interp_fwd", "interp_ray", "interp_rays", "ray_endpoints", "set_threads", "siddon_adj",
    "siddon_adj_voxels", "siddon_fwd", "siddon_ray", "siddon_rays", "siddon_segments", "load", "cgls", "fdk", "fdk_filter",
    "os_sart", "ramp_taps", "sart", "tv_grad", "tv_value", "tv_steps", "tv_steps_split", "grad3", "div3",
    "rof_chambolle", "rof_chambolle_split",
]
