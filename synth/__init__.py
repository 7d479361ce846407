"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package builds scanner geometry, line-of-response (LOR) endpoint lists,
voxel phantoms and listmode events.  It holds none of the projector's
arithmetic: it never projects, interpolates or evaluates a TOF kernel.  Every
array it returns is produced in float64 and rounded once to float32, so the
GPU path and the FP64 oracle consume bit-identical inputs.

The paper benchmarks on a GE Discovery MI geometry and on a measured NEMA
listmode acquisition (Sec. 2.6).  Neither ships here; the workloads below are
synthetic stand-ins with the same structure (cylindrical scanner, span-1
sinogram ordered radial/view/plane, unsorted listmode events with TOF bins).
"""
from .scanner import CylinderScanner, sinogram_planes, sinogram_crystal_pairs
from .phantom import ImageGrid, cylinder_sphere_phantom, ellipsoid_lesion_phantom
from .events import generate_tof_lm_events, tof_per_ray_params
from . import configs

__all__ = [
    "CylinderScanner",
    "sinogram_planes",
    "sinogram_crystal_pairs",
    "ImageGrid",
    "cylinder_sphere_phantom",
    "ellipsoid_lesion_phantom",
    "generate_tof_lm_events",
    "tof_per_ray_params",
    "configs",
]
