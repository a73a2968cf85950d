"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle's tests.

This package draws random numbers and builds input arrays only: point clouds on procedural
surfaces, their value-noise colours, random Gaussian sets and pinhole cameras. It holds none of
the rendering method's arithmetic (no projection, no covariance, no compositing, no kNN-PCA).
"""
from .scenes import (  # noqa: F401
    Camera,
    look_at_camera,
    orbit_cameras,
    focal_for_vfov,
    random_gaussians,
    ProceduralSurface,
    make_surface,
    deformed_surface,
    quantize_10bit,
    CONFIG_SEEDS,
)
