"""pcsplat for MI355X: a 3D elliptical-Gaussian splatting rasterizer (arXiv:2409.16504, Section 3.1)
written as HIP kernels for gfx950 behind the C ABI of libpcsplat.so (include/pcsplat.h).

The package holds the kernels (csrc/), their build script and a thin ctypes binding that takes
PyTorch tensors for device memory and streams.
"""
from ._lib import PcsError, STAGES  # noqa: F401
from .render import (  # noqa: F401
    RenderFunction,
    RenderState,
    Renderer,
    camera_struct,
    default_options,
    render_autograd,
)
