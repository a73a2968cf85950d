"""ctypes declarations of libpcsplat.so (the C ABI in include/pcsplat.h).

Argument marshalling only: the library is loaded from this package's ``_build`` folder and every
step of the renderer runs in its HIP kernels. If the library is missing this raises; nothing falls
back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "libpcsplat.so")

c_f, c_i32, c_i64, c_u32, c_vp = ctypes.c_float, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p

PCS_OK, PCS_ERR_INVALID_ARG, PCS_ERR_HIP, PCS_ERR_OOM, PCS_ERR_CAPACITY, PCS_ERR_UNSUPPORTED = range(6)
FLAG_SAVE_STATE, FLAG_CAPACITY_MODE = 1, 2
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "HIP_ERROR", 3: "OUT_OF_MEMORY", 4: "CAPACITY", 5: "UNSUPPORTED"}
STAGES = ("project", "scan", "binning", "sort", "ranges", "composite", "backward_composite",
          "backward_project", "knn_pca", "voxelize", "conv", "conv_backward", "head", "head_backward",
          "shade")

EXPORTED = ("pcs_last_error", "pcs_context_create", "pcs_context_destroy", "pcs_context_set_allocator",
            "pcs_context_timing",
            "pcs_context_timing_stages", "pcs_shade",
            "pcs_context_timings", "pcs_state_create", "pcs_state_destroy", "pcs_options_default",
            "pcs_render_forward", "pcs_render_backward", "pcs_render_backward_noalloc", "pcs_state_bins",
            "pcs_state_status", "pcs_state_capacity", "pcs_context_set_wait_limit",
            "pcs_measure_lds_bandwidth", "pcs_pool", "pcs_pool_features", "pcs_pool_features_backward",
            "pcs_up_conv_forward", "pcs_up_conv_backward", "pcs_unet_head_forward", "pcs_unet_head_backward",
            "pcs_knn_pca", "pcs_voxels_create", "pcs_voxels_destroy", "pcs_voxelize", "pcs_voxels_get",
            "pcs_subm_conv_forward", "pcs_subm_conv_forward_cat", "pcs_subm_conv_backward", "pcs_estimator_head_forward",
            "pcs_estimator_head_backward")


class Camera(ctypes.Structure):
    _fields_ = [("T", c_f * 9), ("t", c_f * 3), ("fx", c_f), ("fy", c_f), ("cx", c_f), ("cy", c_f),
                ("width", c_i32), ("height", c_i32)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", c_i64), ("mean", c_vp), ("quat", c_vp), ("scale", c_vp), ("opacity", c_vp),
                ("rgb", c_vp), ("normal", c_vp)]


class Options(ctypes.Structure):
    _fields_ = [("z_near", c_f), ("lowpass", c_f), ("sigma_cut", c_f), ("alpha_min", c_f),
                ("alpha_max", c_f), ("t_eps", c_f), ("bg", c_f * 3), ("flags", c_u32)]


class Images(ctypes.Structure):
    _fields_ = [("rgb", c_vp), ("normal", c_vp), ("depth", c_vp), ("alpha", c_vp)]


class Light(ctypes.Structure):
    _fields_ = [("dir", c_f * 3), ("color", c_f * 3), ("ambient", c_f), ("diffuse", c_f),
                ("specular", c_f), ("shininess", c_f)]


class Grads(ctypes.Structure):
    _fields_ = [("mean", c_vp), ("cov6", c_vp), ("quat", c_vp), ("scale", c_vp), ("opacity", c_vp),
                ("rgb", c_vp), ("normal", c_vp)]


# allocator callbacks: alloc(bytes, user) -> device pointer or NULL; release(ptr, user)
ALLOC_FN = ctypes.CFUNCTYPE(c_vp, ctypes.c_size_t, c_vp)
FREE_FN = ctypes.CFUNCTYPE(None, c_vp, c_vp)


class PcsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pcsplat {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch-ROCm bundles the HIP runtime under the same soname; importing torch first makes the
    # library bind to that one runtime, so torch's streams and allocations are valid here.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc, gfx950); there is no other implementation to fall back to")
    L = ctypes.CDLL(LIB_PATH)
    L.pcs_last_error.restype = ctypes.c_char_p
    L.pcs_last_error.argtypes = []
    L.pcs_context_create.argtypes = [ctypes.c_int, ctypes.POINTER(c_vp)]
    L.pcs_context_destroy.argtypes = [c_vp]
    L.pcs_context_destroy.restype = None
    L.pcs_context_timing.argtypes = [c_vp, ctypes.c_int]
    L.pcs_context_set_allocator.argtypes = [c_vp, ALLOC_FN, FREE_FN, c_vp]
    L.pcs_context_timing_stages.argtypes = [c_vp, ctypes.c_uint32]
    L.pcs_context_timings.argtypes = [c_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_i64),
                                      ctypes.c_int, c_vp]
    L.pcs_state_create.argtypes = [c_vp, ctypes.POINTER(c_vp)]
    L.pcs_state_destroy.argtypes = [c_vp]
    L.pcs_state_destroy.restype = None
    L.pcs_options_default.argtypes = [ctypes.POINTER(Options)]
    L.pcs_options_default.restype = None
    L.pcs_render_forward.argtypes = [c_vp, ctypes.POINTER(Gaussians), ctypes.POINTER(Camera), c_i32,
                                     ctypes.POINTER(Options), ctypes.POINTER(Images), c_vp, c_vp]
    L.pcs_render_backward.argtypes = [c_vp, c_vp, ctypes.POINTER(Images), ctypes.POINTER(Grads), c_vp]
    L.pcs_render_backward_noalloc.argtypes = [c_vp, c_vp, ctypes.POINTER(Images), ctypes.POINTER(Grads), c_vp]
    L.pcs_state_bins.argtypes = [c_vp, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp), ctypes.POINTER(c_i64),
                                 ctypes.POINTER(c_vp), ctypes.POINTER(c_i64), ctypes.POINTER(c_vp),
                                 ctypes.POINTER(c_vp)]
    L.pcs_state_status.argtypes = [c_vp, ctypes.POINTER(c_i64), c_vp]
    L.pcs_state_capacity.argtypes = [c_vp, ctypes.POINTER(c_i64)]
    L.pcs_context_set_wait_limit.argtypes = [c_vp, ctypes.c_uint32]
    L.pcs_measure_lds_bandwidth.argtypes = [c_vp, ctypes.POINTER(ctypes.c_double), c_vp]
    L.pcs_pool.argtypes = [c_vp, c_vp, c_vp, ctypes.POINTER(c_i64), c_vp]
    L.pcs_pool_features.argtypes = [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp]
    L.pcs_pool_features_backward.argtypes = [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp]
    L.pcs_up_conv_forward.argtypes = [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_i32, c_i32, c_vp, c_vp]
    L.pcs_up_conv_backward.argtypes = [c_vp, c_vp, c_vp, c_i32, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]
    L.pcs_unet_head_forward.argtypes = [c_vp] * 16
    L.pcs_unet_head_backward.argtypes = [c_vp] * 19
    L.pcs_knn_pca.argtypes = [c_vp, c_vp, c_i64, c_i32, c_f, c_f, c_vp, c_vp, c_vp, c_vp, c_vp]
    L.pcs_shade.argtypes = [c_vp, ctypes.POINTER(Images), ctypes.POINTER(Camera), c_i32,
                            ctypes.POINTER(Light), ctypes.POINTER(c_f * 3), c_vp, c_vp]
    for name in ("pcs_context_create", "pcs_context_set_allocator", "pcs_context_timing", "pcs_context_timing_stages", "pcs_shade",
                 "pcs_context_timings", "pcs_state_create",
                 "pcs_render_forward", "pcs_render_backward", "pcs_render_backward_noalloc",
                 "pcs_state_status", "pcs_state_capacity", "pcs_context_set_wait_limit",
                 "pcs_measure_lds_bandwidth", "pcs_pool", "pcs_pool_features", "pcs_pool_features_backward",
                 "pcs_up_conv_forward", "pcs_up_conv_backward", "pcs_unet_head_forward",
                 "pcs_unet_head_backward",
                 "pcs_state_bins", "pcs_knn_pca", "pcs_voxels_create", "pcs_voxels_destroy", "pcs_voxelize", "pcs_voxels_get",
            "pcs_subm_conv_forward", "pcs_subm_conv_forward_cat", "pcs_subm_conv_backward", "pcs_estimator_head_forward",
            "pcs_estimator_head_backward"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(code: int):
    if code != PCS_OK:
        raise PcsError(code, load().pcs_last_error().decode(errors="replace"))
