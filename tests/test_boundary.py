"""Host-side checks of the C ABI: the library loads, exports every declared entry point, and
rejects bad arguments with status codes (no kernel is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcsplat.h")


@pytest.fixture(scope="module")
def L():
    from paper_2409_16504_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2409_16504_amd.build import build
        build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pcs_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    from paper_2409_16504_amd import _lib
    assert set(_lib.EXPORTED) == set(names)


def test_options_default(L):
    from paper_2409_16504_amd import _lib
    o = _lib.Options()
    L.pcs_options_default(ctypes.byref(o))
    import numpy as np
    assert (o.z_near, o.sigma_cut) == (np.float32(0.2), 3.0)
    assert o.lowpass == np.float32(0.3) and o.alpha_min == np.float32(1 / 255)
    assert o.alpha_max == np.float32(0.99) and o.t_eps == np.float32(1e-4)
    assert list(o.bg) == [0.0, 0.0, 0.0]


def test_null_arguments_are_rejected(L):
    from paper_2409_16504_amd import _lib
    assert L.pcs_render_forward(None, None, None, 0, None, None, None, None) == _lib.PCS_ERR_INVALID_ARG
    assert b"context" in L.pcs_last_error()
    assert L.pcs_render_backward(None, None, None, None, None) == _lib.PCS_ERR_INVALID_ARG
    assert L.pcs_state_bins(None, None, None, None, None, None, None, None) == _lib.PCS_ERR_INVALID_ARG
    assert L.pcs_knn_pca(None, None, 0, 16, 1.0, 0.1, None, None, None, None, None) == _lib.PCS_ERR_INVALID_ARG
    assert L.pcs_context_create(0, None) == _lib.PCS_ERR_INVALID_ARG
    assert L.pcs_context_timing(None, 1) == _lib.PCS_ERR_INVALID_ARG
    assert L.pcs_state_create(None, None) == _lib.PCS_ERR_INVALID_ARG
    L.pcs_state_destroy(None)
    L.pcs_context_destroy(None)


def test_context_without_gpu_reports_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2409_16504_amd import _lib
    h = ctypes.c_void_p()
    rc = L.pcs_context_create(0, ctypes.byref(h))
    assert rc in (_lib.PCS_ERR_HIP, _lib.PCS_ERR_INVALID_ARG)
    assert h.value is None
    assert len(L.pcs_last_error()) > 0


def test_renderer_requires_gpu_and_library():
    import torch
    import paper_2409_16504_amd as P
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        P.Renderer(0)


def test_python_binding_surface():
    """The binding modules import without a GPU and expose the documented names."""
    from paper_2409_16504_amd import estimator, render
    for name in ("build", "mean_neighbours", "arrays"):
        assert callable(getattr(estimator.Voxels, name)), name
    for name in ("adaptive_grid", "conv_forward", "conv_backward", "head_forward", "head_backward",
                 "train_step", "ssim", "psnr"):
        assert callable(getattr(estimator, name)), name
    for name in ("render", "render_backward", "bins", "knn_pca", "timing", "timings"):
        assert callable(getattr(render.Renderer, name)), name
