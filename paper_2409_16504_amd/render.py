"""Torch-facing binding of the C ABI: device memory and streams come from PyTorch, every step of
the renderer runs in libpcsplat.so.

Gaussians are a dict of planar float32 CUDA tensors: mean (3,n), quat (4,n) (w,x,y,z), scale
(3,n), opacity (n,), rgb (3,n), normal (3,n). Cameras are objects or dicts with T (3x3, row-major
world-to-camera rotation), t (3,), fx, fy, cx, cy, width, height (Section 3.1, Eq. 3-4).
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import torch

from . import _lib
from ._lib import Camera, Gaussians, Grads, Images, Light, Options, check

GAUSS_SHAPES = dict(mean=3, quat=4, scale=3, opacity=None, rgb=3, normal=3)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def camera_struct(cam) -> Camera:
    c = cam if isinstance(cam, dict) else cam.as_dict() if hasattr(cam, "as_dict") else vars(cam)
    s = Camera()
    T = np.asarray(c["T"], dtype=np.float32).reshape(9)
    t = np.asarray(c["t"], dtype=np.float32).reshape(3)
    for k in range(9):
        s.T[k] = float(T[k])
    for k in range(3):
        s.t[k] = float(t[k])
    s.fx, s.fy, s.cx, s.cy = (float(np.float32(c[k])) for k in ("fx", "fy", "cx", "cy"))
    s.width, s.height = int(c["width"]), int(c["height"])
    return s


def default_options(**kw) -> Options:
    o = Options()
    _lib.load().pcs_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                o.bg[i] = float(v[i])
        else:
            setattr(o, k, float(v))
    return o


def check_gaussians(g: dict, device=None) -> int:
    n = g["opacity"].shape[-1]
    for k, rows in GAUSS_SHAPES.items():
        t = g[k]
        want = (n,) if rows is None else (rows, n)
        if tuple(t.shape) != want:
            raise ValueError(f"gaussians[{k!r}] has shape {tuple(t.shape)}, expected {want}")
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"gaussians[{k!r}] must be a contiguous float32 CUDA tensor")
        if device is not None and t.device != device:
            raise ValueError(f"gaussians[{k!r}] is on {t.device}, expected {device}")
    return n


def gaussians_struct(g: dict) -> Gaussians:
    n = check_gaussians(g)
    return Gaussians(n, *(_ptr(g[k]) for k in ("mean", "quat", "scale", "opacity", "rgb", "normal")))


class RenderState:
    """Saved forward data (projection records, sorted lists, tile ranges, transmittance)."""

    def __init__(self, renderer: "Renderer"):
        self.renderer = renderer
        self.handle = ctypes.c_void_p()
        L = _lib.load()
        check(L.pcs_state_create(renderer.ctx, ctypes.byref(self.handle)))
        # held by the instance: module globals may already be cleared when __del__ runs
        self._destroy = L.pcs_state_destroy
        self._finalizing = sys.is_finalizing
        self.keep = None          # tensors the state points at (inputs must stay alive)
        self.shape = None

    def status(self) -> tuple[int, int]:
        """(status code, required instances) of the last frame rendered into this state; waits for
        the current stream. Codes: _lib.PCS_OK, PCS_ERR_CAPACITY (capacity mode: more instances
        than the capacity), PCS_ERR_HIP (the instance ordering failed)."""
        req = ctypes.c_int64()
        with torch.cuda.device(self.renderer.device):
            rc = _lib.load().pcs_state_status(self.handle, ctypes.byref(req), _stream())
        return rc, int(req.value)

    def check(self) -> None:
        """Raise PcsError if the last frame rendered into this state failed."""
        rc, _ = self.status()
        check(rc)

    @property
    def capacity(self) -> int:
        c = ctypes.c_int64()
        check(_lib.load().pcs_state_capacity(self.handle, ctypes.byref(c)))
        return int(c.value)

    def __del__(self):
        # at interpreter exit the HIP runtime may be shutting down; process exit frees the memory
        finalizing = getattr(self, "_finalizing", None)
        if finalizing is None or finalizing():
            return
        if getattr(self, "handle", None) and self.handle.value:
            self._destroy(self.handle)
            self.handle = ctypes.c_void_p()


def _torch_allocator(device: int):
    """Allocator callbacks that take the library's workspace from PyTorch's caching allocator (on
    the stream current when the library asks; the library enqueues on that same stream)."""

    def alloc(nbytes, _user):
        try:
            with torch.cuda.device(device):
                return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except Exception:           # out of memory: the library reports PCS_ERR_OOM
            return None

    def release(ptr, _user):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)

    return _lib.ALLOC_FN(alloc), _lib.FREE_FN(release)


class Renderer:
    """One libpcsplat context on a HIP device. With ``torch_allocator`` (the default) the library's
    workspace comes from PyTorch's caching allocator."""

    def __init__(self, device: int | None = None, torch_allocator: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("the splatting renderer needs a HIP GPU")
        self.device = torch.cuda.current_device() if device is None else int(device)
        L = _lib.load()
        self.ctx = ctypes.c_void_p()
        # held by the instance: module globals may already be cleared when __del__ runs
        self._destroy = L.pcs_context_destroy
        self._finalizing = sys.is_finalizing
        with torch.cuda.device(self.device):
            check(L.pcs_context_create(self.device, ctypes.byref(self.ctx)))
        self._alloc_cbs = None
        if torch_allocator:
            self._alloc_cbs = _torch_allocator(self.device)     # kept alive with the context
            check(L.pcs_context_set_allocator(self.ctx, *self._alloc_cbs, None))

    def close(self) -> None:
        """Release the context's device buffers now (also done when the renderer is collected)."""
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self._destroy(ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        # at interpreter exit the HIP runtime may be shutting down; process exit frees the memory
        finalizing = getattr(self, "_finalizing", None)
        if finalizing is None or finalizing():
            return
        self.close()

    # -- forward --------------------------------------------------------------------------
    def render(self, g: dict, cams: list, opts: Options | None = None, state: RenderState | None = None,
               want=("rgb", "normal", "depth", "alpha"), out: dict | None = None,
               capacity: bool = False) -> dict:
        """Render every camera (all share one width and height). Returns planar float32 images
        rgb (C,3,H,W), normal (C,3,H,W), depth (C,H,W), alpha (C,H,W). ``capacity``: capacity mode
        (no wait on the device; check ``state.status()`` afterwards)."""
        dev = torch.device("cuda", self.device)
        check_gaussians(g, dev)
        cams_c = (Camera * len(cams))(*[camera_struct(c) for c in cams])
        C, W, H = len(cams), cams_c[0].width, cams_c[0].height
        if out is None:
            out = {}
            out["rgb"] = torch.empty((C, 3, H, W), device=dev, dtype=torch.float32)
            if "normal" in want:
                out["normal"] = torch.empty((C, 3, H, W), device=dev, dtype=torch.float32)
            if "depth" in want:
                out["depth"] = torch.empty((C, H, W), device=dev, dtype=torch.float32)
            if "alpha" in want:
                out["alpha"] = torch.empty((C, H, W), device=dev, dtype=torch.float32)
        imgs = Images(_ptr(out["rgb"]), _ptr(out.get("normal")), _ptr(out.get("depth")), _ptr(out.get("alpha")))
        gs = gaussians_struct(g)
        o = opts if opts is not None else default_options()
        if capacity:
            o = Options.from_buffer_copy(o)
            o.flags |= _lib.FLAG_CAPACITY_MODE
        with torch.cuda.device(self.device):
            check(_lib.load().pcs_render_forward(self.ctx, ctypes.byref(gs), cams_c, C, ctypes.byref(o),
                                                 ctypes.byref(imgs), state.handle if state else None,
                                                 _stream()))
        if state is not None:
            state.keep = dict(g)
            state.shape = (C, H, W, gs.n)
        return out

    # -- backward -------------------------------------------------------------------------
    def render_backward(self, state: RenderState, grad_out: dict, want_cov=False) -> dict:
        """Gradients of sum(grad_out * images) with respect to the saved Gaussians (planar)."""
        C, H, W, n = state.shape
        dev = torch.device("cuda", self.device)
        gi = {}
        for k in ("rgb", "normal", "depth", "alpha"):
            t = grad_out.get(k)
            if t is not None:
                t = t.to(device=dev, dtype=torch.float32).contiguous()
            gi[k] = t
        imgs = Images(_ptr(gi["rgb"]), _ptr(gi["normal"]), _ptr(gi["depth"]), _ptr(gi["alpha"]))
        grads = {k: torch.zeros((r, n) if r else (n,), device=dev, dtype=torch.float32)
                 for k, r in dict(mean=3, quat=4, scale=3, opacity=None, rgb=3, normal=3).items()}
        if want_cov:
            grads["cov6"] = torch.zeros((6, n), device=dev, dtype=torch.float32)
        gs = Grads(_ptr(grads["mean"]), _ptr(grads.get("cov6")), _ptr(grads["quat"]), _ptr(grads["scale"]),
                   _ptr(grads["opacity"]), _ptr(grads["rgb"]), _ptr(grads["normal"]))
        with torch.cuda.device(self.device):
            check(_lib.load().pcs_render_backward(self.ctx, state.handle, ctypes.byref(imgs), ctypes.byref(gs),
                                                  _stream()))
        return grads

    # -- parity export ----------------------------------------------------------------------
    def bins(self, state: RenderState) -> dict:
        """Copies of the sorted (key, value) lists, tile ranges, last-contributor index and final
        transmittance of a saved render."""
        L = _lib.load()
        kp, vp, rp, ncp, tp = (ctypes.c_void_p() for _ in range(5))
        m, nt = ctypes.c_int64(), ctypes.c_int64()
        with torch.cuda.device(self.device):
            check(L.pcs_state_bins(state.handle, ctypes.byref(kp), ctypes.byref(vp), ctypes.byref(m),
                                   ctypes.byref(rp), ctypes.byref(nt), ctypes.byref(ncp), ctypes.byref(tp)))
        C, H, W, _ = state.shape
        keys = _copy_device(kp.value, m.value, np.uint64)
        vals = _copy_device(vp.value, m.value, np.uint32)
        ranges = _copy_device(rp.value, 2 * nt.value, np.uint32).reshape(2, nt.value)
        nc = _copy_device(ncp.value, C * H * W, np.int32).reshape(C, H, W)
        tf = _copy_device(tp.value, C * H * W, np.float32).reshape(C, H, W)
        return dict(keys=keys, vals=vals, ranges=ranges, n_contrib=nc, t_final=tf)

    # -- kNN-PCA ------------------------------------------------------------------------------
    def knn_pca(self, xyz: torch.Tensor, k=16, kappa=1.0, floor=0.1, out: dict | None = None,
                nn_dist: bool = False) -> dict:
        """kNN-PCA surfels of the points xyz (3, n); with ``nn_dist`` also each point's distance to
        its nearest other point (key "nn_dist")."""
        n = xyz.shape[1]
        if xyz.shape != (3, n) or xyz.dtype != torch.float32 or not xyz.is_cuda or not xyz.is_contiguous():
            raise ValueError("xyz must be a contiguous float32 CUDA tensor of shape (3, n)")
        dev = xyz.device
        if out is None:
            out = dict(quat=torch.empty((4, n), device=dev), scale=torch.empty((3, n), device=dev),
                       normal=torch.empty((3, n), device=dev))
        if nn_dist and "nn_dist" not in out:
            out["nn_dist"] = torch.empty((n,), device=dev)
        with torch.cuda.device(self.device):
            check(_lib.load().pcs_knn_pca(self.ctx, _ptr(xyz), n, int(k), float(kappa), float(floor),
                                          _ptr(out["quat"]), _ptr(out["scale"]), _ptr(out["normal"]),
                                          _ptr(out["nn_dist"]) if nn_dist else None, _stream()))
        return out

    # -- late shading ---------------------------------------------------------------------------
    def shade(self, images: dict, cams: list, light: dict, bg=(0.0, 0.0, 0.0), out: torch.Tensor | None = None):
        """Blinn-Phong late shading of rendered frames (rgb, normal (C,3,H,W), alpha (C,H,W)) with
        one directional light: dir (towards the light), color, ambient, diffuse, specular,
        shininess. Returns the shaded rgb (C,3,H,W); ``out`` may be images["rgb"]."""
        for k in ("rgb", "normal", "alpha"):
            t = images[k]
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{k} must be a contiguous float32 CUDA tensor")
        cams_c = (Camera * len(cams))(*[camera_struct(c) for c in cams])
        C, W, H = len(cams), cams_c[0].width, cams_c[0].height
        if images["rgb"].shape != (C, 3, H, W) or images["normal"].shape != (C, 3, H, W) or \
                images["alpha"].shape != (C, H, W):
            raise ValueError("image shapes do not match the cameras")
        if out is None:
            out = torch.empty_like(images["rgb"])
        imgs = Images(_ptr(images["rgb"]), _ptr(images["normal"]), None, _ptr(images["alpha"]))
        lt = Light((ctypes.c_float * 3)(*light["dir"]), (ctypes.c_float * 3)(*light.get("color", (1.0, 1.0, 1.0))),
                   float(light.get("ambient", 0.1)), float(light.get("diffuse", 0.7)),
                   float(light.get("specular", 0.2)), float(light.get("shininess", 16.0)))
        bgc = (ctypes.c_float * 3)(*bg)
        with torch.cuda.device(self.device):
            check(_lib.load().pcs_shade(self.ctx, ctypes.byref(imgs), cams_c, C, ctypes.byref(lt), ctypes.byref(bgc),
                                        _ptr(out), _stream()))
        return out

    def lds_bandwidth(self) -> float:
        """Measured LDS read bandwidth of the device, GB/s."""
        v = ctypes.c_double()
        with torch.cuda.device(self.device):
            check(_lib.load().pcs_measure_lds_bandwidth(self.ctx, ctypes.byref(v), _stream()))
        return float(v.value)

    def set_wait_limit(self, rounds: int) -> None:
        """Bound of the ordering kernels' look-back waits (0: the default); see the C header."""
        check(_lib.load().pcs_context_set_wait_limit(self.ctx, int(rounds)))

    # -- timing -------------------------------------------------------------------------------
    def timing(self, enable=True, stages=None):
        """Enable per-stage HIP-event timing (resetting the totals); ``stages`` limits the events to
        the named stages."""
        if stages is None or not enable:
            check(_lib.load().pcs_context_timing(self.ctx, int(enable)))
        else:
            mask = 0
            for st in stages:
                mask |= 1 << _lib.STAGES.index(st)
            check(_lib.load().pcs_context_timing_stages(self.ctx, mask))

    def timings(self) -> dict:
        n = len(_lib.STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        with torch.cuda.device(self.device):
            check(_lib.load().pcs_context_timings(self.ctx, ms, cnt, n, _stream()))
        return {s: (ms[i], cnt[i]) for i, s in enumerate(_lib.STAGES)}


def _copy_device(ptr: int, count: int, dtype) -> np.ndarray:
    """Copy `count` items of a library-owned device buffer to host (via a torch byte tensor)."""
    dtype = np.dtype(dtype)
    out = np.empty(count, dtype=dtype)
    if count == 0:
        return out
    nbytes = count * dtype.itemsize
    host = torch.empty(nbytes, dtype=torch.uint8)
    torch.cuda.synchronize()
    _hip_memcpy_d2h(host.data_ptr(), ptr, nbytes)
    out[:] = host.numpy().view(dtype)
    return out


_hip = None


def _hip_memcpy_d2h(dst: int, src: int, nbytes: int):
    """hipMemcpy through the HIP runtime already loaded by torch (same soname)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    rc = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes), 2)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy device-to-host failed with {rc}")


class RenderFunction(torch.autograd.Function):
    """Differentiable render: images from (mean, quat, scale, opacity, rgb, normal); the backward
    is the hand-written adjoint kernel of libpcsplat. All four outputs (rgb, normal, depth, alpha)
    carry gradients. The adjoint reads the Gaussians the forward rendered: they are saved for
    backward, so modifying one in place in between makes autograd raise."""

    @staticmethod
    def forward(ctx, mean, quat, scale, opacity, rgb, normal, renderer, cams, opts):
        g = dict(mean=mean.contiguous(), quat=quat.contiguous(), scale=scale.contiguous(),
                 opacity=opacity.contiguous(), rgb=rgb.contiguous(), normal=normal.contiguous())
        state = RenderState(renderer)
        out = renderer.render(g, cams, opts, state=state)
        ctx.save_for_backward(*(g[k] for k in ("mean", "quat", "scale", "opacity", "rgb", "normal")))
        ctx.renderer = renderer
        ctx.state = state
        return out["rgb"], out["normal"], out["depth"], out["alpha"]

    @staticmethod
    def backward(ctx, g_rgb, g_nrm, g_depth, g_alpha):
        ctx.saved_tensors          # raises if a saved Gaussian tensor was modified in place
        grads = ctx.renderer.render_backward(ctx.state, dict(rgb=g_rgb, normal=g_nrm, depth=g_depth,
                                                             alpha=g_alpha))
        ctx.state = None
        return (grads["mean"], grads["quat"], grads["scale"], grads["opacity"], grads["rgb"],
                grads["normal"], None, None, None)


def render_autograd(renderer: Renderer, g: dict, cams: list, opts: Options | None = None):
    """(rgb, normal, depth, alpha) with gradients flowing to the six Gaussian tensors."""
    return RenderFunction.apply(g["mean"], g["quat"], g["scale"], g["opacity"], g["rgb"], g["normal"],
                                renderer, cams, opts)
