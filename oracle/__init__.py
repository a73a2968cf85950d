"""CPU oracle of the splatting renderer: test infrastructure, never part of the product path.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package. It
shares no code with the GPU library. It implements, plainly and slowly, what the paper's renderer
computes (Section 3.1):

* projection of each ellipsoid (Sigma = R diag(s^2) R^T, Eq. 3 view transform, Eq. 4 EWA screen
  covariance) -- in FP64, and as the exact FP32 operation sequence that fixes the binning;
* the 3-sigma splat boundary, (tile | depth) keys and their lexicographic sort;
* front-to-back alpha blending of RGB, normal and depth (Eq. 1 with the opacity of Eq. 2);
* the FP64 adjoint of the render (``backward``);
* the FP64 pull-back of screen-space gradients to the Gaussian parameters alone (``pull_back``);
* kNN-PCA surfel ellipsoids (``knn_pca``), a tiny-scene brute-force renderer (``brute``), the
  sparse-convolution estimator reference (``estimator``), the image metrics PSNR and SSIM
  (``metrics``) and a second, numpy.float32 emulation of the exact-FP32 projection
  (``emulate32``), in their own modules.

``render(..., mode="ref")`` composites in FP64 from the exact-FP32 projection (the image the GPU
is held to); ``mode="f64"`` runs every step in FP64.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build as _build

DEFAULT_OPTIONS = dict(z_near=0.2, lowpass=0.3, sigma_cut=3.0, alpha_min=1.0 / 255.0,
                       alpha_max=0.99, t_eps=1e-4, bg=(0.0, 0.0, 0.0))

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            _build()
        _lib = ctypes.CDLL(LIB)
        _setup(_lib)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _setup(L):
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.orc_project_f32.argtypes = [i64] + [vp] * 7 + [i32, i32, i32, vp] + [vp] * 10
    L.orc_project_f32.restype = None
    L.orc_project_f64.argtypes = [i64] + [vp] * 6 + [i32, i32, i32, vp] + [vp] * 12
    L.orc_cov3d_f64.argtypes = [i64, vp, vp, vp]
    L.orc_cov3d_f64.restype = None
    L.orc_project_f64.restype = None
    L.orc_bin.argtypes = [i64, i32, i32, i32, vp, vp, vp, vp, vp]
    L.orc_bin.restype = i64
    L.orc_composite.argtypes = ([i64] + [vp] * 9 + [i64, vp, vp, ctypes.c_uint64, i32, i32, i32, vp,
                                vp, i64] + [vp] * 9)
    L.orc_composite.restype = i64
    L.orc_backward.argtypes = ([i64] + [vp] * 7 + [i32, vp, i32, i32, i32, vp, vp, vp, vp, vp, i64, vp,
                               vp, vp])
    L.orc_backward.restype = None
    L.orc_pull_back.argtypes = [i64] + [vp] * 8
    L.orc_pull_back.restype = None


def options_vector(opts=None) -> np.ndarray:
    o = dict(DEFAULT_OPTIONS)
    if opts:
        o.update(opts)
    return np.array([o["z_near"], o["lowpass"], o["sigma_cut"], o["alpha_min"], o["alpha_max"],
                     o["t_eps"], *o["bg"]], dtype=np.float32)


def camera_vector(cam, dtype=np.float32) -> np.ndarray:
    c = cam if isinstance(cam, dict) else cam.as_dict()
    v = np.concatenate([np.asarray(c["T"], dtype=np.float32).reshape(9),
                        np.asarray(c["t"], dtype=np.float32).reshape(3),
                        np.array([c["fx"], c["fy"], c["cx"], c["cy"]], dtype=np.float32)])
    return v.astype(dtype)


def _cam_wh(cam):
    c = cam if isinstance(cam, dict) else cam.as_dict()
    return int(c["width"]), int(c["height"])


def _f32(g, k):
    return np.ascontiguousarray(g[k], dtype=np.float32)


def project_f32(g: dict, cam, opts=None, tile=16) -> dict:
    """Exact-FP32 projection of every Gaussian through one camera."""
    n = g["opacity"].shape[-1]
    W, H = _cam_wh(cam)
    out = {k: np.zeros(n, np.float32) for k in ("u", "v", "z", "A", "B", "C")}
    ext = np.zeros((2, n), np.float32)
    out["valid"] = np.zeros(n, np.uint8)
    out["rect"] = np.zeros((4, n), np.int32)
    out["count"] = np.zeros(n, np.uint32)
    arrs = [_f32(g, k) for k in ("mean", "quat", "scale", "opacity", "rgb", "normal")]
    lib().orc_project_f32(n, *[_p(a) for a in arrs], _p(camera_vector(cam)), W, H, tile,
                          _p(options_vector(opts)), _p(out["valid"]), _p(out["u"]), _p(out["v"]),
                          _p(out["z"]), _p(out["A"]), _p(out["B"]), _p(out["C"]), _p(ext),
                          _p(out["rect"]), _p(out["count"]))
    out["ex"], out["ey"] = ext[0], ext[1]
    return out


def project_f64(g: dict, cam, opts=None, tile=16, cov6=None) -> dict:
    """FP64 projection; parameters are read as float64 (``cov6`` overrides quat/scale)."""
    n = g["opacity"].shape[-1]
    W, H = _cam_wh(cam)
    out = {k: np.zeros(n, np.float64) for k in ("u", "v", "z", "A", "B", "C")}
    ext = np.zeros((2, n), np.float64)
    out["valid"] = np.zeros(n, np.uint8)
    out["rect"] = np.zeros((4, n), np.int32)
    out["count"] = np.zeros(n, np.uint32)
    out["cov2d"] = np.zeros((3, n), np.float64)
    out["zf"] = np.zeros(n, np.float32)      # FP32 depth of the exact projection: the depth order
    d = {k: np.ascontiguousarray(g[k], dtype=np.float64) for k in ("mean", "quat", "scale", "opacity")}
    c6 = None if cov6 is None else np.ascontiguousarray(cov6, dtype=np.float64)
    lib().orc_project_f64(n, _p(d["mean"]), _p(d["quat"]), _p(d["scale"]), _p(c6), _p(d["opacity"]),
                          _p(camera_vector(cam, np.float64)), W, H, tile, _p(options_vector(opts)),
                          _p(out["valid"]), _p(out["u"]), _p(out["v"]), _p(out["z"]), _p(out["A"]),
                          _p(out["B"]), _p(out["C"]), _p(ext), _p(out["rect"]),
                          _p(out["count"]), _p(out["cov2d"]), _p(out["zf"]))
    out["ex"], out["ey"] = ext[0], ext[1]
    return out


def covariance_f64(quat: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """Sigma = R diag(s^2) R^T of every Gaussian, shape (n, 3, 3), FP64."""
    n = quat.shape[-1]
    q = np.ascontiguousarray(quat, dtype=np.float64)
    s = np.ascontiguousarray(scale, dtype=np.float64)
    out = np.zeros((9, n))
    lib().orc_cov3d_f64(n, _p(q), _p(s), _p(out))
    return out.T.reshape(n, 3, 3)


def bin_sorted(projs: list, n: int, W: int, H: int, tile=16):
    """Sorted (key, value) lists of all cameras from their projections (list, one per camera)."""
    TX, TY = (W + tile - 1) // tile, (H + tile - 1) // tile
    C = len(projs)
    valid = np.ascontiguousarray(np.stack([p["valid"] for p in projs]))
    zf = np.ascontiguousarray(np.stack([np.asarray(p["zf"] if "zf" in p else p["z"], np.float32)
                                        for p in projs]))
    rect = np.ascontiguousarray(np.stack([p["rect"] for p in projs]))
    m = int(sum(int(p["count"].astype(np.int64).sum()) for p in projs))
    keys = np.zeros(m, np.uint64)
    vals = np.zeros(m, np.uint32)
    got = lib().orc_bin(n, C, TX * TY, TX, _p(valid), _p(zf), _p(rect), _p(keys), _p(vals))
    assert got == m
    return keys, vals


def tile_ranges(keys: np.ndarray, n_tiles_total: int) -> np.ndarray:
    """(start, end) of every tile's run in a sorted key list; empty tiles are (0, 0)."""
    rng = np.zeros((2, n_tiles_total), np.uint32)
    if keys.size == 0:
        return rng
    t = (keys >> np.uint64(32)).astype(np.int64)
    first = np.ones(t.size, bool)
    first[1:] = t[1:] != t[:-1]
    last = np.ones(t.size, bool)
    last[:-1] = t[1:] != t[:-1]
    idx = np.arange(t.size)
    rng[0, t[first]] = idx[first]
    rng[1, t[last]] = idx[last] + 1
    return rng


def render(g: dict, cams: list, opts=None, mode="ref", tile=16, pixels=None, cov6=None,
           margin_vs=None) -> dict:
    """Render every camera. Returns planar float64 images [C][3][H][W] / [C][H][W], the final
    transmittance, n_contrib, margin flags, the sorted key/value lists and the visit count.
    ``margin_vs`` ("ref" or "f64"): also flag the pixels where the other projection's quadratic
    forms could take a decision differently (the margins widen by the difference between the two);
    the images are unchanged."""
    n = g["opacity"].shape[-1]
    W, H = _cam_wh(cams[0])
    TX, TY = (W + tile - 1) // tile, (H + tile - 1) // tile
    ntiles = TX * TY
    ov = options_vector(opts)
    if mode == "ref":
        projs = [project_f32(g, c, opts, tile) for c in cams]
    elif mode == "f64":
        projs = [project_f64(g, c, opts, tile, cov6=cov6) for c in cams]
    else:
        raise ValueError(mode)
    alts = [None] * len(cams)
    if margin_vs is not None:
        other = [project_f32(g, c, opts, tile) if margin_vs == "ref" else project_f64(g, c, opts, tile, cov6=cov6)
                 for c in cams]
        alts = [np.ascontiguousarray(np.stack([np.asarray(o[k], np.float64) for k in ("u", "v", "A", "B", "C")]))
                for o in other]
    keys, vals = bin_sorted(projs, n, W, H, tile)
    C = len(cams)
    HW = W * H
    res = dict(rgb=np.zeros((C, 3, H, W)), normal=np.zeros((C, 3, H, W)), depth=np.zeros((C, H, W)),
               alpha=np.zeros((C, H, W)), T=np.zeros((C, H, W)), n_contrib=np.zeros((C, H, W), np.int32),
               flags=np.zeros((C, H, W), np.uint8), keys=keys, vals=vals, proj=projs, visits=0, blends=0)
    opac = np.ascontiguousarray(g["opacity"], dtype=np.float64)
    rgb = np.ascontiguousarray(g["rgb"], dtype=np.float64)
    nrm = np.ascontiguousarray(g["normal"], dtype=np.float64)
    tile_id = (keys >> np.uint64(32)).astype(np.int64)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
    for ci in range(C):
        p = projs[ci]
        lo = np.searchsorted(tile_id, ci * ntiles)
        hi = np.searchsorted(tile_id, (ci + 1) * ntiles)
        k_c = np.ascontiguousarray(keys[lo:hi])
        v_c = np.ascontiguousarray(vals[lo:hi])
        sp = {k: np.ascontiguousarray(p[k], dtype=np.float64) for k in ("u", "v", "A", "B", "C", "z")}
        o_rgb = np.zeros((3, HW))
        o_nrm = np.zeros((3, HW))
        o_d = np.zeros(HW)
        o_a = np.zeros(HW)
        o_T = np.ones(HW)
        o_nc = np.zeros(HW, np.int32)
        o_f = np.zeros(HW, np.uint8)
        o_b = np.zeros(1, np.int64)
        visits = lib().orc_composite(n, _p(sp["u"]), _p(sp["v"]), _p(sp["A"]), _p(sp["B"]), _p(sp["C"]),
                                     _p(sp["z"]), _p(opac), _p(rgb), _p(nrm), int(hi - lo), _p(k_c),
                                     _p(v_c), ci * ntiles, W, H, tile, _p(ov), _p(pix),
                                     0 if pix is None else pix.size, _p(o_rgb), _p(o_nrm), _p(o_d),
                                     _p(o_a), _p(o_T), _p(o_nc), _p(o_f), _p(o_b), _p(alts[ci]))
        res["rgb"][ci] = o_rgb.reshape(3, H, W)
        res["normal"][ci] = o_nrm.reshape(3, H, W)
        res["depth"][ci] = o_d.reshape(H, W)
        res["alpha"][ci] = o_a.reshape(H, W)
        res["T"][ci] = o_T.reshape(H, W)
        res["n_contrib"][ci] = o_nc.reshape(H, W)
        res["flags"][ci] = o_f.reshape(H, W)
        res["visits"] += int(visits)
        res["blends"] += int(o_b[0])
    return res


GRAD_LAYOUT = dict(mean=(0, 3), cov6=(3, 9), quat=(9, 13), scale=(13, 16), opacity=(16, 17),
                   rgb=(17, 20), normal=(20, 23))


def backward(g: dict, cams: list, grad_out: dict, opts=None, tile=16, cov6=None, sabs_for=-1):
    """FP64 adjoint of the FP64 render. ``grad_out`` holds rgb [C][3][H][W], normal [C][3][H][W]
    and depth [C][H][W], optionally alpha [C][H][W]. Returns (grads, sabs, signature): dicts keyed like GRAD_LAYOUT with
    planar (k, n) float64 arrays; ``sabs`` is the sum over pixels of each per-pixel term's absolute
    value (``sabs_for``: -1 every Gaussian, i only Gaussian i, -2 none)."""
    n = g["opacity"].shape[-1]
    W, H = _cam_wh(cams[0])
    d = {k: np.ascontiguousarray(g[k], dtype=np.float64)
         for k in ("mean", "quat", "scale", "opacity", "rgb", "normal")}
    c6 = None if cov6 is None else np.ascontiguousarray(cov6, dtype=np.float64)
    camv = np.ascontiguousarray(np.stack([camera_vector(c, np.float64) for c in cams]))
    gr = np.ascontiguousarray(grad_out["rgb"], dtype=np.float64)
    gn = np.ascontiguousarray(grad_out["normal"], dtype=np.float64)
    gd = np.ascontiguousarray(grad_out["depth"], dtype=np.float64)
    ga = grad_out.get("alpha")
    ga = None if ga is None else np.ascontiguousarray(ga, dtype=np.float64)
    grad = np.zeros((23, n))
    sabs = np.zeros((23, n))
    sig = np.zeros(1, np.uint64)
    lib().orc_backward(n, _p(d["mean"]), _p(d["quat"]), _p(d["scale"]), _p(c6), _p(d["opacity"]),
                       _p(d["rgb"]), _p(d["normal"]), len(cams), _p(camv), W, H, tile,
                       _p(options_vector(opts)), _p(gr), _p(gn), _p(gd), _p(ga), int(sabs_for), _p(grad),
                       _p(sabs), _p(sig))
    split = lambda a: {k: a[lo:hi] for k, (lo, hi) in GRAD_LAYOUT.items()}  # noqa: E731
    return split(grad), split(sabs), int(sig[0])


SCREEN_GRADS = ("u", "v", "A", "B", "C", "opacity", "depth", "r", "g", "b", "nx", "ny", "nz")


def pull_back(g: dict, cam, sgrad: np.ndarray, opts=None, cov6=None) -> dict:
    """FP64 chain of screen-space gradients ``sgrad`` [13][n] (order SCREEN_GRADS: the splat's pixel
    position, conic, opacity, depth, colour and normal in camera ``cam``) to the Gaussian
    parameters; a dict keyed like GRAD_LAYOUT of planar (k, n) arrays."""
    n = g["opacity"].shape[-1]
    d = {k: np.ascontiguousarray(g[k], dtype=np.float64) for k in ("mean", "quat", "scale")}
    c6 = None if cov6 is None else np.ascontiguousarray(cov6, dtype=np.float64)
    sg = np.ascontiguousarray(sgrad, dtype=np.float64).reshape(len(SCREEN_GRADS), n)
    grad = np.zeros((23, n))
    lib().orc_pull_back(n, _p(d["mean"]), _p(d["quat"]), _p(d["scale"]), _p(c6),
                        _p(camera_vector(cam, np.float64)), _p(options_vector(opts)), _p(sg), _p(grad))
    return {k: grad[lo:hi] for k, (lo, hi) in GRAD_LAYOUT.items()}
