"""FP64 reference of late shading from the rendered normal map (test infrastructure only).

Section 3.1 renders a normal map by blending the per-splat normals like colours and shades it in a
pixel shader afterwards; the paper fixes no shading model. Reading used here (Blinn-Phong, one
directional light), per pixel of camera C:

* fg = rgb - T * bg is the blended (premultiplied) albedo, alpha = 1 - T its coverage;
* n = normal / |normal| (world space); pixels with |normal| = 0 keep only the ambient term;
* v = direction from the pixel towards the camera: the pixel ray (x + 0.5 - cx) / fx,
  (y + 0.5 - cy) / fy, 1 in camera coordinates, rotated to world by T^T, normalised and negated;
* l = the unit direction towards the light, h = (l + v) / |l + v|;
* out = fg * (ambient + diffuse * max(0, n.l)) * light
        + alpha * specular * max(0, n.h)^shininess * light + T * bg.
"""
from __future__ import annotations

import numpy as np


def pixel_view_dirs(cam, W: int, H: int) -> np.ndarray:
    """(3, H, W) unit vectors from each pixel centre towards the camera, world frame."""
    c = cam.as_dict() if hasattr(cam, "as_dict") else cam
    T = np.asarray(c["T"], np.float64).reshape(3, 3)
    x = (np.arange(W) + 0.5 - float(c["cx"])) / float(c["fx"])
    y = (np.arange(H) + 0.5 - float(c["cy"])) / float(c["fy"])
    ray = np.stack(np.broadcast_arrays(x[None, :], y[:, None], np.ones((H, W))), 0)   # camera frame
    d = np.einsum("ji,jhw->ihw", T, ray)                                                 # T^T ray
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return -d


def shade(rgb, normal, alpha, cams, light: dict, bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    """rgb, normal (C, 3, H, W); alpha (C, H, W); light: dir (towards the light), color, ambient,
    diffuse, specular, shininess. Returns (C, 3, H, W) FP64."""
    rgb = np.asarray(rgb, np.float64)
    nrm = np.asarray(normal, np.float64)
    a = np.asarray(alpha, np.float64)
    C, _, H, W = rgb.shape
    bgv = np.asarray(bg, np.float64)[:, None, None]
    l = np.asarray(light["dir"], np.float64)
    l = l / np.linalg.norm(l)
    col = np.asarray(light["color"], np.float64)[:, None, None]
    out = np.empty_like(rgb)
    for ci in range(C):
        T = 1.0 - a[ci]
        fg = rgb[ci] - T[None] * bgv
        ln = np.linalg.norm(nrm[ci], axis=0)
        has = ln > 0
        n = np.where(has[None], nrm[ci] / np.where(has, ln, 1.0)[None], 0.0)
        v = pixel_view_dirs(cams[ci], W, H)
        h = l[:, None, None] + v
        h /= np.linalg.norm(h, axis=0, keepdims=True)
        ndl = np.maximum(np.einsum("k,khw->hw", l, n), 0.0)
        ndh = np.maximum(np.einsum("khw,khw->hw", h, n), 0.0)
        spec = np.where(has, ndh ** float(light["shininess"]), 0.0)
        out[ci] = (fg * (float(light["ambient"]) + float(light["diffuse"]) * ndl)[None] * col
                   + (a[ci] * float(light["specular"]) * spec)[None] * col + T[None] * bgv)
    return out
