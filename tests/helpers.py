"""Shared helpers of the GPU parity tests (inputs and comparisons; no renderer arithmetic)."""
from __future__ import annotations

import functools

import numpy as np

from synthetic import look_at_camera, make_surface, random_gaussians, CONFIG_SEEDS


def to_torch(g: dict, device="cuda"):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(device) for k, v in g.items()}


def c1_scene():
    """2,000 random ellipsoids, camera at (0,0,3) looking at the origin, 128x128, 60 deg FOV."""
    rng = np.random.default_rng(CONFIG_SEEDS[1])
    return random_gaussians(2000, rng), [look_at_camera([0, 0, 3], width=128, height=128)]


@functools.lru_cache(maxsize=4)
def surface_gaussians(n: int, seed: int, kappa: float = 1.0):
    """Procedural-surface cloud (quantised to the 1024^3 lattice, value-noise colour) with
    kNN-PCA ellipsoids computed by the oracle (k = 16), opacity 0.9."""
    from oracle import knn_pca as kp
    _, p, rgb = make_surface(n, seed, quantize=True)
    est = kp.knn_pca(p, k=16, kappa=kappa)
    return dict(mean=p, quat=est["quat"].astype(np.float32), scale=est["scale"].astype(np.float32),
                opacity=np.full(n, 0.9, np.float32), rgb=rgb, normal=est["normal"].astype(np.float32))


def image_errors(gpu: dict, ref: dict, cam_index=None):
    """Max-abs differences on unflagged pixels for rgb/normal/depth/alpha and the flagged count."""
    flags = ref["flags"] != 0
    out = {"flagged": int(flags.sum())}
    for k in ("rgb", "normal"):
        d = np.abs(gpu[k].astype(np.float64) - ref[k])
        d = np.where(flags[:, None], 0.0, d)
        out[k] = float(d.max())
    for k in ("depth", "alpha"):
        d = np.abs(gpu[k].astype(np.float64) - ref[k])
        out[k] = float(np.where(flags, 0.0, d).max())
    return out
