"""FP64 reference of the point-to-ellipsoid estimator (test infrastructure only).

Section 3.2 voxelises the cloud, feeds colour and coordinate residuals to a sparse 3D
convolutional network and predicts per-point Gaussian parameters with a shared head. The
estimator built here is the configuration-4 stand-in for it: eight submanifold 3x3x3 convolutions
with ReLU and a per-voxel linear head. This module defines each step plainly:

* ``voxelize``: voxel coordinate c = clamp(floor((p + 1) * G/2), 0, G-1) on a G^3 grid over
  [-1,1]^3 (G = 1024 is the 10-bit quantisation of Section 3.3); unique voxels in ascending linear
  key (x << 20 | y << 10 | z); per voxel the mean colour, the mean residual
  (p + 1) * G/2 - (c + 0.5) (the coordinate residual of Section 3.2) and the mean absolute
  position p of its points (Section 3.2 feeds coordinates, colour and residuals). The cloud's
  coordinates are FP32, so the voxel decision floor is taken on the FP32 sum p + 1 (times the
  power of two G/2, exact); the residual is FP64.
* ``kernel_map``: for voxel i and offset k = 9 (dx + 1) + 3 (dy + 1) + (dz + 1) the index of the
  voxel at c_i + (dx, dy, dz), or -1.
* ``subm_conv``: y_i = b + sum_k W_k^T x_{nbr_k(i)} over present neighbours (submanifold: outputs
  only at active sites), optional ReLU.
* ``head``: raw = W_h^T f + b_h per voxel; scale = (2/G) exp(raw[0:3]) (voxel edge times exp); q = normalise(raw[3:7] +
  (1, 0, 0, 0)); opacity = sigmoid(raw[7]); rgb = colour + raw[8:11]; normal = the rotated axis of
  the smallest scale, oriented away from the cloud centroid.
"""
from __future__ import annotations

import numpy as np

GRID = 1024
VOXEL = 2.0 / GRID
OFFSETS = np.array([(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)])


def voxel_key(c: np.ndarray) -> np.ndarray:
    """Linear key of integer coordinates c (n, 3)."""
    c = c.astype(np.int64)
    return (c[:, 0] << 20) | (c[:, 1] << 10) | c[:, 2]


def voxelize(xyz: np.ndarray, rgb: np.ndarray, grid: int = GRID) -> dict:
    if grid < 2 or grid > GRID or grid & (grid - 1):
        raise ValueError("grid must be a power of two in [2, 1024]")
    p32 = np.asarray(xyz, np.float32).T                     # (n, 3)
    p = p32.astype(np.float64)
    c = np.clip(np.floor((p32 + np.float32(1.0)).astype(np.float64) * (grid / 2)), 0, grid - 1).astype(np.int64)
    keys = voxel_key(c)
    ukeys, inv = np.unique(keys, return_inverse=True)
    V = ukeys.size
    coords = np.stack([(ukeys >> 20) & 1023, (ukeys >> 10) & 1023, ukeys & 1023], axis=1)
    count = np.bincount(inv, minlength=V).astype(np.float64)
    col = np.stack([np.bincount(inv, weights=np.asarray(rgb, np.float64)[a], minlength=V) for a in range(3)], 1)
    res_p = (p + 1.0) * (grid / 2) - (c + 0.5)
    res = np.stack([np.bincount(inv, weights=res_p[:, a], minlength=V) for a in range(3)], 1)
    pos = np.stack([np.bincount(inv, weights=p[:, a], minlength=V) for a in range(3)], 1)
    return dict(coords=coords, keys=ukeys, point_voxel=inv.astype(np.int64),
                color=col / count[:, None], residual=res / count[:, None], position=pos / count[:, None],
                count=count)


def kernel_map(coords: np.ndarray, grid: int = GRID) -> np.ndarray:
    """nbr (27, V) int64: index of the neighbour at each offset or -1."""
    keys = voxel_key(coords)
    order = np.argsort(keys)
    sk = keys[order]
    V = coords.shape[0]
    nbr = np.full((27, V), -1, np.int64)
    for k, off in enumerate(OFFSETS):
        q = coords + off
        ok = np.all((q >= 0) & (q < grid), axis=1)
        qk = voxel_key(np.clip(q, 0, grid - 1))
        pos = np.searchsorted(sk, qk)
        pos = np.minimum(pos, V - 1)
        hit = ok & (sk[pos] == qk)
        nbr[k, hit] = order[pos[hit]]
    return nbr


def subm_conv(x: np.ndarray, W: np.ndarray, b: np.ndarray, nbr: np.ndarray, relu: bool) -> np.ndarray:
    """x (V, Cin), W (27, Cin, Cout), b (Cout,) -> (V, Cout), all FP64."""
    V = x.shape[0]
    y = np.tile(np.asarray(b, np.float64), (V, 1))
    for k in range(27):
        idx = nbr[k]
        ok = idx >= 0
        y[ok] += np.asarray(x, np.float64)[idx[ok]] @ np.asarray(W[k], np.float64)
    return np.maximum(y, 0.0) if relu else y


def head(f: np.ndarray, Wh: np.ndarray, bh: np.ndarray, color: np.ndarray, points: np.ndarray,
         point_voxel: np.ndarray, grid: int = GRID) -> dict:
    """Per-point Gaussian parameters from voxel features f (V, C); planar outputs like the renderer."""
    raw = np.asarray(f, np.float64) @ np.asarray(Wh, np.float64) + np.asarray(bh, np.float64)
    scale = (2.0 / grid) * np.exp(raw[:, 0:3])
    q = raw[:, 3:7] + np.array([1.0, 0, 0, 0])
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    opac = 1.0 / (1.0 + np.exp(-raw[:, 7]))
    drgb = raw[:, 8:11]
    pv = point_voxel
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)
    axis = np.argmin(scale, axis=1)
    n_v = R[np.arange(R.shape[0]), :, axis]                  # column of the smallest scale
    P = np.asarray(points, np.float64).T
    centroid = P.mean(axis=0)
    n_p = n_v[pv]
    flip = np.einsum("ni,ni->n", n_p, P - centroid) < 0
    n_p[flip] *= -1
    return dict(raw=raw, quat=q[pv].T, scale=scale[pv].T, opacity=opac[pv],
                rgb=(np.asarray(color, np.float64).T + drgb[pv]).T, normal=n_p.T)


def subm_conv_backward(x: np.ndarray, W: np.ndarray, nbr: np.ndarray, dy: np.ndarray):
    """Adjoint of ``subm_conv`` without ReLU for the upstream gradient dy (V, Cout):
    dW_k = x[nbr_k]^T dy over present neighbours, dx_j = sum over (k, i) with nbr_k(i) = j of
    W_k dy_i, db = sum_i dy_i. FP64."""
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    dW = np.zeros(W.shape)
    dx = np.zeros(x.shape)
    for k in range(27):
        idx = nbr[k]
        ok = idx >= 0
        dW[k] = x[idx[ok]].T @ dy[ok]
        np.add.at(dx, idx[ok], dy[ok] @ np.asarray(W[k], np.float64).T)
    return dx, dW, dy.sum(axis=0)


def head_torch(f, Wh, bh, color, point_voxel, grid: int = GRID):
    """The head of ``head`` (without the normal) in FP64 torch ops, so that autograd gives its
    adjoint: returns per-point quat (4,n), scale (3,n), opacity (n,), rgb (3,n)."""
    import torch
    raw = f @ Wh + bh
    scale = (2.0 / grid) * torch.exp(raw[:, 0:3])
    q = raw[:, 3:7] + torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=raw.dtype)
    q = q / torch.linalg.norm(q, dim=1, keepdim=True)
    opac = torch.sigmoid(raw[:, 7])
    pv = torch.as_tensor(point_voxel)
    return q[pv].T, scale[pv].T, opac[pv], color + raw[pv, 8:11].T
