"""FP64 reference of the paper's UNet-like point-to-ellipsoid estimator (test infrastructure only).

Section 3.2 (and its network figure) builds the estimator from:

* ``pool``: the encoder's 2x2x2 downsampling of the sparse voxel grid: every parent voxel (child
  coordinates halved, c >> 1) takes the mean feature of its occupied children only;
* ``up_conv``: the decoder's transposed 2x2x2 convolution with stride 2, whose output is pruned
  to the occupancy of the encoder at that level: each occupied child voxel receives
  W[k] x[parent] + b, k its position inside the parent's 2x2x2 block;
* skip connections (the encoder's features at a level joined with the decoder's there);
* ``head``: a shared MLP on the last decoder features predicting, for every point, the offset
  delta, the scale, the rotation, the opacity and the surface normal.

Readings where the paper is silent (its figure's channel widths are not in the text): the
channel plan and activations of ``LAYOUT`` and ``head``; the head's input per point is its
voxel's decoder features and its own coordinate residual (several points can share a voxel, and
the head is to give each its own parameters); skip connections concatenate channels
(as the sparse-convolution UNets the paper builds on do). Everything is FP64 numpy; submanifold
convolutions come from ``oracle.estimator.subm_conv``.
"""
from __future__ import annotations

import numpy as np

from .estimator import kernel_map, subm_conv, voxel_key

# (name, kind, cin, cout): the encoder at levels 0-3 and the decoder back to level 0
LAYOUT = [
    ("e0a", "subm", 32, 32), ("e0b", "subm", 32, 32),
    ("e1", "subm", 32, 64), ("e2", "subm", 64, 64), ("e3", "subm", 64, 64),
    ("u3", "up", 64, 64), ("d2", "subm", 128, 64),
    ("u2", "up", 64, 64), ("d1", "subm", 128, 64),
    ("u1", "up", 64, 32), ("d0", "subm", 64, 32),
]
HEAD_HIDDEN, HEAD_OUT = 32, 14


def _decode(keys: np.ndarray) -> np.ndarray:
    return np.stack([(keys >> 20) & 1023, (keys >> 10) & 1023, keys & 1023], axis=1).astype(np.int64)


def pool(coords: np.ndarray, feat: np.ndarray | None = None) -> dict:
    """Parent voxels of integer coordinates (V, 3) on the grid of half the resolution, in ascending
    linear key; child -> parent index, child counts and, if given, the mean features of the
    occupied children (V, C)."""
    pk = voxel_key(np.asarray(coords, np.int64) >> 1)
    ukeys, inv = np.unique(pk, return_inverse=True)
    cnt = np.bincount(inv, minlength=ukeys.size)
    out = dict(coords=_decode(ukeys), parent_of=inv.astype(np.int64), count=cnt)
    if feat is not None:
        f = np.asarray(feat, np.float64)
        sums = np.zeros((ukeys.size, f.shape[1]))
        np.add.at(sums, inv, f)
        out["feat"] = sums / cnt[:, None]
    return out


def child_offset(coords: np.ndarray) -> np.ndarray:
    """Position of each child inside its parent's 2x2x2 block: 4 (x & 1) + 2 (y & 1) + (z & 1)."""
    c = np.asarray(coords, np.int64)
    return 4 * (c[:, 0] & 1) + 2 * (c[:, 1] & 1) + (c[:, 2] & 1)


def up_conv(x_parent: np.ndarray, W: np.ndarray, b, child_coords: np.ndarray, parent_of: np.ndarray,
            relu: bool) -> np.ndarray:
    """Transposed 2x2x2 stride-2 convolution pruned to the children: W (8, Cin, Cout)."""
    k = child_offset(child_coords)
    x = np.asarray(x_parent, np.float64)[parent_of]
    y = np.einsum("vc,vco->vo", x, np.asarray(W, np.float64)[k])
    if b is not None:
        y = y + np.asarray(b, np.float64)
    return np.maximum(y, 0.0) if relu else y


def head(f: np.ndarray, W1: np.ndarray, b1, W2: np.ndarray, b2, points: np.ndarray, rgb: np.ndarray,
         point_voxel: np.ndarray, grid: int, coords: np.ndarray) -> dict:
    """Per-point Gaussians from the level-0 decoder features f (V, 32) by a shared MLP (Section 3.2:
    the last decoder layer holds the cloud's points and each one's parameters come from its own
    features). Point i of voxel v = point_voxel[i] (integer coordinates coords[v], (V, 3)) has the
    input x_i = [f[v], r_i] with r_i = (p_i + 1) grid / 2 - (coords[v] + 0.5), its residual inside
    the voxel in edges (the per-point attribute that merging points into one voxel averages away).
    raw_i = relu(x_i W1 + b1) W2 + b2 with W1 (35, 32), W2 (32, 14). Edge e = 2 / grid:
    mean = p + e tanh(raw[0:3]), scale = e exp(raw[3:6]), q = normalise(raw[6:10] + (1,0,0,0)),
    opacity = sigmoid(raw[10]), normal = normalise(raw[11:14]), colour = the point's own."""
    P = np.asarray(points, np.float64)
    pv = np.asarray(point_voxel)
    r = (P.T + 1.0) * (grid / 2.0) - (np.asarray(coords, np.float64)[pv] + 0.5)
    x = np.concatenate([np.asarray(f, np.float64)[pv], r], axis=1)
    h = np.maximum(x @ W1 + b1, 0.0)
    raw = h @ W2 + b2
    e = 2.0 / grid
    q = raw[:, 6:10] + np.array([1.0, 0.0, 0.0, 0.0])
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    nrm = raw[:, 11:14] / np.linalg.norm(raw[:, 11:14], axis=1, keepdims=True)
    return dict(input=x, raw=raw, mean=P + e * np.tanh(raw[:, 0:3]).T, scale=(e * np.exp(raw[:, 3:6])).T,
                quat=q.T, opacity=1.0 / (1.0 + np.exp(-raw[:, 10])), rgb=np.asarray(rgb, np.float64),
                normal=nrm.T)


def levels(coords0: np.ndarray, grid: int, depth: int = 3) -> list:
    """The voxel sets of levels 0..depth: coordinates, kernel maps, and for l >= 1 the pooling of
    level l - 1 (parent_of, count)."""
    out = [dict(coords=np.asarray(coords0, np.int64), grid=grid, nbr=kernel_map(coords0, grid))]
    for _ in range(depth):
        prev = out[-1]
        p = pool(prev["coords"])
        g = prev["grid"] // 2
        out.append(dict(coords=p["coords"], grid=g, nbr=kernel_map(p["coords"], g), parent_of=p["parent_of"],
                        count=p["count"]))
    return out


def forward(x0: np.ndarray, lv: list, weights: dict) -> np.ndarray:
    """Level-0 decoder features (V0, 32) of the network: weights[name] = (W, b) with W (27, Cin,
    Cout) for "subm" and (8, Cin, Cout) for "up" layers; every convolution is followed by ReLU."""
    def conv(name, x, level):
        W, b = weights[name]
        return subm_conv(x, W, b, lv[level]["nbr"], relu=True)

    def up(name, x, level):       # from level + 1 to level
        W, b = weights[name]
        return up_conv(x, W, b, lv[level]["coords"], lv[level + 1]["parent_of"], relu=True)

    def down(x, level):           # from level to level + 1
        nxt = lv[level + 1]
        sums = np.zeros((nxt["coords"].shape[0], x.shape[1]))
        np.add.at(sums, nxt["parent_of"], x)
        return sums / nxt["count"][:, None]

    s0 = conv("e0b", conv("e0a", x0, 0), 0)
    s1 = conv("e1", down(s0, 0), 1)
    s2 = conv("e2", down(s1, 1), 2)
    b3 = conv("e3", down(s2, 2), 3)
    d2 = conv("d2", np.concatenate([up("u3", b3, 2), s2], axis=1), 2)
    d1 = conv("d1", np.concatenate([up("u2", d2, 1), s1], axis=1), 1)
    return conv("d0", np.concatenate([up("u1", d1, 0), s0], axis=1), 0)
