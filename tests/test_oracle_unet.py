"""Pins of the UNet oracle (oracle/unet.py) against brute force, closed forms and library routines
(torch's avg_pool3d, conv3d and conv_transpose3d on dense grids)."""
import numpy as np
import pytest
import torch

from oracle import estimator as E
from oracle import unet as U


def _rand_coords(rng, n, grid):
    c = rng.integers(0, grid, size=(n, 3))
    keys = np.unique(E.voxel_key(c))
    return np.stack([(keys >> 20) & 1023, (keys >> 10) & 1023, keys & 1023], axis=1)


def test_pool_equals_bruteforce_grouping():
    rng = np.random.default_rng(1)
    coords = _rand_coords(rng, 3000, 32)
    feat = rng.normal(size=(coords.shape[0], 5))
    p = U.pool(coords, feat)
    groups = {}
    for i, c in enumerate(coords):
        groups.setdefault(tuple(int(v) >> 1 for v in c), []).append(i)
    keys = sorted(groups, key=lambda t: (t[0] << 20) | (t[1] << 10) | t[2])
    assert np.array_equal(p["coords"], np.array(keys))
    for pi, k in enumerate(keys):
        idx = groups[k]
        assert p["count"][pi] == len(idx)
        assert np.allclose(p["feat"][pi], feat[idx].mean(axis=0), rtol=0, atol=1e-14)
        assert np.all(p["parent_of"][idx] == pi)


def test_pool_closed_forms():
    # a full 2x2x2 block averages all eight children; a lone child passes its feature through
    block = np.array([(x, y, z) for x in (4, 5) for y in (6, 7) for z in (0, 1)] + [(9, 9, 9)])
    feat = np.arange(block.shape[0] * 2, dtype=np.float64).reshape(-1, 2)
    p = U.pool(block, feat)
    assert p["coords"].tolist() == [[2, 3, 0], [4, 4, 4]]
    assert p["count"].tolist() == [8, 1]
    assert np.array_equal(p["feat"][0], feat[:8].mean(axis=0)) and np.array_equal(p["feat"][1], feat[8])


def _dense(coords, feat, grid):
    t = torch.zeros((1, feat.shape[1], grid, grid, grid), dtype=torch.float64)
    t[0, :, coords[:, 0], coords[:, 1], coords[:, 2]] = torch.from_numpy(feat).T
    return t


def test_up_conv_equals_transposed_convolution_at_the_children():
    rng = np.random.default_rng(2)
    child = _rand_coords(rng, 1500, 16)
    p = U.pool(child)
    xp = rng.normal(size=(p["coords"].shape[0], 4))
    W = rng.normal(size=(8, 4, 3))
    b = rng.normal(size=3)
    got = U.up_conv(xp, W, b, child, p["parent_of"], relu=False)
    # torch weight (Cin, Cout, 2, 2, 2): the child at offset (a, b, c) of its parent uses W[4a+2b+c]
    wt = torch.from_numpy(W.reshape(2, 2, 2, 4, 3).transpose(3, 4, 0, 1, 2).copy())
    dense = torch.nn.functional.conv_transpose3d(_dense(p["coords"], xp, 8), wt, torch.from_numpy(b), stride=2)
    ref = dense[0, :, child[:, 0], child[:, 1], child[:, 2]].T.numpy()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    assert np.array_equal(U.up_conv(xp, W, b, child, p["parent_of"], relu=True), np.maximum(got, 0.0))


def test_head_closed_forms():
    rng = np.random.default_rng(3)
    V, n, grid = 50, 80, 64
    coords = rng.integers(0, grid, size=(V, 3))
    f = rng.normal(size=(V, 32))
    W1, b1 = rng.normal(size=(35, 32)) * 0.3, rng.normal(size=32) * 0.1
    W2, b2 = rng.normal(size=(32, 14)) * 0.3, rng.normal(size=14) * 0.1
    pv = rng.integers(0, V, size=n)
    # each point inside its voxel: p = (c + u) 2 / grid - 1 with u in [0, 1)^3
    u = rng.uniform(0, 1, size=(n, 3))
    pts = ((coords[pv] + u) * (2.0 / grid) - 1.0).T
    rgb = rng.uniform(0, 1, size=(3, n))
    h = U.head(f, W1, b1, W2, b2, pts, rgb, pv, grid, coords)
    # the input is the voxel's features and the point's residual, which lies in [-1/2, 1/2)^3
    assert np.array_equal(h["input"][:, :32], f[pv])
    assert np.allclose(h["input"][:, 32:], u - 0.5, atol=1e-12)
    raw = np.array([np.maximum(np.r_[f[pv[i]], u[i] - 0.5] @ W1 + b1, 0.0) @ W2 + b2 for i in range(n)])
    e = 2.0 / grid
    assert np.allclose(h["raw"], raw)
    assert np.all(np.abs(h["mean"] - pts) < e)                       # the offset stays within a voxel edge
    assert np.allclose(h["mean"] - pts, e * np.tanh(raw[:, 0:3]).T)
    assert np.allclose(np.log(h["scale"] / e), raw[:, 3:6].T)
    assert np.allclose(np.linalg.norm(h["quat"], axis=0), 1.0) and np.allclose(np.linalg.norm(h["normal"], axis=0), 1.0)
    assert np.allclose(h["opacity"], 1 / (1 + np.exp(-raw[:, 10])))
    assert np.array_equal(h["rgb"], rgb)
    # two points of one voxel get different outputs through their residuals only; with zero
    # residual weights they get the same (the head is then one per voxel)
    same = np.flatnonzero(pv == pv[0])
    if same.size < 2:
        pv[1] = pv[0]
        pts[:, 1] = ((coords[pv[0]] + u[1]) * (2.0 / grid) - 1.0)
        same = np.array([0, 1])
    W1z = W1.copy()
    W1z[32:] = 0.0
    hz = U.head(f, W1z, b1, W2, b2, pts, rgb, pv, grid, coords)
    assert np.allclose(hz["raw"][same[0]], hz["raw"][same[1]])
    h2 = U.head(f, W1, b1, W2, b2, pts, rgb, pv, grid, coords)
    assert not np.allclose(h2["raw"][same[0]], h2["raw"][same[1]])
    # zero rotation outputs give the identity quaternion; a normal output is its own direction
    q = U.head(np.zeros((1, 32)), W1 * 0, np.zeros(32), W2 * 0, np.r_[np.zeros(11), 0, 0, 2.0], pts[:, :1],
               rgb[:, :1], np.zeros(1, int), grid, coords[pv[:1]])
    assert np.allclose(q["quat"][:, 0], [1, 0, 0, 0]) and np.allclose(q["normal"][:, 0], [0, 0, 1])


def test_forward_on_a_full_cube_equals_a_dense_unet():
    """On a fully occupied 8^3 cube pooling is avg_pool3d, the submanifold convolution is conv3d
    with zero padding and the pruned transposed convolution is conv_transpose3d, so the sparse
    network must equal the dense one built from those library routines."""
    rng = np.random.default_rng(4)
    g = 8
    coords = np.array([(x, y, z) for x in range(g) for y in range(g) for z in range(g)])
    keys = E.voxel_key(coords)
    coords = coords[np.argsort(keys)]
    x0 = np.zeros((coords.shape[0], 32))
    x0[:, :6] = rng.normal(size=(coords.shape[0], 6))
    weights = {}
    for name, kind, ci, co in U.LAYOUT:
        k = 27 if kind == "subm" else 8
        weights[name] = (rng.normal(size=(k, ci, co)) * np.sqrt(2.0 / (k * ci)), rng.normal(size=co) * 0.05)
    lv = U.levels(coords, g)
    got = U.forward(x0, lv, weights)

    def conv(name, t):
        W, b = weights[name]     # (27, Cin, Cout), offset k = 9 (dx+1) + 3 (dy+1) + (dz+1)
        w = torch.from_numpy(W.reshape(3, 3, 3, W.shape[1], W.shape[2]).transpose(4, 3, 0, 1, 2).copy())
        return torch.relu(torch.nn.functional.conv3d(t, w, torch.from_numpy(b), padding=1))

    def up(name, t):
        W, b = weights[name]
        w = torch.from_numpy(W.reshape(2, 2, 2, W.shape[1], W.shape[2]).transpose(3, 4, 0, 1, 2).copy())
        return torch.relu(torch.nn.functional.conv_transpose3d(t, w, torch.from_numpy(b), stride=2))

    pool = lambda t: torch.nn.functional.avg_pool3d(t, 2)  # noqa: E731
    t0 = _dense(coords, x0, g)
    s0 = conv("e0b", conv("e0a", t0))
    s1 = conv("e1", pool(s0))
    s2 = conv("e2", pool(s1))
    b3 = conv("e3", pool(s2))
    d2 = conv("d2", torch.cat([up("u3", b3), s2], 1))
    d1 = conv("d1", torch.cat([up("u2", d2), s1], 1))
    d0 = conv("d0", torch.cat([up("u1", d1), s0], 1))
    ref = d0[0, :, coords[:, 0], coords[:, 1], coords[:, 2]].T.numpy()
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)
    assert np.abs(ref).max() > 0.1


def test_synthetic_normals_are_the_surfaces_normals():
    from synthetic.scenes import ProceduralSurface
    s = ProceduralSurface(np.random.default_rng(6))
    p, n = s.sample(4000, np.random.default_rng(7), with_normals=True)
    world = p / s.norm_scale + s.norm_center[:, None]
    # each point lies on one primitive; for spheres the normal is (p - c) / r, for tori it is
    # orthogonal to both surface tangents: check the sphere points and the unit length of all
    assert np.allclose(np.linalg.norm(n, axis=0), 1.0)
    hits = 0
    for i, kind in enumerate(s.kinds):
        if kind != "sphere":
            continue
        d = world - s.center[i][:, None]
        on = np.abs(np.linalg.norm(d, axis=0) - s.radius[i]) < 1e-9
        hits += int(on.sum())
        assert np.allclose(n[:, on], d[:, on] / s.radius[i], atol=1e-9)
    assert hits > 500
