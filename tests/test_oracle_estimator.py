"""Pins of the oracle's estimator steps: voxelisation, kernel map, submanifold convolution (equal to
a dense masked conv3d, a library routine) and the head's activations."""
import numpy as np
import pytest
import torch

from oracle import estimator as E
from synthetic import make_surface


def test_voxelize_lattice_points():
    _, p, rgb = make_surface(20000, 3, quantize=True)
    v = E.voxelize(p, rgb)
    assert v["count"].sum() == 20000
    assert np.all(np.abs(v["residual"]) < 1e-9)                 # lattice points sit at centres
    c = v["coords"][v["point_voxel"]]
    assert np.allclose((c + 0.5) / 512.0 - 1.0, p.T, atol=1e-7)
    assert np.all(np.diff(v["keys"]) > 0)
    # mean colour of the voxel's points
    i = np.argmax(v["count"])
    pts = np.flatnonzero(v["point_voxel"] == i)
    assert np.allclose(v["color"][i], rgb[:, pts].mean(axis=1))


def test_voxelize_residuals_unquantized():
    rng = np.random.default_rng(0)
    p = rng.uniform(-0.99, 0.99, (3, 500)).astype(np.float32).astype(np.float64)
    v = E.voxelize(p, rng.uniform(0, 1, (3, 500)))
    c = v["coords"][v["point_voxel"]]
    r = (p.T + 1) * 512 - (c + 0.5)
    assert np.all(np.abs(r) <= 0.5)
    assert np.allclose(v["residual"][v["point_voxel"]][v["count"][v["point_voxel"]] == 1],
                       r[v["count"][v["point_voxel"]] == 1])


def test_kernel_map_bruteforce():
    rng = np.random.default_rng(1)
    coords = np.unique(rng.integers(0, 12, (600, 3)), axis=0)
    coords[0] = [0, 0, 0]
    coords[-1] = [1023, 1023, 1023]
    nbr = E.kernel_map(coords)
    lookup = {tuple(c): i for i, c in enumerate(coords)}
    for i, c in enumerate(coords):
        for k, off in enumerate(E.OFFSETS):
            want = lookup.get(tuple(c + off), -1)
            assert nbr[k, i] == want
    assert np.all(nbr[13] == np.arange(coords.shape[0]))          # centre offset is the voxel itself


def test_subm_conv_equals_masked_dense_conv3d():
    rng = np.random.default_rng(2)
    D, Cin, Cout = 14, 5, 7
    coords = np.unique(rng.integers(0, D, (700, 3)), axis=0)
    V = coords.shape[0]
    x = rng.normal(size=(V, Cin))
    W = rng.normal(size=(27, Cin, Cout))
    b = rng.normal(size=Cout)
    y = E.subm_conv(x, W, b, E.kernel_map(coords), relu=False)
    X = torch.zeros((1, Cin, D, D, D), dtype=torch.float64)
    X[0, :, coords[:, 0], coords[:, 1], coords[:, 2]] = torch.from_numpy(x.T)
    Wt = torch.zeros((Cout, Cin, 3, 3, 3), dtype=torch.float64)
    for k, (dx, dy, dz) in enumerate(E.OFFSETS):
        Wt[:, :, dx + 1, dy + 1, dz + 1] = torch.from_numpy(W[k].T)
    out = torch.nn.functional.conv3d(X, Wt, torch.from_numpy(b), padding=1)
    ref = out[0, :, coords[:, 0], coords[:, 1], coords[:, 2]].numpy().T
    assert np.allclose(y, ref, atol=1e-12)
    yr = E.subm_conv(x, W, b, E.kernel_map(coords), relu=True)
    assert np.allclose(yr, np.maximum(ref, 0), atol=1e-12)


def test_head_activations():
    rng = np.random.default_rng(3)
    V, C, n = 40, 32, 100
    f = rng.normal(size=(V, C))
    Wh = rng.normal(size=(C, 11)) * 0.1
    bh = rng.normal(size=11) * 0.1
    pv = rng.integers(0, V, n)
    pts = rng.uniform(-1, 1, (3, n))
    col = rng.uniform(0, 1, (3, n))
    out = E.head(f, Wh, bh, col, pts, pv)
    raw = f @ Wh + bh
    assert np.allclose(out["scale"], (np.exp(raw[pv, 0:3]) / 512.0).T)
    q = raw[pv, 3:7] + [1, 0, 0, 0]
    assert np.allclose(out["quat"], (q / np.linalg.norm(q, axis=1, keepdims=True)).T)
    assert np.allclose(out["opacity"], 1 / (1 + np.exp(-raw[pv, 7])))
    assert np.allclose(out["rgb"], col + raw[pv, 8:11].T)
    # the normal is an eigenvector of the ellipsoid covariance with the smallest eigenvalue
    from scipy.spatial.transform import Rotation
    for i in range(n):
        qq = out["quat"][:, i]
        R = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
        S = R @ np.diag(out["scale"][:, i] ** 2) @ R.T
        nn = out["normal"][:, i]
        assert np.allclose(S @ nn, out["scale"][:, i].min() ** 2 * nn, atol=1e-12)
        assert nn @ (pts[:, i] - pts.mean(axis=1)) >= 0


def test_subm_conv_backward_finite_differences():
    rng = np.random.default_rng(4)
    coords = np.unique(rng.integers(0, 6, (80, 3)), axis=0)
    V, Cin, Cout = coords.shape[0], 3, 4
    nbr = E.kernel_map(coords)
    x = rng.normal(size=(V, Cin))
    W = rng.normal(size=(27, Cin, Cout))
    b = rng.normal(size=Cout)
    dy = rng.normal(size=(V, Cout))
    dx, dW, db = E.subm_conv_backward(x, W, nbr, dy)
    L = lambda xx, WW, bb: float((E.subm_conv(xx, WW, bb, nbr, relu=False) * dy).sum())  # noqa: E731
    h = 1e-6
    for (i, c) in [(0, 0), (V // 2, 1), (V - 1, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[i, c] += h
        xm[i, c] -= h
        assert abs((L(xp, W, b) - L(xm, W, b)) / (2 * h) - dx[i, c]) < 1e-6
    for (k, c, o) in [(0, 0, 0), (13, 1, 2), (26, 2, 3), (5, 0, 1)]:
        Wp, Wm = W.copy(), W.copy()
        Wp[k, c, o] += h
        Wm[k, c, o] -= h
        assert abs((L(x, Wp, b) - L(x, Wm, b)) / (2 * h) - dW[k, c, o]) < 1e-6
    bp = b.copy()
    bp[1] += h
    bm = b.copy()
    bm[1] -= h
    assert abs((L(x, W, bp) - L(x, W, bm)) / (2 * h) - db[1]) < 1e-6


def test_head_torch_matches_head():
    rng = np.random.default_rng(5)
    V, n = 30, 70
    f = rng.normal(size=(V, 32))
    Wh = rng.normal(size=(32, 11)) * 0.2
    bh = rng.normal(size=11) * 0.2
    pv = rng.integers(0, V, n)
    col = rng.uniform(0, 1, (3, n))
    ref = E.head(f, Wh, bh, col, rng.uniform(-1, 1, (3, n)), pv)
    q, s, o, c = E.head_torch(torch.from_numpy(f), torch.from_numpy(Wh), torch.from_numpy(bh),
                              torch.from_numpy(col), pv)
    assert np.allclose(q.numpy(), ref["quat"]) and np.allclose(s.numpy(), ref["scale"])
    assert np.allclose(o.numpy(), ref["opacity"]) and np.allclose(c.numpy(), ref["rgb"])


def test_voxelize_coarse_grid_lattice():
    """On a G^3 grid the centres (c + 0.5) * 2/G - 1 voxelise to c with zero residual; every
    power of two G works and other sizes are refused."""
    rng = np.random.default_rng(5)
    for g in (2, 64, 256):
        c = np.unique(rng.integers(0, g, (400, 3)), axis=0)
        p = ((c + 0.5) * (2.0 / g) - 1.0).T.astype(np.float32)
        v = E.voxelize(p, rng.uniform(0, 1, p.shape), g)
        assert np.array_equal(v["coords"], c)                  # unique keys ascend like np.unique rows
        assert np.all(np.abs(v["residual"]) < 1e-6)
        nb = E.kernel_map(v["coords"], g)
        lo = np.all(c == 0, axis=1)
        assert np.all(nb[0, lo] == -1)                          # offset (-1,-1,-1) leaves the grid
    for bad in (0, 100, 2048):
        with pytest.raises(ValueError):
            E.voxelize(np.zeros((3, 1), np.float32), np.zeros((3, 1)), bad)


def test_voxel_decision_on_fp32_sum():
    """The floor is taken on the FP32 value of p + 1: a coordinate whose FP64 sum lies just below a
    voxel boundary but rounds onto it in FP32 belongs to the upper voxel."""
    b = np.float32(0.25)                                        # boundary k/512 - 1 for k = 640
    below = np.nextafter(b, np.float32(-1))                     # FP32 just below the boundary
    # below + 1 in FP64 is 1.25 - 2^-26, which rounds to 1.25 in FP32 (ulp 2^-23 at 1.25)
    assert np.float64(below) + 1.0 < 1.25 and np.float32(below) + np.float32(1) == np.float32(1.25)
    v = E.voxelize(np.array([[below], [0.0], [0.0]], np.float32), np.zeros((3, 1)), 1024)
    assert v["coords"][0, 0] == 640
