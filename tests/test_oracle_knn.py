"""Pins of the oracle's kNN-PCA surfel estimate (closed forms, brute force)."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import knn_pca as kp
from synthetic import make_surface


def test_tree_knn_equals_bruteforce_with_lattice_ties():
    _, p, _ = make_surface(3000, 7, quantize=True)
    nb_b = kp.knn_bruteforce(p, 16)
    nb_t, _ = kp.knn(p, 16, brute_max=0)
    assert np.array_equal(nb_b, nb_t)
    # lattice points produce exact distance ties; every row starts with the point itself or a duplicate
    d2 = ((p.T[nb_b] - p.T[:, None, :]).astype(np.float64) ** 2).sum(-1)
    assert np.all(d2[:, 0] == 0)
    assert np.all(np.diff(d2, axis=1) >= 0)


def _place(local, R, c):
    return (R @ local.T).T + c


def test_ring_closed_form():
    """Centre point plus 15 points on a ring of radius rho, tilted, isolated: the neighbourhood is
    exactly these 16 points, mu = centre, C has eigenvalues (15/32 rho^2, 15/32 rho^2, 0)."""
    rho = 0.05
    t = 2 * math.pi * np.arange(15) / 15
    local = np.concatenate([[[0, 0, 0]], np.stack([rho * np.cos(t), rho * np.sin(t), 0 * t], 1)])
    R = Rotation.from_euler("xyz", [0.4, -0.3, 1.2]).as_matrix()
    c = np.array([0.3, -0.2, 0.5])
    pts = _place(local, R, c)
    far = np.random.default_rng(0).uniform(-1, 1, (40, 3)) * 0.2 + np.array([-0.6, 0.6, -0.6])
    allp = np.concatenate([pts, far]).T
    out = kp.knn_pca(allp, k=16, kappa=1.0)
    i = 0
    lam = out["eig"][i]
    assert np.allclose(lam, [15 / 32 * rho ** 2, 15 / 32 * rho ** 2, 0.0], atol=1e-15)
    n = out["normal"][:, i]
    assert abs(abs(n @ R[:, 2]) - 1) < 1e-9
    s = out["scale"][:, i]
    assert np.allclose(s[:2], rho * math.sqrt(15 / 32), rtol=1e-9)
    assert math.isclose(s[2], 0.1 * s[1], rel_tol=1e-9)
    # orientation: away from the cloud centroid
    assert n @ (allp[:, i] - allp.mean(axis=1)) >= 0


def test_ellipse_axes_closed_form():
    """16 points on an ellipse (a, b) in a tilted plane: mu = centre, C = diag(a^2/2, b^2/2, 0) in
    the ellipse frame, so the major axis is e1 and s = kappa (a, b)/sqrt(2)."""
    a, b, kappa = 0.08, 0.03, 1.2
    t = 2 * math.pi * np.arange(16) / 16
    local = np.stack([a * np.cos(t), b * np.sin(t), 0 * t], 1)
    R = Rotation.from_euler("zyx", [0.7, 0.2, -0.5]).as_matrix()
    pts = _place(local, R, np.array([0.1, 0.1, 0.1]))
    out = kp.knn_pca(pts.T, k=16, kappa=kappa)
    for i in range(16):
        s = out["scale"][:, i]
        assert np.allclose(s[:2], [kappa * a / math.sqrt(2), kappa * b / math.sqrt(2)], rtol=1e-9)
        q = out["quat"][:, i]
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert abs(abs(Rq[:, 0] @ R[:, 0]) - 1) < 1e-9       # major axis
        assert abs(abs(Rq[:, 2] @ R[:, 2]) - 1) < 1e-9       # normal
        assert np.allclose(Rq[:, 2], out["normal"][:, i], atol=1e-12)
        want = R @ np.diag([s[0] ** 2, s[1] ** 2, s[2] ** 2]) @ R.T
        assert np.allclose(out["cov"][i], want, atol=1e-15)


def test_plane_normals():
    rng = np.random.default_rng(3)
    nrm = np.array([0.3, -0.5, 0.8]); nrm /= np.linalg.norm(nrm)
    u = np.cross(nrm, [1, 0, 0]); u /= np.linalg.norm(u)
    v = np.cross(nrm, u)
    ab = rng.uniform(-0.5, 0.5, (2, 1500))
    p = (u[:, None] * ab[0] + v[:, None] * ab[1]) + 0.2 * nrm[:, None]
    out = kp.knn_pca(p, k=16)
    assert np.all(np.abs(out["eig"][:, 2]) < 1e-15)
    assert np.allclose(np.abs(out["normal"].T @ nrm), 1.0, atol=1e-9)
    # centroid lies in the plane, so the orientation rule leaves n . (p - centroid) = 0 for all
    assert np.all(out["scale"][2] <= 0.1 * out["scale"][1] + 1e-15)


def test_duplicate_points_degenerate():
    p = np.zeros((3, 20))
    p[:, 16:] = np.random.default_rng(0).uniform(-1, 1, (3, 4))
    out = kp.knn_pca(p, k=16)
    assert np.all(out["scale"][:, 0] == 0.0)
    assert np.all(np.isfinite(out["quat"]))
