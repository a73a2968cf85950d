"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU involved).

Each test ties one part of the oracle to something other than itself: a closed form that follows
from Eq. 1-4 of Section 3.1, a library routine a special case reduces to, a brute-force
evaluation of the definition, an invariant, or central finite differences.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from oracle import brute
from synthetic import look_at_camera, random_gaussians, focal_for_vfov

LP = float(np.float32(0.3))      # the low-pass option travels as FP32


def gauss(means, quats=None, scales=None, opac=None, rgb=None, nrm=None, dtype=np.float32):
    means = np.asarray(means, np.float64).reshape(-1, 3).T
    n = means.shape[1]
    quats = np.tile([[1.0], [0], [0], [0]], (1, n)) if quats is None else np.asarray(quats, np.float64).reshape(-1, 4).T
    scales = np.full((3, n), 0.05) if scales is None else np.asarray(scales, np.float64).reshape(-1, 3).T
    opac = np.full(n, 0.8) if opac is None else np.asarray(opac, np.float64).reshape(n)
    rgb = np.tile([[0.2], [0.5], [0.9]], (1, n)) if rgb is None else np.asarray(rgb, np.float64).reshape(-1, 3).T
    nrm = np.tile([[0.0], [0], [1]], (1, n)) if nrm is None else np.asarray(nrm, np.float64).reshape(-1, 3).T
    return {k: np.ascontiguousarray(v, dtype=dtype) for k, v in
            dict(mean=means, quat=quats, scale=scales, opacity=opac, rgb=rgb, normal=nrm).items()}


def identity_camera(W, H, f=None):
    """Camera at the origin looking down +z (x right, y down): T = I, t = 0."""
    f = float(np.float32(focal_for_vfov(H) if f is None else f))
    return dict(T=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), fx=f, fy=f,
                cx=W / 2.0, cy=H / 2.0, width=W, height=H)


# --------------------------------------------------------------------------------------------
# Covariance Sigma = R diag(s^2) R^T (Section 3.1)
# --------------------------------------------------------------------------------------------
def test_covariance_matches_library_rotation():
    rng = np.random.default_rng(0)
    g = random_gaussians(64, rng)
    S = oracle.covariance_f64(g["quat"], g["scale"])
    q = g["quat"].astype(np.float64)
    R = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], axis=1)).as_matrix()   # scipy: x,y,z,w
    s2 = g["scale"].astype(np.float64).T ** 2
    ref = np.einsum("nij,nj,nkj->nik", R, s2, R)
    assert np.allclose(S, ref, rtol=0, atol=1e-15)
    # eigen-decomposition returns the squared scales and the rotation's columns (up to sign)
    for i in range(8):
        w, V = np.linalg.eigh(S[i])
        order = np.argsort(s2[i])
        assert np.allclose(w, s2[i][order], rtol=1e-9, atol=1e-18)
        for j, col in enumerate(order):
            assert abs(abs(V[:, j] @ R[i][:, col]) - 1.0) < 1e-6
    assert np.all(np.linalg.eigvalsh(S) >= -1e-18)     # positive semi-definite


def test_unnormalised_and_zero_quaternions():
    g1 = gauss([[0, 0, 0]], quats=[[0.5, 0.1, -0.2, 0.3]], scales=[[0.1, 0.2, 0.3]], dtype=np.float64)
    g2 = gauss([[0, 0, 0]], quats=[[5.0, 1.0, -2.0, 3.0]], scales=[[0.1, 0.2, 0.3]], dtype=np.float64)
    S1 = oracle.covariance_f64(g1["quat"], g1["scale"])
    S2 = oracle.covariance_f64(g2["quat"], g2["scale"])
    assert np.allclose(S1, S2, atol=1e-16)
    g0 = gauss([[0, 0, 0]], quats=[[0.0, 0, 0, 0]], scales=[[0.1, 0.2, 0.3]], dtype=np.float64)
    assert np.allclose(oracle.covariance_f64(g0["quat"], g0["scale"])[0], np.diag([0.01, 0.04, 0.09]))


# --------------------------------------------------------------------------------------------
# Projection (Eq. 3-4)
# --------------------------------------------------------------------------------------------
def test_pinhole_position_of_camera_relative_points():
    rng = np.random.default_rng(1)
    for _ in range(5):
        eye = rng.normal(size=3)
        eye *= 3.0 / np.linalg.norm(eye)
        cam = look_at_camera(eye, width=200, height=150)
        fwd = -eye / np.linalg.norm(eye)
        right = np.cross(fwd, [0, 1, 0]); right /= np.linalg.norm(right)
        down = np.cross(fwd, right)
        d, h, k = rng.uniform(1, 4), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)
        P = eye + d * fwd + h * right + k * down
        p = oracle.project_f64(gauss([P], dtype=np.float64), cam)
        assert p["valid"][0]
        assert abs(p["u"][0] - (cam.cx + cam.fx * h / d)) < 1e-5
        assert abs(p["v"][0] - (cam.cy + cam.fy * k / d)) < 1e-5
        assert abs(p["z"][0] - d) < 1e-6


def test_ewa_screen_covariance_equals_jacobian_sandwich():
    """Sigma_s - lowpass*I must equal Jp Sigma Jp^T with Jp the finite-difference Jacobian of the
    oracle's own projected pixel position with respect to the world-space mean (Eq. 4)."""
    rng = np.random.default_rng(2)
    g = random_gaussians(6, rng, mean_range=0.6)
    g = {k: v.astype(np.float64) for k, v in g.items()}
    cam = look_at_camera([1.1, 0.7, 2.6], width=320, height=240)
    lp = LP
    base = oracle.project_f64(g, cam)
    S = oracle.covariance_f64(g["quat"], g["scale"])
    for i in range(6):
        assert base["valid"][i]
        Jp = np.zeros((2, 3))
        for k in range(3):
            h = 1e-6
            gp = {kk: vv.copy() for kk, vv in g.items()}
            gm = {kk: vv.copy() for kk, vv in g.items()}
            gp["mean"][k, i] += h
            gm["mean"][k, i] -= h
            pp, pm = oracle.project_f64(gp, cam), oracle.project_f64(gm, cam)
            Jp[0, k] = (pp["u"][i] - pm["u"][i]) / (2 * h)
            Jp[1, k] = (pp["v"][i] - pm["v"][i]) / (2 * h)
        want = Jp @ S[i] @ Jp.T
        a, b, c = base["cov2d"][:, i]
        got = np.array([[a - lp, b], [b, c - lp]])
        assert np.allclose(got, want, rtol=1e-6, atol=1e-9 * np.abs(want).max())


def test_isotropic_closed_form_off_axis():
    """Isotropic sigma at (x, 0, z) seen by the identity camera:
    Sigma_s = (sigma f / z)^2 diag(1 + x^2/z^2, 1) + lowpass I."""
    W = H = 256
    cam = identity_camera(W, H)
    f = cam["fx"]
    for x, z, s in [(0.3, 2.0, 0.05), (-0.7, 3.0, 0.1), (0.0, 1.5, 0.02)]:
        g = gauss([[x, 0.0, z]], scales=[[s, s, s]], quats=[[0.3, 0.2, -0.7, 0.1]], dtype=np.float64)
        p = oracle.project_f64(g, cam)
        k = (s * f / z) ** 2
        a, b, c = p["cov2d"][:, 0]
        assert math.isclose(a, k * (1 + x * x / (z * z)) + LP, rel_tol=1e-12)
        assert abs(b) < 1e-12 * k
        assert math.isclose(c, k + LP, rel_tol=1e-12)


def test_rotated_anisotropic_on_axis():
    """A Gaussian rotated by theta about the viewing axis, on the axis of the camera at (0,0,3)
    (rows right=(1,0,0), down=(0,-1,0)): Sigma_s = (f/z)^2 [[Sxx, -Sxy], [-Sxy, Syy]] + lp I with
    Sxx = s1^2 cos^2 + s2^2 sin^2, Sxy = (s1^2 - s2^2) cos sin."""
    cam = look_at_camera([0, 0, 3], width=128, height=128)
    f, z = cam.fx, 3.0
    s1, s2, s3 = 0.2, 0.05, 0.1
    for th in (0.3, 1.1, -0.8):
        q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
        g = gauss([[0, 0, 0]], quats=[q], scales=[[s1, s2, s3]], dtype=np.float64)
        p = oracle.project_f64(g, cam)
        c, s = math.cos(th), math.sin(th)
        Sxx, Syy, Sxy = s1 ** 2 * c * c + s2 ** 2 * s * s, s1 ** 2 * s * s + s2 ** 2 * c * c, (s1 ** 2 - s2 ** 2) * c * s
        k = (f / z) ** 2
        a, b, cc = p["cov2d"][:, 0]
        assert math.isclose(a, k * Sxx + LP, rel_tol=1e-9)
        assert math.isclose(b, -k * Sxy, rel_tol=1e-9)
        assert math.isclose(cc, k * Syy + LP, rel_tol=1e-9)


def test_conic_is_inverse_and_extents_bound_the_three_sigma_ellipse():
    """The binning box is the axis-aligned box of the 3-sigma ellipse x^T Sigma_s^-1 x <= 9: points
    of the ellipse's boundary, built from the eigen-decomposition of Sigma_s (x = 3 V L^1/2
    (cos t, sin t)), reach 3 sqrt(a) in x and 3 sqrt(c) in y and never pass the padded extents."""
    rng = np.random.default_rng(3)
    g = random_gaussians(200, rng)
    cam = look_at_camera([0, 0, 3], width=128, height=128)
    p = oracle.project_f64(g, cam)
    idx = np.nonzero(p["valid"])[0]
    assert idx.size > 150
    t = np.linspace(0.0, 2.0 * np.pi, 4001)
    circle = np.stack([np.cos(t), np.sin(t)])
    for i in idx:
        a, b, c = p["cov2d"][:, i]
        Ss = np.array([[a, b], [b, c]])
        Cn = np.array([[p["A"][i], p["B"][i]], [p["B"][i], p["C"][i]]])
        assert np.allclose(Cn @ Ss, np.eye(2), atol=1e-12)
        lam, V = np.linalg.eigh(Ss)
        pts = 3.0 * (V * np.sqrt(lam)) @ circle                # the boundary q = 9
        reach = np.abs(pts).max(axis=1)
        assert np.all(reach <= np.array([p["ex"][i], p["ey"][i]]))
        assert np.allclose(reach, [3.0 * math.sqrt(a), 3.0 * math.sqrt(c)], rtol=1e-6)
        assert p["ex"][i] == 3.0 * math.sqrt(a) * 1.001 + 0.01 and p["ey"][i] == 3.0 * math.sqrt(c) * 1.001 + 0.01


def test_fp32_projection_tracks_fp64():
    rng = np.random.default_rng(4)
    g = random_gaussians(2000, rng)
    cam = look_at_camera([0, 0, 3], width=128, height=128)
    p32, p64 = oracle.project_f32(g, cam), oracle.project_f64(g, cam)
    both = (p32["valid"] == 1) & (p64["valid"] == 1)
    assert both.sum() > 1500
    assert np.max(np.abs(p32["u"][both] - p64["u"][both])) < 1e-4
    assert np.max(np.abs(p32["v"][both] - p64["v"][both])) < 1e-4
    for k in ("A", "B", "C"):
        scale = np.maximum(np.abs(p64["A"][both]), np.abs(p64["C"][both]))
        assert np.max(np.abs(p32[k][both] - p64[k][both]) / scale) < 1e-4
    # extents agree to FP32 rounding; rectangles differ only where a box edge sits on a tile edge
    for k in ("ex", "ey"):
        assert np.max(np.abs(p32[k][both] - p64[k][both]) / p64[k][both]) < 1e-5
    differ = both & np.any(p32["rect"] != p64["rect"], axis=0)
    assert differ.sum() <= 2


def test_fp64_projection_orders_by_the_exact_fp32_depth():
    """Reading C-8: the depth order is defined on the FP32 depth of the exact projection, in the
    FP64 render too (the FP64 depth rounded to FP32 can differ from it by an ulp and would swap
    splats of nearly equal depth)."""
    rng = np.random.default_rng(14)
    g = random_gaussians(2000, rng)
    cam = look_at_camera([0.3, -0.2, 3], width=128, height=128)
    p32, p64 = oracle.project_f32(g, cam), oracle.project_f64(g, cam)
    both = (p32["valid"] == 1) & (p64["valid"] == 1)
    assert both.sum() > 1500
    assert np.array_equal(p64["zf"][both].view(np.uint32), np.asarray(p32["z"], np.float32)[both].view(np.uint32))
    # and the rounded FP64 depth is not always that value (otherwise the pin would be empty)
    rounded = np.asarray(p64["z"], np.float32)
    assert (rounded[both] != p64["zf"][both]).any()


def test_margins_against_the_other_projection_only_add_flags():
    g, cam = _c1_scene()
    plain = oracle.render(g, [cam], mode="ref")
    wide = oracle.render(g, [cam], mode="ref", margin_vs="f64")
    for k in ("rgb", "normal", "depth", "alpha", "n_contrib"):
        assert np.array_equal(plain[k], wide[k]), k
    assert np.all(wide["flags"][plain["flags"] != 0] != 0)
    assert (wide["flags"] != 0).sum() >= (plain["flags"] != 0).sum()


def test_near_plane_and_nonfinite_culled():
    cam = look_at_camera([0, 0, 3], width=64, height=64)
    g = gauss([[0, 0, 2.9], [0, 0, 2.85], [0, 0, 0], [0, 0, 0], [0, 0, 0]], opac=[0.8, 0.8, 0.8, 0.8, 0.001])
    g["rgb"][1, 3] = np.nan
    p32, p64 = oracle.project_f32(g, cam), oracle.project_f64(g, cam)
    # z = 0.1 and 0.15 are inside the 0.2 near plane; NaN colour; opacity below the alpha cutoff
    assert list(p32["valid"]) == [0, 0, 1, 0, 0]
    assert list(p64["valid"][:3]) == [0, 0, 1]


# --------------------------------------------------------------------------------------------
# Compositing (Eq. 1-2)
# --------------------------------------------------------------------------------------------
def _centered_scene(W=65):
    cam = look_at_camera([0, 0, 3], width=W, height=W)
    assert cam.cx == (W // 2) + 0.5
    return cam


@pytest.mark.parametrize("mode", ["ref", "f64"])
def test_single_splat_head_on(mode):
    cam = _centered_scene(65)
    sigma, o = 0.1, 0.7
    g = gauss([[0, 0, 0]], scales=[[sigma] * 3], opac=[o], rgb=[[0.3, 0.6, 0.9]])
    img = oracle.render(g, [cam], mode=mode)
    s2 = (sigma * cam.fx / 3.0) ** 2 + LP
    c = 32
    assert math.isclose(img["rgb"][0, 1, c, c], o * 0.6, rel_tol=1e-6)
    assert math.isclose(img["alpha"][0, c, c], o, rel_tol=1e-6)
    p = oracle.project_f64(g, cam)
    assert math.isclose(p["ex"][0], 3 * math.sqrt(s2) * 1.001 + 0.01, rel_tol=1e-6)   # FP32 inputs
    assert math.isclose(p["ey"][0], 3 * math.sqrt(s2) * 1.001 + 0.01, rel_tol=1e-6)
    for d in range(0, 10):
        a = o * math.exp(-d * d / (2 * s2))
        if d * d > 9 * s2 or a < 1 / 255:
            a = 0.0
        assert abs(img["alpha"][0, c, c + d] - a) < 2e-6, d
        assert abs(img["rgb"][0, 2, c + d, c] - a * 0.9) < 2e-6, d
        assert abs(img["depth"][0, c, c + d] - a * 3.0) < 1e-5, d


@pytest.mark.parametrize("o", [0.5, 0.02])
def test_integrated_mass(o):
    """Sum over pixels of alpha = o * 2 pi sqrt(det Sigma_s) * (1 - exp(-q*/2)),
    q* = min(9, 2 ln(255 o)) for a single large anisotropic splat."""
    W = 257
    cam = _centered_scene(W)
    th = 0.6
    g = gauss([[0, 0, 0]], quats=[[math.cos(th / 2), 0.2, 0.1, math.sin(th / 2)]],
              scales=[[0.3, 0.15, 0.2]], opac=[o])
    img = oracle.render(g, [cam], mode="f64")
    p = oracle.project_f64(g, cam)
    a, b, c = p["cov2d"][:, 0]
    det = a * c - b * b
    assert min(a, c) > 100.0              # s >= 10 px
    qs = min(9.0, 2.0 * math.log(255.0 * o))
    want = o * 2 * math.pi * math.sqrt(det) * (1.0 - math.exp(-qs / 2))
    got = img["alpha"][0].sum()
    assert abs(got / want - 1.0) < 1e-3


def test_two_splats_blend_in_depth_order():
    cam = _centered_scene(65)
    # index 0 is the far one: order must come from depth, not index
    g = gauss([[0, 0, -0.5], [0, 0, 0.5]], scales=[[0.1] * 3, [0.1] * 3], opac=[0.6, 0.3],
              rgb=[[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    img = oracle.render(g, [cam], mode="ref")
    c = 32
    a_near, a_far = 0.3, 0.6
    want_r = (1 - a_near) * a_far * 1.0
    want_g = a_near * 1.0
    assert math.isclose(img["rgb"][0, 0, c, c], want_r, rel_tol=1e-6)
    assert math.isclose(img["rgb"][0, 1, c, c], want_g, rel_tol=1e-6)
    assert math.isclose(img["alpha"][0, c, c], 1 - (1 - a_near) * (1 - a_far), rel_tol=1e-6)
    assert img["n_contrib"][0, c, c] == 2


def test_truncation_bound_and_stop_position():
    cam = _centered_scene(65)
    n = 10
    rng = np.random.default_rng(5)
    g = gauss([[0, 0, -0.1 * k] for k in range(n)], scales=[[0.1] * 3] * n, opac=[0.85] * n,
              rgb=rng.uniform(0, 1, (n, 3)))
    img = oracle.render(g, [cam], mode="ref")
    full = oracle.render(g, [cam], mode="ref", opts=dict(t_eps=0.0))
    assert img["n_contrib"][0, 32, 32] == 5          # 0.15^4 > 1e-4 > 0.15^5
    assert full["n_contrib"][0, 32, 32] == n
    for k in ("rgb", "normal"):
        assert np.max(np.abs(img[k] - full[k])) < 1e-4 * 1.0


def test_alpha_cutoff_zeroes_faint_pixels():
    """With o = 0.02 only pixels where o exp(-q/2) >= 1/255 receive colour."""
    cam = _centered_scene(65)
    g = gauss([[0, 0, 0]], scales=[[0.15] * 3], opac=[0.02])
    img = oracle.render(g, [cam], mode="f64")
    s2 = (0.15 * cam.fx / 3.0) ** 2 + LP
    yy, xx = np.mgrid[0:65, 0:65]
    q = ((xx + 0.5 - 32.5) ** 2 + (yy + 0.5 - 32.5) ** 2) / s2
    a = 0.02 * np.exp(-q / 2)
    keep = (q <= 9) & (a >= np.float32(1 / 255))
    assert np.abs(img["alpha"][0] - np.where(keep, a, 0)).max() < 1e-9
    assert (~keep).sum() > 0 and keep.sum() > 0


# --------------------------------------------------------------------------------------------
# Binning and sort
# --------------------------------------------------------------------------------------------
def test_binning_matches_bruteforce_tile_test_and_python_sorted():
    rng = np.random.default_rng(1001)
    g = random_gaussians(2000, rng)
    W = H = 128
    cams = [look_at_camera([0, 0, 3], width=W, height=H), look_at_camera([0.5, 0.3, 2.9], width=W, height=H)]
    projs = [oracle.project_f32(g, c) for c in cams]
    keys, vals = oracle.bin_sorted(projs, 2000, W, H)
    TX = TY = 8
    pairs = []
    for ci, p in enumerate(projs):
        zb = p["z"].view(np.uint32)
        for i in np.nonzero(p["valid"])[0]:
            u, v = float(p["u"][i]), float(p["v"][i])
            ex, ey = float(p["ex"][i]), float(p["ey"][i])
            for ty in range(TY):
                for tx in range(TX):
                    if 16 * tx <= u + ex and 16 * (tx + 1) > u - ex and 16 * ty <= v + ey and 16 * (ty + 1) > v - ey:
                        pairs.append((((ci * TX * TY + ty * TX + tx) << 32) | int(zb[i]), int(i)))
    pairs = sorted(pairs)
    assert len(pairs) == keys.size
    assert [int(k) for k in keys] == [k for k, _ in pairs]
    assert [int(v) for v in vals] == [v for _, v in pairs]
    rng_t = oracle.tile_ranges(keys, 2 * TX * TY)
    for t in range(2 * TX * TY):
        s, e = rng_t[:, t]
        assert all(int(keys[j]) >> 32 == t for j in range(s, e))
        assert (e - s) == sum(1 for k, _ in pairs if k >> 32 == t)


# --------------------------------------------------------------------------------------------
# Tiled composite == tile-free brute force, exactly
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("mode", ["ref", "f64"])
def test_tiled_composite_equals_bruteforce(seed, mode):
    rng = np.random.default_rng(100 + seed)
    g = random_gaussians(64, rng, mean_range=0.35, scale_range=(0.04, 0.25), opacity_range=(0.05, 0.99))
    cam = look_at_camera([0.2, -0.1, 2.0], width=37, height=29)
    img = oracle.render(g, [cam], mode=mode)
    proj = img["proj"][0]
    ref = brute.composite(proj, g["opacity"].astype(np.float64), g["rgb"].astype(np.float64),
                          g["normal"].astype(np.float64), 37, 29, oracle.options_vector())
    for k in ("rgb", "normal", "depth", "T"):
        assert np.array_equal(img[k][0], ref[k]), k
    assert (img["n_contrib"][0] > 0).sum() > 300


@pytest.mark.parametrize("mode", ["ref", "f64"])
def test_tiled_composite_equals_bruteforce_on_thin_tilted_ellipses(mode):
    """Surfel-like splats (one long, one short and one near-zero axis, random orientations) give
    long thin screen ellipses at every angle, where the axis-aligned box of the 3-sigma ellipse is
    far smaller than the square of half width 3 sqrt(lambda_max): the tiled render must still equal
    the tile-free brute force exactly, so the box holds every pixel the 3-sigma test accepts."""
    rng = np.random.default_rng(77)
    n = 48
    g = random_gaussians(n, rng, mean_range=0.35, opacity_range=(0.3, 0.99))
    g["scale"] = np.ascontiguousarray(np.stack([rng.uniform(0.08, 0.3, n), rng.uniform(0.002, 0.02, n),
                                                np.full(n, 5e-4)]).astype(np.float32))
    W, H = 61, 47
    cam = look_at_camera([0.4, -0.3, 1.6], width=W, height=H)
    img = oracle.render(g, [cam], mode=mode)
    proj = img["proj"][0]
    ref = brute.composite(proj, g["opacity"].astype(np.float64), g["rgb"].astype(np.float64),
                          g["normal"].astype(np.float64), W, H, oracle.options_vector())
    for k in ("rgb", "normal", "depth", "T"):
        assert np.array_equal(img[k][0], ref[k]), k
    assert (img["n_contrib"][0] > 0).sum() > 300
    # the regime where the box matters: its area is well below the square's
    v = proj["valid"] == 1
    A, B, C = (np.asarray(proj[k], np.float64)[v] for k in ("A", "B", "C"))
    lam_max = 1.0 / np.linalg.eigvalsh(np.stack([np.stack([A, B], -1), np.stack([B, C], -1)], -2))[:, 0]
    square = (2 * np.ceil(3 * np.sqrt(lam_max))) ** 2
    box = 4 * np.asarray(proj["ex"], np.float64)[v] * np.asarray(proj["ey"], np.float64)[v]
    assert v.sum() > 40 and np.mean(box / square) < 0.6


# --------------------------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------------------------
def _c1_scene(n=2000, seed=1001):
    rng = np.random.default_rng(seed)
    return random_gaussians(n, rng), look_at_camera([0, 0, 3], width=128, height=128)


def test_permutation_invariance():
    g, cam = _c1_scene()
    p = oracle.project_f32(g, cam)
    z = p["z"][p["valid"] == 1]
    assert np.unique(z).size == z.size           # no FP32 depth ties
    perm = np.random.default_rng(9).permutation(2000)
    gp = {k: np.ascontiguousarray(v[..., perm]) for k, v in g.items()}
    a, b = oracle.render(g, [cam]), oracle.render(gp, [cam])
    for k in ("rgb", "normal", "depth", "alpha"):
        assert np.array_equal(a[k], b[k]), k


def test_opaque_front_layer_hides_everything_behind():
    g, cam = _c1_scene()
    wall = gauss([[0, 0, 1.0], [0, 0, 1.01], [0, 0, 1.02]], scales=[[10.0, 10.0, 0.01]] * 3,
                 opac=[1.0] * 3)
    both = {k: np.concatenate([wall[k], g[k]], axis=-1) for k in g}
    img1 = oracle.render(both, [cam])
    g2 = {k: v.copy() for k, v in g.items()}
    g2["rgb"] = np.random.default_rng(3).uniform(0, 1, g2["rgb"].shape).astype(np.float32)
    g2["normal"] = -g2["normal"]
    img2 = oracle.render({k: np.concatenate([wall[k], g2[k]], axis=-1) for k in g}, [cam])
    img3 = oracle.render(wall, [cam])
    for k in ("rgb", "normal", "depth", "alpha"):
        assert np.array_equal(img1[k], img2[k]), k
        assert np.array_equal(img1[k], img3[k]), k
    assert np.all((img1["n_contrib"] >= 2) & (img1["n_contrib"] <= 3))
    assert np.all(img1["T"] < 1e-4)


def test_faint_splat_insertion_changes_nothing():
    g, cam = _c1_scene()
    faint = gauss([[0, 0, 0.5]], scales=[[0.3] * 3], opac=[np.float32(1 / 255) * np.float32(0.99)])
    img1 = oracle.render(g, [cam])
    img2 = oracle.render({k: np.concatenate([faint[k], g[k]], axis=-1) for k in g}, [cam])
    for k in ("rgb", "normal", "depth", "alpha"):
        assert np.array_equal(img1[k], img2[k]), k


def test_tile_size_independence():
    g, cam = _c1_scene()
    a = oracle.render(g, [cam], tile=16)
    b = oracle.render(g, [cam], tile=8)
    for k in ("rgb", "normal", "depth", "alpha"):
        assert np.array_equal(a[k], b[k]), k


# --------------------------------------------------------------------------------------------
# Adjoint vs central finite differences (FP64)
# --------------------------------------------------------------------------------------------
def _fd_scene():
    rng = np.random.default_rng(77)
    g = random_gaussians(10, rng, mean_range=0.35, scale_range=(0.05, 0.15), opacity_range=(0.2, 0.95))
    g = {k: v.astype(np.float64) for k, v in g.items()}
    cams = [look_at_camera([0.3, 0.2, 2.2], width=40, height=36), look_at_camera([-1.0, 0.4, 1.9], width=40, height=36)]
    C, H, W = 2, 36, 40
    grng = np.random.default_rng(78)
    go = dict(rgb=grng.normal(size=(C, 3, H, W)), normal=grng.normal(size=(C, 3, H, W)),
              depth=grng.normal(size=(C, H, W)), alpha=grng.normal(size=(C, H, W)))
    return g, cams, go


def _loss(g, cams, go, cov6=None, opts=None):
    img = oracle.render(g, cams, opts, mode="f64", cov6=cov6)
    return float((img["rgb"] * go["rgb"]).sum() + (img["normal"] * go["normal"]).sum()
                 + (img["depth"] * go["depth"]).sum() + (img["alpha"] * go["alpha"]).sum())


# default options, and a background colour with an alpha clamp that binds (opacities up to 0.95
# against alpha_max 0.8) and a stop threshold far below the default
FD_OPTIONS = [None, dict(bg=(0.3, 0.6, 0.2), alpha_max=0.8, t_eps=1e-7)]


@pytest.mark.parametrize("opts", FD_OPTIONS)
def test_adjoint_matches_finite_differences(opts):
    g, cams, go = _fd_scene()
    grads, sabs, sig0 = oracle.backward(g, cams, go, opts)
    params = [("mean", 3), ("quat", 4), ("scale", 3), ("opacity", 1), ("rgb", 3), ("normal", 3)]
    checked = skipped = 0
    for i in range(10):
        for name, k in params:
            for c in range(k):
                arr = g[name] if name != "opacity" else g[name][None, :]
                theta = arr[c, i]
                h = 1e-6 * max(1.0, abs(theta))
                gp = {kk: vv.copy() for kk, vv in g.items()}
                gm = {kk: vv.copy() for kk, vv in g.items()}
                (gp[name] if name != "opacity" else gp[name][None, :])[c, i] += h
                (gm[name] if name != "opacity" else gm[name][None, :])[c, i] -= h
                _, _, sp = oracle.backward(gp, cams, go, opts, sabs_for=-2)
                _, _, sm = oracle.backward(gm, cams, go, opts, sabs_for=-2)
                if sp != sig0 or sm != sig0:
                    skipped += 1
                    continue
                fd = (_loss(gp, cams, go, opts=opts) - _loss(gm, cams, go, opts=opts)) / (2 * h)
                an = grads[name][c, i]
                tol = 1e-6 * sabs[name][c, i] + 1e-7
                assert abs(fd - an) <= tol, (name, c, i, fd, an, sabs[name][c, i])
                checked += 1
    assert checked > 150 and skipped < 20


def test_covariance_adjoint_matches_finite_differences():
    g, cams, go = _fd_scene()
    S = oracle.covariance_f64(g["quat"], g["scale"])
    cov6 = np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]])
    grads, sabs, sig0 = oracle.backward(g, cams, go, cov6=cov6)
    grads_q, _, _ = oracle.backward(g, cams, go, sabs_for=-2)
    # same render whichever way Sigma enters
    assert np.allclose(grads["cov6"], grads_q["cov6"], rtol=1e-9, atol=1e-12)
    checked = 0
    for i in range(10):
        for c in range(6):
            h = 1e-7 * max(1e-3, abs(cov6[c, i]))
            cp, cm = cov6.copy(), cov6.copy()
            cp[c, i] += h
            cm[c, i] -= h
            if oracle.backward(g, cams, go, cov6=cp, sabs_for=-2)[2] != sig0:
                continue
            if oracle.backward(g, cams, go, cov6=cm, sabs_for=-2)[2] != sig0:
                continue
            fd = (_loss(g, cams, go, cp) - _loss(g, cams, go, cm)) / (2 * h)
            an = grads["cov6"][c, i]
            assert abs(fd - an) <= 1e-5 * sabs["cov6"][c, i] + 1e-4, (c, i, fd, an)
            checked += 1
    assert checked > 40
