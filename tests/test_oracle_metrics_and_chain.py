"""Pins of three oracle parts that judge results: the image metrics (PSNR, SSIM), the exact-FP32
projection that fixes the binning, and the FP64 chain from screen-space gradients back to the
Gaussian parameters. No GPU involved.

* PSNR and SSIM against closed forms and an explicit per-window evaluation of the definition;
  the product's metric functions (used by training and by the quality figures) must equal them.
* The C++ exact-FP32 projection against a second, independently written numpy.float32 emulation
  of the same operation sequence: bit for bit.
* The C++ pull-back (conic -> screen covariance -> EWA Jacobian -> rotation and scale) against
  PyTorch FP64 autograd through a projection built another way: the rotation from quaternion
  sandwich products, the Jacobian of Eq. 4 by differentiating the pinhole map, the conic by a
  matrix inverse.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import emulate32, metrics
from synthetic import look_at_camera, make_surface, orbit_cameras, random_gaussians, CONFIG_SEEDS


# --------------------------------------------------------------------------------------------
# PSNR / SSIM (Section 4.1's quality metric; the SSIM term of the training loss)
# --------------------------------------------------------------------------------------------
def test_psnr_constant_offset_and_clamp():
    rng = np.random.default_rng(0)
    a = rng.uniform(0.2, 0.7, size=(2, 3, 16, 16))
    for d in (0.1, 0.01, 0.003):
        assert metrics.psnr(a, a + d) == pytest.approx(-20.0 * math.log10(d), abs=1e-9)
    # values beyond [0, 1] are clamped before the error is taken
    b = a.copy()
    b[0, 0, 0, 0] = 5.0
    c = a.copy()
    c[0, 0, 0, 0] = 1.0
    assert metrics.psnr(a, b) == metrics.psnr(a, c)
    assert metrics.psnr(a, a) == float("inf")


def test_ssim_identity_and_constant_images():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, size=(1, 3, 20, 24))
    assert metrics.ssim(x, x) == pytest.approx(1.0, abs=1e-12)
    for a, b in ((0.2, 0.7), (0.5, 0.5), (0.9, 0.05)):
        xa, xb = np.full((1, 1, 13, 13), a), np.full((1, 1, 13, 13), b)
        want = (2 * a * b + metrics.C1) / (a * a + b * b + metrics.C1)
        assert metrics.ssim(xa, xb) == pytest.approx(want, abs=1e-12)


def _window_stats_bruteforce(x, y, i0, j0):
    """Weighted means, variances and covariance of the 11x11 window at (i0, j0), by explicit
    loops over the Gaussian weights exp(-(di^2 + dj^2) / (2 * 1.5^2)), normalised."""
    wsum = 0.0
    acc = dict(mx=0.0, my=0.0, xx=0.0, yy=0.0, xy=0.0)
    for di in range(11):
        for dj in range(11):
            w = math.exp(-((di - 5) ** 2 + (dj - 5) ** 2) / (2 * 1.5 ** 2))
            a, b = x[i0 + di, j0 + dj], y[i0 + di, j0 + dj]
            wsum += w
            acc["mx"] += w * a
            acc["my"] += w * b
            acc["xx"] += w * a * a
            acc["yy"] += w * b * b
            acc["xy"] += w * a * b
    s = {k: v / wsum for k, v in acc.items()}
    return s["mx"], s["my"], s["xx"] - s["mx"] ** 2, s["yy"] - s["my"] ** 2, s["xy"] - s["mx"] * s["my"]


def test_ssim_equals_per_window_bruteforce():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=(14, 15))
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1)
    vals = []
    for i0 in range(14 - 10):
        for j0 in range(15 - 10):
            mx, my, sxx, syy, sxy = _window_stats_bruteforce(x, y, i0, j0)
            vals.append((2 * mx * my + 1e-4) * (2 * sxy + 9e-4) / ((mx * mx + my * my + 1e-4) * (sxx + syy + 9e-4)))
    assert metrics.ssim(x[None, None], y[None, None]) == pytest.approx(np.mean(vals), abs=1e-12)


@pytest.mark.parametrize("shift,scale", [(0.1, 1.0), (0.0, 0.5), (0.05, 1.7)])
def test_ssim_of_affine_copy_closed_form(shift, scale):
    """y = s x + t: per window mu_y = s mu_x + t, var_y = s^2 var_x, cov = s var_x, so
    SSIM = (2 mu_x mu_y + C1)(2 s var_x + C2) / ((mu_x^2 + mu_y^2 + C1)((1 + s^2) var_x + C2))."""
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 0.5, size=(12, 13))
    y = scale * x + shift
    vals = []
    for i0 in range(2):
        for j0 in range(3):
            mx, _, sxx, _, _ = _window_stats_bruteforce(x, x, i0, j0)
            my = scale * mx + shift
            vals.append((2 * mx * my + 1e-4) * (2 * scale * sxx + 9e-4) /
                        ((mx * mx + my * my + 1e-4) * ((1 + scale * scale) * sxx + 9e-4)))
    assert metrics.ssim(x[None, None], y[None, None]) == pytest.approx(np.mean(vals), abs=1e-12)


def test_product_metrics_equal_the_oracle():
    """The estimator's psnr (the quality figures) and ssim (the training loss) equal the pinned
    definitions (CPU tensors; the functions are device-agnostic)."""
    import torch
    from paper_2409_16504_amd.estimator import psnr, ssim
    rng = np.random.default_rng(4)
    a = rng.uniform(-0.1, 1.1, size=(2, 3, 32, 40))
    b = np.clip(a + rng.normal(0, 0.05, size=a.shape), -0.2, 1.2)
    ta, tb = torch.from_numpy(a), torch.from_numpy(b)
    assert psnr(ta, tb) == pytest.approx(metrics.psnr(a, b), abs=1e-9)
    ca, cb = np.clip(a, 0, 1), np.clip(b, 0, 1)
    assert float(ssim(torch.from_numpy(ca), torch.from_numpy(cb))) == pytest.approx(metrics.ssim(ca, cb), abs=1e-12)


# --------------------------------------------------------------------------------------------
# The exact-FP32 projection, written twice
# --------------------------------------------------------------------------------------------
def _same_bits(a, b):
    if a.dtype == np.float32:
        return np.array_equal(a.view(np.uint32), b.view(np.uint32))
    return np.array_equal(a, b)


def _check_projection(g, cam, opts=None):
    a = oracle.project_f32(g, cam, opts)
    b = emulate32.project(g, cam, opts)
    for k in ("valid", "u", "v", "z", "A", "B", "C", "ex", "ey", "rect", "count"):
        assert _same_bits(a[k], b[k]), (k, int(np.sum(a[k] != b[k])))
    return int(a["valid"].sum())


def test_fp32_projection_small_scene_bitexact():
    rng = np.random.default_rng(CONFIG_SEEDS[1])
    g = random_gaussians(2000, rng)
    assert _check_projection(g, look_at_camera([0, 0, 3], width=128, height=128)) == 2000
    # options that move every threshold
    _check_projection(g, look_at_camera([0.4, -0.3, 2.6], width=131, height=97),
                      dict(lowpass=0.0, sigma_cut=2.5, alpha_min=0.3, z_near=2.4))


def test_fp32_projection_surface_1080p_bitexact():
    from oracle import knn_pca as kp
    _, p, rgb = make_surface(60_000, 1006, quantize=True)
    est = kp.knn_pca(p, k=16, kappa=1.0)
    g = dict(mean=p, quat=est["quat"].astype(np.float32), scale=est["scale"].astype(np.float32),
             opacity=np.full(p.shape[1], 0.9, np.float32), rgb=rgb, normal=est["normal"].astype(np.float32))
    assert _check_projection(g, look_at_camera([0, 0, 3], width=1920, height=1080)) > 50_000
    for cam in orbit_cameras(3, np.random.default_rng(1003), width=1024, height=1024):
        _check_projection(g, cam)


def test_fp32_projection_culls_alike():
    rng = np.random.default_rng(9)
    g = random_gaussians(64, rng)
    g["mean"][2, :8] = 2.95                 # at the near plane of a camera at z = 3
    g["mean"][0, 8] = np.nan
    g["quat"][:, 9] = 0.0                    # zero quaternion: identity rotation
    g["opacity"][10] = 1e-3                  # below the alpha cut-off
    g["mean"][0, 11] = 40.0                  # off screen
    n_valid = _check_projection(g, look_at_camera([0, 0, 3], width=64, height=64))
    assert n_valid < 64 - 10


# --------------------------------------------------------------------------------------------
# The FP64 pull-back against autograd through an independently built projection
# --------------------------------------------------------------------------------------------
def _qmul(a, b):
    """Hamilton product of quaternions (w, x, y, z) stacked on the first axis."""
    import torch
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return torch.stack([aw * bw - ax * bx - ay * by - az * bz,
                        aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw])


def _screen_torch(mean, quat, scale, cov6, cam, lowpass):
    """(u, v, A, B, C, z) per Gaussian, FP64 torch, differentiable."""
    import torch
    n = mean.shape[1]
    if cov6 is None:
        q = quat / torch.sqrt((quat * quat).sum(0, keepdim=True))
        qc = q * torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=q.dtype)[:, None]
        cols = []
        for k in range(3):                    # R e_k = vector part of q (0, e_k) q*
            e = torch.zeros((4, n), dtype=q.dtype)
            e[1 + k] = 1.0
            cols.append(_qmul(_qmul(q, e), qc)[1:])
        R = torch.stack(cols, dim=-1).permute(1, 0, 2)          # (n, 3, 3), columns = axes
        Sig = R @ torch.diag_embed((scale * scale).T) @ R.transpose(1, 2)
    else:
        xx, xy, xz, yy, yz, zz = cov6
        Sig = torch.stack([torch.stack([xx, xy, xz], -1), torch.stack([xy, yy, yz], -1),
                           torch.stack([xz, yz, zz], -1)], -2)
    T = torch.tensor(np.asarray(cam["T"], np.float64).reshape(3, 3))
    t = torch.tensor(np.asarray(cam["t"], np.float64))
    xc = (T @ mean).T + t                                         # (n, 3), Eq. 3
    fx, fy, cx, cy = (float(np.float32(cam[k])) for k in ("fx", "fy", "cx", "cy"))

    def pinhole(p):
        return torch.stack([fx * p[:, 0] / p[:, 2] + cx, fy * p[:, 1] / p[:, 2] + cy], -1)

    uv = pinhole(xc)
    # the Jacobian of Eq. 4 by differentiating the pinhole map (kept in the graph)
    ju = torch.autograd.grad(uv[:, 0].sum(), xc, create_graph=True)[0]
    jv = torch.autograd.grad(uv[:, 1].sum(), xc, create_graph=True)[0]
    J = torch.stack([ju, jv], 1)                                 # (n, 2, 3)
    JT = J @ T
    Ss = JT @ Sig @ JT.transpose(1, 2) + lowpass * torch.eye(2, dtype=Sig.dtype)
    conic = torch.linalg.inv(Ss)
    return uv[:, 0], uv[:, 1], conic[:, 0, 0], conic[:, 0, 1], conic[:, 1, 1], xc[:, 2]


@pytest.mark.parametrize("use_cov", [False, True])
def test_pull_back_matches_autograd(use_cov):
    import torch
    rng = np.random.default_rng(31)
    n = 40
    g = random_gaussians(n, rng, mean_range=0.5, scale_range=(0.02, 0.2))
    g["quat"] = g["quat"] * rng.uniform(0.5, 2.0, size=(1, n))   # not unit: normalisation enters
    g = {k: v.astype(np.float64) for k, v in g.items()}
    cams = orbit_cameras(2, rng, radius=2.5, width=200, height=150)
    lp = float(np.float32(0.3))
    cov6 = None
    if use_cov:
        S = oracle.covariance_f64(g["quat"], g["scale"])
        cov6 = np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]])
    for cam in cams:
        c = cam if isinstance(cam, dict) else cam.as_dict()
        sg = rng.normal(size=(13, n))
        want = oracle.pull_back(g, c, sg, cov6=cov6)
        mean = torch.tensor(g["mean"], requires_grad=True)
        quat = torch.tensor(g["quat"], requires_grad=True)
        scale = torch.tensor(g["scale"], requires_grad=True)
        c6 = torch.tensor(cov6, requires_grad=True) if use_cov else None
        opac = torch.tensor(g["opacity"], requires_grad=True)
        rgb = torch.tensor(g["rgb"], requires_grad=True)
        nrm = torch.tensor(g["normal"], requires_grad=True)
        mean_x = mean * 1.0
        u, v, A, B, C, z = _screen_torch(mean_x, quat, scale, c6, c, lp)
        sgt = torch.tensor(sg)
        # the conic's off-diagonal entry B enters the quadratic form twice (2 B dx dy); the
        # screen-space gradient of B is taken with respect to that one parameter
        L = (sgt[0] * u + sgt[1] * v + sgt[2] * A + sgt[3] * B + sgt[4] * C + sgt[5] * opac +
             sgt[6] * z + (sgt[7:10] * rgb).sum(0) + (sgt[10:13] * nrm).sum(0)).sum()
        params = [mean, opac, rgb, nrm] + ([c6] if use_cov else [quat, scale])
        got = torch.autograd.grad(L, params)
        pairs = [("mean", got[0]), ("opacity", got[1][None]), ("rgb", got[2]), ("normal", got[3])]
        pairs += [("cov6", got[4])] if use_cov else [("quat", got[4]), ("scale", got[5])]
        for name, t in pairs:
            a = t.detach().numpy()
            b = want[name]
            scale_ = np.abs(a).max() + 1e-30
            assert np.max(np.abs(a - b)) <= 1e-10 * scale_, (name, np.max(np.abs(a - b)), scale_)
