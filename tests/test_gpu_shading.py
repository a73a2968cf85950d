"""GPU parity of late shading against the FP64 reference on seeded synthetic frames (colour,
normal map and coverage drawn at random: the images do not come from the GPU renderer)."""
import numpy as np
import pytest
import torch

from oracle import shading as S
from synthetic import look_at_camera

pytestmark = pytest.mark.gpu

LIGHT = dict(dir=(0.3, 0.8, 0.5), color=(1.0, 0.9, 0.8), ambient=0.15, diffuse=0.7, specular=0.3, shininess=24.0)


@pytest.fixture(scope="module")
def R():
    import paper_2409_16504_amd as P
    return P.Renderer(0)


def frames(rng, C, H, W, bg):
    a = rng.uniform(0, 1, (C, H, W))
    a[:, :3] = 0.0                                        # uncovered rows
    fg = rng.uniform(0, 1, (C, 3, H, W)) * a[:, None]
    rgb = fg + (1 - a[:, None]) * np.asarray(bg)[None, :, None, None]
    n = rng.normal(size=(C, 3, H, W)) * a[:, None]
    n[:, :, 3:5] = 0.0                                    # covered pixels with a zero normal
    return rgb.astype(np.float32), n.astype(np.float32), a.astype(np.float32)


@pytest.mark.parametrize("H,W", [(23, 37), (64, 64)])
def test_shading_matches_reference(R, H, W):
    rng = np.random.default_rng(H * 1000 + W)
    bg = (0.1, 0.2, 0.3)
    cams = [look_at_camera([3.0 * np.sin(t), 0.5, 3.0 * np.cos(t)], width=W, height=H) for t in (0.3, 2.0)]
    rgb, n, a = frames(rng, 2, H, W, bg)
    imgs = {k: torch.from_numpy(v).cuda() for k, v in dict(rgb=rgb, normal=n, alpha=a).items()}
    out = R.shade(imgs, cams, LIGHT, bg=bg).cpu().numpy().astype(np.float64)
    # FP64 reference on the same FP32 inputs; the normalisations and the power run in FP32 on the GPU
    ref = S.shade(rgb, n, a, cams, LIGHT, bg=bg)
    assert np.all(np.abs(out - ref) <= 2e-5 * np.abs(ref) + 2e-6), np.max(np.abs(out - ref))
    # in place gives the same result
    same = R.shade(imgs, cams, LIGHT, bg=bg, out=imgs["rgb"]).cpu().numpy()
    assert np.array_equal(same, out.astype(np.float32))


def test_shading_rejects_bad_arguments(R):
    cams = [look_at_camera([0.0, 0.0, 3.0], width=8, height=8)]
    z = torch.zeros((1, 3, 8, 8), device="cuda")
    imgs = dict(rgb=z, normal=z.clone(), alpha=torch.zeros((1, 8, 8), device="cuda"))
    with pytest.raises(RuntimeError):
        R.shade(imgs, cams, dict(LIGHT, dir=(0.0, 0.0, 0.0)))
    with pytest.raises(RuntimeError):
        R.shade(imgs, cams, dict(LIGHT, shininess=0.0))
    with pytest.raises(ValueError):
        R.shade(dict(imgs, alpha=torch.zeros((1, 7, 8), device="cuda")), cams, LIGHT)
