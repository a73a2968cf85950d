"""Pins of the late-shading reference: closed forms of the Blinn-Phong terms on constructed normal
maps, the view rays of the pinhole camera, and background pass-through."""
import numpy as np

from oracle import shading as S
from synthetic import look_at_camera

LIGHT = dict(dir=(0.0, 0.0, 1.0), color=(1.0, 1.0, 1.0), ambient=0.1, diffuse=0.7, specular=0.2, shininess=16.0)


def test_view_rays_point_back_to_the_camera():
    cam = look_at_camera([0.0, 0.0, 3.0], width=9, height=7)
    v = S.pixel_view_dirs(cam, 9, 7)
    assert np.allclose(np.linalg.norm(v, axis=0), 1.0)
    # at the principal point the direction back to the camera is minus the optical axis (the
    # third row of the world-to-camera rotation): +z here, the camera sitting at z = 3
    c = cam.as_dict()
    T = np.asarray(c["T"], np.float64).reshape(3, 3)
    centre = v[:, 3, 4]                      # pixel (4, 3) has its centre at the principal point
    assert np.allclose(centre, -T[2], atol=1e-12) and np.allclose(centre, [0.0, 0.0, 1.0])
    # a pixel d to the right: the ray angle is atan(d / f)
    ang = np.arccos(np.clip(np.dot(v[:, 3, 8], centre), -1, 1))
    assert np.isclose(np.tan(ang), 4.0 / float(c["fx"]))


def test_lambert_and_specular_closed_forms():
    cam = look_at_camera([0.0, 0.0, 3.0], width=5, height=5)
    rgb = np.full((1, 3, 5, 5), 0.5)
    alpha = np.ones((1, 5, 5))
    # normals tilted by theta from the light direction (+z) in the x-z plane
    th = np.deg2rad(60.0)
    nrm = np.zeros((1, 3, 5, 5))
    nrm[0, 0], nrm[0, 2] = np.sin(th) * 2.0, np.cos(th) * 2.0          # unnormalised on purpose
    out = S.shade(rgb, nrm, alpha, [cam], dict(LIGHT, specular=0.0))
    assert np.allclose(out, 0.5 * (0.1 + 0.7 * np.cos(th)))
    # a normal facing away from the light: ambient only; a zero normal: ambient, no specular
    nrm2 = -nrm
    assert np.allclose(S.shade(rgb, nrm2, alpha, [cam], LIGHT), 0.5 * 0.1)
    assert np.allclose(S.shade(rgb, np.zeros_like(nrm), alpha, [cam], LIGHT), 0.5 * 0.1)
    # mirror configuration at the centre pixel: camera on the light axis, normal = h gives n.h = 1
    n3 = np.zeros((1, 3, 5, 5))
    v = S.pixel_view_dirs(cam, 5, 5)
    h = np.array([0.0, 0.0, 1.0]) + v[:, 2, 2]
    h /= np.linalg.norm(h)
    n3[0, :, 2, 2] = h
    o3 = S.shade(rgb, n3, alpha, [cam], LIGHT)
    ndl = h[2]
    assert np.allclose(o3[0, :, 2, 2], 0.5 * (0.1 + 0.7 * ndl) + 0.2)


def test_background_and_partial_coverage():
    cam = look_at_camera([0.0, 0.0, 3.0], width=4, height=4)
    bg = (0.2, 0.3, 0.4)
    alpha = np.zeros((1, 4, 4))
    rgb = np.broadcast_to(np.asarray(bg)[None, :, None, None], (1, 3, 4, 4)).copy()
    out = S.shade(rgb, np.zeros((1, 3, 4, 4)), alpha, [cam], LIGHT, bg=bg)
    assert np.allclose(out, rgb)                                        # uncovered: background only
    # half coverage: the premultiplied albedo is shaded, the background passes through
    alpha[:] = 0.5
    fg = 0.3
    rgb2 = fg + 0.5 * np.asarray(bg)[None, :, None, None] + np.zeros((1, 3, 4, 4))
    nrm = np.zeros((1, 3, 4, 4)); nrm[0, 2] = 1.0
    out2 = S.shade(rgb2, nrm, alpha, [cam], dict(LIGHT, specular=0.0), bg=bg)
    assert np.allclose(out2, fg * (0.1 + 0.7) + 0.5 * np.asarray(bg)[None, :, None, None])
