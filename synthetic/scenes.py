"""Seeded synthetic workloads shaped like the paper's (its datasets are not available).

The paper evaluates on scanned humans and captured scenes (Section 4.1). Those datasets are not
here, so every workload is procedural:

* ``random_gaussians``: the small forward case, 2,000 ellipsoids with uniform means in [-1,1]^3,
  random rotations, log-uniform per-axis scales, uniform opacity and colour, random unit normals.
* ``make_surface``: a union of 6 spheres and 4 tori with random radii, orientations and centres,
  normalised into the 2x2x2 box around the origin (as Section 3.3 does with its meshes), sampled
  area-uniformly, optionally quantised to the 10-bit lattice of Section 3.3 (scale 512, round),
  and coloured with 3-octave value noise.
* ``deformed_surface``: the same union with radii modulated over time, for dynamic sequences.
* ``look_at_camera`` / ``orbit_cameras``: pinhole cameras (OpenCV axes: x right, y down,
  z forward) with a 60 degree vertical field of view and the principal point at the image centre.

All arrays are float32 and planar (component-major ``[k][n]``), the layout the renderer consumes.
Nothing here projects, composites or estimates ellipsoids.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

# Seeds: numpy default_rng(1000 + workload id); held-out evaluation clouds use 2000+.
CONFIG_SEEDS = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005, "headline": 1006}


@dataclass
class Camera:
    """World-to-camera rigid transform x_c = T p + t (the W of Eq. 3) plus pinhole intrinsics."""
    T: np.ndarray          # (3, 3) float32, row-major
    t: np.ndarray          # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    eye: np.ndarray = field(default=None)

    def as_dict(self):
        return dict(T=self.T, t=self.t, fx=self.fx, fy=self.fy, cx=self.cx, cy=self.cy,
                    width=self.width, height=self.height)


def focal_for_vfov(height: int, vfov_deg: float = 60.0) -> float:
    """Focal length in pixels for a vertical field of view."""
    return (height / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)


def look_at_camera(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), width=128, height=128,
                   vfov_deg=60.0) -> Camera:
    """Camera at ``eye`` looking at ``target``; rows of T are (right, down, forward)."""
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    T = np.stack([right, down, fwd])
    t = -T @ eye
    f = focal_for_vfov(height, vfov_deg)
    f32 = float(np.float32(f))
    return Camera(T=T.astype(np.float32), t=t.astype(np.float32), fx=f32, fy=f32,
                  cx=float(np.float32(width / 2.0)), cy=float(np.float32(height / 2.0)),
                  width=int(width), height=int(height), eye=eye)


def orbit_cameras(n: int, rng: np.random.Generator, radius=3.0, width=1024, height=1024,
                  elev_range_deg=(-30.0, 30.0)) -> list:
    """``n`` cameras on a circle of radius 3 around the origin: azimuth k*360/n degrees,
    elevation uniform in the given range, all looking at the origin with +y up."""
    cams = []
    elev = rng.uniform(elev_range_deg[0], elev_range_deg[1], size=n)
    for k in range(n):
        az = 2.0 * math.pi * k / n
        el = math.radians(elev[k])
        eye = radius * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
        cams.append(look_at_camera(eye, width=width, height=height))
    return cams


def random_gaussians(n: int, rng: np.random.Generator, mean_range=1.0, scale_range=(0.005, 0.05),
                     opacity_range=(0.1, 0.99)) -> dict:
    """Random ellipsoids of the small forward workload (planar float32 arrays)."""
    mean = rng.uniform(-mean_range, mean_range, size=(3, n))
    q = rng.standard_normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    lo, hi = math.log(scale_range[0]), math.log(scale_range[1])
    scale = np.exp(rng.uniform(lo, hi, size=(3, n)))
    opacity = rng.uniform(opacity_range[0], opacity_range[1], size=n)
    rgb = rng.uniform(0.0, 1.0, size=(3, n))
    nrm = rng.standard_normal(size=(3, n))
    nrm /= np.linalg.norm(nrm, axis=0, keepdims=True)
    return dict(mean=mean.astype(np.float32), quat=q.astype(np.float32),
                scale=scale.astype(np.float32), opacity=opacity.astype(np.float32),
                rgb=rgb.astype(np.float32), normal=nrm.astype(np.float32))


def quantize_10bit(p: np.ndarray) -> np.ndarray:
    """Snap coordinates in [-1,1] to the centres of a 1024^3 lattice (scale 512, Section 3.3)."""
    idx = np.clip(np.floor((p.astype(np.float64) + 1.0) * 512.0), 0, 1023)
    return (idx + 0.5) / 512.0 - 1.0


class _ValueNoise:
    """3-octave value noise in [0,1]: lattice frequencies 4/8/16, amplitudes 1/0.5/0.25,
    smoothstep-weighted trilinear interpolation of random lattice values."""

    FREQS = (4, 8, 16)
    AMPS = (1.0, 0.5, 0.25)

    def __init__(self, rng: np.random.Generator, channels=3):
        self.tables = [[rng.uniform(0.0, 1.0, size=(f + 1, f + 1, f + 1)) for f in self.FREQS]
                       for _ in range(channels)]

    def __call__(self, p: np.ndarray) -> np.ndarray:
        p = np.asarray(p, dtype=np.float64)
        out = np.zeros((len(self.tables), p.shape[1]), dtype=np.float64)
        for f, amp, oi in zip(self.FREQS, self.AMPS, range(3)):
            g = np.clip((p + 1.0) * 0.5 * f, 0.0, float(f))
            i0 = np.minimum(np.floor(g).astype(np.int64), f - 1)
            fr = g - i0
            w = fr * fr * (3.0 - 2.0 * fr)
            for c, tabs in enumerate(self.tables):
                tab = tabs[oi]
                acc = np.zeros(p.shape[1])
                for dx in (0, 1):
                    wx = w[0] if dx else 1.0 - w[0]
                    for dy in (0, 1):
                        wy = w[1] if dy else 1.0 - w[1]
                        for dz in (0, 1):
                            wz = w[2] if dz else 1.0 - w[2]
                            acc += wx * wy * wz * tab[i0[0] + dx, i0[1] + dy, i0[2] + dz]
                out[c] += amp * acc
        return out / sum(self.AMPS)


class ProceduralSurface:
    """Union (no CSG) of spheres and tori, normalised into [-1,1]^3."""

    def __init__(self, rng: np.random.Generator, n_spheres=6, n_tori=4, radius_range=(0.2, 0.6),
                 center_range=0.5, torus_minor_ratio=1.0 / 3.0, margin_scale=1.0):
        self.kinds = ["sphere"] * n_spheres + ["torus"] * n_tori
        k = len(self.kinds)
        self.radius = rng.uniform(radius_range[0], radius_range[1], size=k)
        self.minor_ratio = torus_minor_ratio
        self.center = rng.uniform(-center_range, center_range, size=(k, 3))
        self.rot = Rotation.random(k, random_state=rng).as_matrix()
        self.phase = rng.uniform(0.0, 2.0 * math.pi, size=k)
        self.noise = _ValueNoise(rng)
        # Normalisation from the analytic bounding box of the union, with radii scaled by
        # margin_scale so deformed versions stay inside the box.
        lo = np.full(3, np.inf)
        hi = np.full(3, -np.inf)
        for i, kind in enumerate(self.kinds):
            r = self.radius[i] * margin_scale
            if kind == "sphere":
                ext = np.full(3, r)
            else:
                axis = self.rot[i][:, 2]
                ext = r * np.sqrt(np.clip(1.0 - axis ** 2, 0.0, 1.0)) + r * self.minor_ratio
            lo = np.minimum(lo, self.center[i] - ext)
            hi = np.maximum(hi, self.center[i] + ext)
        self.norm_center = 0.5 * (lo + hi)
        self.norm_scale = 2.0 * (1.0 - 1e-3) / float(np.max(hi - lo))

    def _areas(self, radius_scale):
        a = []
        for i, kind in enumerate(self.kinds):
            r = self.radius[i] * radius_scale[i]
            a.append(4 * math.pi * r * r if kind == "sphere" else 4 * math.pi ** 2 * r * (r * self.minor_ratio))
        return np.asarray(a)

    def sample(self, n: int, rng: np.random.Generator, radius_scale=None, with_normals=False):
        """``n`` area-uniform points on the union, normalised into [-1,1]^3, shape (3, n) float64;
        with ``with_normals`` also their analytic outward unit normals (3, n) (same random draws)."""
        if radius_scale is None:
            radius_scale = np.ones(len(self.kinds))
        areas = self._areas(radius_scale)
        counts = rng.multinomial(n, areas / areas.sum())
        pts, nrms = [], []
        for i, (kind, m) in enumerate(zip(self.kinds, counts)):
            if m == 0:
                continue
            r = self.radius[i] * radius_scale[i]
            if kind == "sphere":
                d = rng.standard_normal(size=(3, m))
                d /= np.linalg.norm(d, axis=0, keepdims=True)
                local = r * d
                local_n = d
            else:
                rr = r * self.minor_ratio
                theta = np.empty(0)
                while theta.size < m:   # area element is proportional to (R + r cos theta)
                    th = rng.uniform(0.0, 2.0 * math.pi, size=2 * (m - theta.size) + 16)
                    acc = rng.uniform(0.0, r + rr, size=th.size) < (r + rr * np.cos(th))
                    theta = np.concatenate([theta, th[acc]])
                theta = theta[:m]
                phi = rng.uniform(0.0, 2.0 * math.pi, size=m)
                ring = r + rr * np.cos(theta)
                local = np.stack([ring * np.cos(phi), ring * np.sin(phi), rr * np.sin(theta)])
                local_n = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), np.sin(theta)])
            pts.append(self.center[i][:, None] + self.rot[i] @ local)
            nrms.append(self.rot[i] @ local_n)
        p = np.concatenate(pts, axis=1)
        perm = rng.permutation(p.shape[1])
        p = np.ascontiguousarray(p[:, perm])
        p = (p - self.norm_center[:, None]) * self.norm_scale
        if with_normals:
            return p, np.ascontiguousarray(np.concatenate(nrms, axis=1)[:, perm])
        return p

    def color(self, p: np.ndarray) -> np.ndarray:
        """Value-noise RGB in [0,1] at positions p (3, n)."""
        return self.noise(p)


def make_surface(n: int, seed: int, quantize=True, margin_scale=1.0):
    """Points and colours of the procedural union: returns (surface, xyz float32 (3,n), rgb float32 (3,n))."""
    rng = np.random.default_rng(seed)
    surf = ProceduralSurface(rng, margin_scale=margin_scale)
    p = surf.sample(n, rng)
    if quantize:
        p = quantize_10bit(p)
    rgb = surf.color(p)
    return surf, np.ascontiguousarray(p, np.float32), np.ascontiguousarray(rgb, np.float32)


def deformed_surface(surf: ProceduralSurface, frame: int, n: int, rng: np.random.Generator,
                     period=30, amplitude=0.2, noise_std=0.002):
    """Frame ``frame`` of a deforming sequence: every radius is scaled by
    1 + amplitude*sin(2*pi*frame/period + phase_i); positions get N(0, noise_std^2) noise."""
    scale = 1.0 + amplitude * np.sin(2.0 * math.pi * frame / period + surf.phase)
    p = surf.sample(n, rng, radius_scale=scale)
    p = p + rng.normal(0.0, noise_std, size=p.shape)
    rgb = surf.color(p)
    return np.ascontiguousarray(p, np.float32), np.ascontiguousarray(rgb, np.float32)
