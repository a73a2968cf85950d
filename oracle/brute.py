"""Tile-free brute-force compositing for tiny scenes (test infrastructure only).

For every pixel, every projected splat is visited in (FP32 depth, index) order and Eq. 1-2 are
applied directly: a splat contributes where its screen-space Mahalanobis distance is inside the
3-sigma boundary of Section 3.1 and its opacity reaches the cutoff; blending stops once the
transmittance falls below the stop threshold. No tiles, no keys, no sort of instances: this is
the definition the tiled oracle must reproduce exactly. Pure Python with ``math.exp`` so every
FP64 operation happens in the same order as the tiled C++ oracle.
"""
from __future__ import annotations

import math

import numpy as np


def composite(proj: dict, opacity, rgb, normal, width: int, height: int, opts_vec) -> dict:
    z_near, lowpass, sigma_cut, amin, amax, teps, bg0, bg1, bg2 = [float(x) for x in opts_vec]
    cut2 = sigma_cut * sigma_cut
    valid = np.nonzero(proj["valid"])[0]
    # the depth order is taken on the FP32 depth of the exact projection (an FP64 projection carries
    # it as "zf"; the FP32 projection's own depth is that value)
    zbits = np.asarray(proj["zf"] if "zf" in proj else proj["z"], np.float32).view(np.uint32)
    order = sorted(valid.tolist(), key=lambda i: (int(zbits[i]), i))
    u = [float(x) for x in proj["u"]]
    v = [float(x) for x in proj["v"]]
    A = [float(x) for x in proj["A"]]
    B = [float(x) for x in proj["B"]]
    C = [float(x) for x in proj["C"]]
    z = [float(x) for x in proj["z"]]
    o = [float(x) for x in np.asarray(opacity)]
    f_rgb = np.asarray(rgb, np.float64)
    f_nrm = np.asarray(normal, np.float64)
    out_rgb = np.zeros((3, height, width))
    out_nrm = np.zeros((3, height, width))
    out_d = np.zeros((height, width))
    out_T = np.ones((height, width))
    for y in range(height):
        for x in range(width):
            px, py = x + 0.5, y + 0.5
            T = 1.0
            acc = [0.0] * 7
            for g in order:
                dx = px - u[g]
                dy = py - v[g]
                q = A[g] * dx * dx + 2.0 * B[g] * dx * dy + C[g] * dy * dy
                if not (q <= cut2):
                    continue
                alpha = min(amax, o[g] * math.exp(-0.5 * q))
                if alpha < amin:
                    continue
                w = alpha * T
                for ch in range(3):
                    acc[ch] += w * f_rgb[ch, g]
                    acc[3 + ch] += w * f_nrm[ch, g]
                acc[6] += w * z[g]
                T = T * (1.0 - alpha)
                if T < teps:
                    break
            bg = (bg0, bg1, bg2)
            for ch in range(3):
                out_rgb[ch, y, x] = acc[ch] + T * bg[ch]
                out_nrm[ch, y, x] = acc[3 + ch]
            out_d[y, x] = acc[6]
            out_T[y, x] = T
    return dict(rgb=out_rgb, normal=out_nrm, depth=out_d, alpha=1.0 - out_T, T=out_T)
