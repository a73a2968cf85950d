"""Second, independent emulation of the FP32 projection that fixes the binning (test
infrastructure only, like the rest of ``oracle``).

The binning contract is an exact FP32 operation sequence for the EWA projection of Section 3.1
(Eq. 3 view transform, Eq. 4 screen covariance): every step is one IEEE-754 single-precision
operation rounded to nearest-even, evaluated left to right, with no fused multiply-add. The C++
oracle (``orc_project_f32``) implements it one Gaussian at a time; this module writes the same
sequence again, vectorised over Gaussians with numpy float32 arrays (each ufunc call rounds its
result to FP32, and numpy never contracts a multiply and an add), so that a regrouped sum or a
reordered product in either implementation shows up as a bit difference.

The sequence, step by step:
  (1) |q|^2 = ((w w + x x) + y y) + z z; q / sqrt(|q|^2) per component (q = 0: identity).
  (2) R from the products xx, yy, zz, xy, xz, yz, wx, wy, wz of the unit quaternion (Hamilton):
      diagonal 1 - 2 (sum of two squares), off-diagonal 2 (product -/+ product).
  (3) v_k = s_k s_k; Sigma_jk = ((R_j0 v0) R_k0 + (R_j1 v1) R_k1) + (R_j2 v2) R_k2 for j <= k,
      mirrored below the diagonal.
  (4) x_c = ((T_r0 p_x + T_r1 p_y) + T_r2 p_z) + t_r for each row r.
  (5) u = (f_x x) / z + c_x, v = (f_y y) / z + c_y.
  (6) j00 = f_x / z, j02 = -((f_x x) / (z z)); j11 = f_y / z, j12 = -((f_y y) / (z z)).
  (7) M = J T: M_0k = j00 T_0k + j02 T_2k, M_1k = j11 T_1k + j12 T_2k.
  (8) P = M Sigma with P_rk = (M_r0 S_0k + M_r1 S_1k) + M_r2 S_2k; a = ((P_00 M_00 + P_01 M_01)
      + P_02 M_02) + lowpass, b = (P_00 M_10 + P_01 M_11) + P_02 M_12, c likewise from row 1 plus
      lowpass.
  (9) det = a c - b b; A = c / det, B = -(b / det), C = a / det; half extents of the
      sigma_cut ellipse's axis-aligned box e_x = (sigma_cut sqrt(a)) 1.001 + 0.01 and
      e_y = (sigma_cut sqrt(c)) 1.001 + 0.01.
 (10) tile range floor((u - e_x) / 16) .. floor((u + e_x) / 16) clamped to the frame, likewise in
      y with e_y.
Culled (valid = 0): any non-finite input field, opacity below alpha_min (alpha <= o never reaches
the cut-off), z <= z_near or a non-finite camera-space point, det <= 0, a non-finite u, v, conic or
extents, and a rectangle that misses the frame.
"""
from __future__ import annotations

import numpy as np

F = np.float32


def _f(x):
    return np.asarray(x, dtype=F)


def project(g: dict, cam: dict, opts: dict | None = None, tile: int = 16) -> dict:
    """Outputs as ``oracle.project_f32``: valid, u, v, z, A, B, C, ex, ey, rect[4] (x0, x1, y0,
    y1 inclusive), count."""
    from . import DEFAULT_OPTIONS
    o = dict(DEFAULT_OPTIONS)
    if opts:
        o.update(opts)
    z_near, lowpass, cut, amin = F(o["z_near"]), F(o["lowpass"]), F(o["sigma_cut"]), F(o["alpha_min"])
    c = cam if isinstance(cam, dict) else cam.as_dict()
    T = _f(c["T"]).reshape(3, 3)
    t = _f(c["t"]).reshape(3)
    fx, fy, cx, cy = F(c["fx"]), F(c["fy"]), F(c["cx"]), F(c["cy"])
    W, H = int(c["width"]), int(c["height"])
    TX, TY = (W + tile - 1) // tile, (H + tile - 1) // tile

    p = _f(g["mean"])
    q = _f(g["quat"])
    s = _f(g["scale"])
    op = _f(g["opacity"])
    n = op.shape[-1]
    with np.errstate(all="ignore"):
        ok = np.ones(n, bool)
        for k in ("mean", "quat", "scale", "opacity", "rgb", "normal"):
            arr = _f(g[k]).reshape(-1, n)
            ok &= np.isfinite(arr).all(axis=0)
        ok &= op >= amin

        # (1) unit quaternion
        w, x, y, z = q[0], q[1], q[2], q[3]
        nq = w * w + x * x
        nq = nq + y * y
        nq = nq + z * z
        ok &= np.isfinite(nq)
        zero = nq == F(0)
        ln = np.sqrt(nq)
        ln = np.where(zero, F(1), ln)
        w = np.where(zero, F(1), w / ln)
        x = np.where(zero, F(0), x / ln)
        y = np.where(zero, F(0), y / ln)
        z = np.where(zero, F(0), z / ln)
        # (2) rotation (columns are the ellipsoid's axes)
        xx, yy, zz = x * x, y * y, z * z
        xy, xz, yz = x * y, x * z, y * z
        wx, wy, wz = w * x, w * y, w * z
        one, two = F(1), F(2)
        R = [[one - two * (yy + zz), two * (xy - wz), two * (xz + wy)],
             [two * (xy + wz), one - two * (xx + zz), two * (yz - wx)],
             [two * (xz - wy), two * (yz + wx), one - two * (xx + yy)]]
        # (3) Sigma = R diag(s^2) R^T, upper triangle computed
        v = [s[0] * s[0], s[1] * s[1], s[2] * s[2]]
        S = [[None] * 3 for _ in range(3)]
        for j in range(3):
            for k in range(j, 3):
                e = (R[j][0] * v[0]) * R[k][0] + (R[j][1] * v[1]) * R[k][1]
                e = e + (R[j][2] * v[2]) * R[k][2]
                S[j][k] = e
                S[k][j] = e
        # (4) camera-space point (Eq. 3)
        xc = [((T[r, 0] * p[0] + T[r, 1] * p[1]) + T[r, 2] * p[2]) + t[r] for r in range(3)]
        ok &= (xc[2] > z_near) & np.isfinite(xc[0]) & np.isfinite(xc[1]) & np.isfinite(xc[2])
        # (5) pixel position
        fxx, fyy = fx * xc[0], fy * xc[1]
        u = fxx / xc[2] + cx
        vv = fyy / xc[2] + cy
        # (6) Jacobian of the perspective map (Eq. 4)
        z2 = xc[2] * xc[2]
        j00, j02 = fx / xc[2], -(fxx / z2)
        j11, j12 = fy / xc[2], -(fyy / z2)
        # (7) M = J T
        M0 = [j00 * T[0, k] + j02 * T[2, k] for k in range(3)]
        M1 = [j11 * T[1, k] + j12 * T[2, k] for k in range(3)]
        # (8) screen covariance with the low-pass
        P0 = [(M0[0] * S[0][k] + M0[1] * S[1][k]) + M0[2] * S[2][k] for k in range(3)]
        P1 = [(M1[0] * S[0][k] + M1[1] * S[1][k]) + M1[2] * S[2][k] for k in range(3)]
        a = ((P0[0] * M0[0] + P0[1] * M0[1]) + P0[2] * M0[2]) + lowpass
        b = (P0[0] * M1[0] + P0[1] * M1[1]) + P0[2] * M1[2]
        cc = ((P1[0] * M1[0] + P1[1] * M1[1]) + P1[2] * M1[2]) + lowpass
        # (9) conic and the padded half extents of the sigma_cut ellipse's box
        det = a * cc - b * b
        ok &= det > F(0)
        A = cc / det
        B = -(b / det)
        C = a / det
        ex = (cut * np.sqrt(a)) * F(1.001) + F(0.01)
        ey = (cut * np.sqrt(cc)) * F(1.001) + F(0.01)
        for arr in (u, vv, A, B, C, ex, ey):
            ok &= np.isfinite(arr)
        # (10) tile rectangle of the box [u - e_x, u + e_x] x [v - e_y, v + e_y]
        ts = F(tile)
        x0, x1 = np.floor((u - ex) / ts), np.floor((u + ex) / ts)
        y0, y1 = np.floor((vv - ey) / ts), np.floor((vv + ey) / ts)
        ok &= ~((x1 < 0) | (y1 < 0) | (x0 > TX - 1) | (y0 > TY - 1))
    out = dict(valid=ok.astype(np.uint8))
    for name, arr in (("u", u), ("v", vv), ("z", xc[2]), ("A", A), ("B", B), ("C", C), ("ex", ex), ("ey", ey)):
        out[name] = np.where(ok, arr, F(0)).astype(F)
    with np.errstate(invalid="ignore"):
        rect = np.stack([np.maximum(x0, 0), np.minimum(x1, TX - 1), np.maximum(y0, 0), np.minimum(y1, TY - 1)])
    out["rect"] = np.where(ok[None, :], rect, 0).astype(np.int32)
    r = out["rect"].astype(np.int64)
    out["count"] = np.where(ok, (r[1] - r[0] + 1) * (r[3] - r[2] + 1), 0).astype(np.uint32)
    return out
