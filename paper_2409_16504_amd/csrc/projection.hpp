// Shared FP32 projection geometry (Section 3.1, Eq. 3-4) for the forward projection and its
// adjoint. Each statement is one correctly rounded FP32 operation evaluated left to right; the
// library is built without multiply-add contraction, so the forward values are a fixed sequence.
#pragma once

#include "pcs_internal.hpp"

namespace pcs {

struct ProjGeo {
  float qw, qx, qy, qz;   // unit quaternion
  float qlen;             // norm of the input quaternion (0: identity was used)
  float R[9];             // rotation, row-major; columns are the ellipsoid axes
  float v[3];             // squared scales
  float S[9];             // Sigma = R diag(v) R^T
  float xc, yc, zc;       // camera-space mean (Eq. 3)
  float fxx, fyy;         // fx * xc, fy * yc
  float j00, j02, j11, j12;  // Jacobian of the perspective map (Eq. 4)
  float M[6];             // J T
  float a, b, c;          // Sigma_s = M Sigma M^T + lowpass I
  float det;
  float u, v2;            // pixel position of the mean
};

// Returns false when the quaternion norm is not finite; other checks are the caller's.
__device__ __forceinline__ bool proj_geometry(float px, float py, float pz, float qw, float qx,
                                              float qy, float qz, float s0, float s1, float s2,
                                              const DevCamera& cam, float lowpass, ProjGeo& G) {
  float nq = qw * qw + qx * qx;
  nq = nq + qy * qy;
  nq = nq + qz * qz;
  const bool ok = isfinite(nq);
  if (nq == 0.0f) {
    G.qlen = 0.0f;
    qw = 1.0f; qx = 0.0f; qy = 0.0f; qz = 0.0f;
  } else {
    const float len = sqrtf(nq);
    G.qlen = len;
    qw = qw / len; qx = qx / len; qy = qy / len; qz = qz / len;
  }
  G.qw = qw; G.qx = qx; G.qy = qy; G.qz = qz;
  const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
  const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
  const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
  float* R = G.R;
  R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - wz);        R[2] = 2.0f * (xz + wy);
  R[3] = 2.0f * (xy + wz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - wx);
  R[6] = 2.0f * (xz - wy);        R[7] = 2.0f * (yz + wx);        R[8] = 1.0f - 2.0f * (xx + yy);
  G.v[0] = s0 * s0; G.v[1] = s1 * s1; G.v[2] = s2 * s2;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = j; k < 3; ++k) {
      const float t0 = (R[3 * j + 0] * G.v[0]) * R[3 * k + 0];
      const float t1 = (R[3 * j + 1] * G.v[1]) * R[3 * k + 1];
      const float t2 = (R[3 * j + 2] * G.v[2]) * R[3 * k + 2];
      const float sjk = (t0 + t1) + t2;
      G.S[3 * j + k] = sjk;
      G.S[3 * k + j] = sjk;
    }
  const float* T = cam.T;
  G.xc = ((T[0] * px + T[1] * py) + T[2] * pz) + cam.t[0];
  G.yc = ((T[3] * px + T[4] * py) + T[5] * pz) + cam.t[1];
  G.zc = ((T[6] * px + T[7] * py) + T[8] * pz) + cam.t[2];
  G.fxx = cam.fx * G.xc;
  G.fyy = cam.fy * G.yc;
  G.u = G.fxx / G.zc + cam.cx;
  G.v2 = G.fyy / G.zc + cam.cy;
  const float zz2 = G.zc * G.zc;
  G.j00 = cam.fx / G.zc;
  G.j02 = -(G.fxx / zz2);
  G.j11 = cam.fy / G.zc;
  G.j12 = -(G.fyy / zz2);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    G.M[k] = G.j00 * T[k] + G.j02 * T[6 + k];
    G.M[3 + k] = G.j11 * T[3 + k] + G.j12 * T[6 + k];
  }
  float P[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      P[3 * r + k] = (G.M[3 * r + 0] * G.S[0 + k] + G.M[3 * r + 1] * G.S[3 + k]) + G.M[3 * r + 2] * G.S[6 + k];
  G.a = ((P[0] * G.M[0] + P[1] * G.M[1]) + P[2] * G.M[2]) + lowpass;
  G.b = (P[0] * G.M[3] + P[1] * G.M[4]) + P[2] * G.M[5];
  G.c = ((P[3] * G.M[3] + P[4] * G.M[4]) + P[5] * G.M[5]) + lowpass;
  G.det = G.a * G.c - G.b * G.b;
  return ok;
}

// Mahalanobis distance q = A dx^2 + 2 B dx dy + C dy^2 of a pixel offset (dx, dy) under the conic
// (A, B, C); the forward and the adjoint evaluate it with this exact operation sequence so their
// discrete decisions agree.
__device__ __forceinline__ float conic_q(float A, float B, float C, float dx, float dy) {
  const float b2dy = (2.0f * B) * dy;
  const float t = fmaf(A, dx, b2dy);
  const float cdy2 = (C * dy) * dy;
  return fmaf(dx, t, cdy2);
}

}  // namespace pcs
