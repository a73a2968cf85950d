// Test infrastructure only: the plain, slow CPU oracle of the splatting renderer.
//
// Nothing in the product path may call this file. It exists so the tests and the benchmark's CPU
// baseline can check the GPU renderer against an independent implementation written from the
// paper (Section 3.1, Eq. 1-4). It shares no code with the GPU library.
//
// Contents
//   * orc_project_f32 : projection of every (camera, Gaussian) as an exact IEEE-FP32 operation
//                       sequence (round-to-nearest-even, no fused multiply-add, correctly rounded
//                       division and square root). This sequence is the binning contract: the
//                       keys, values and tile ranges derived from it are compared bit-exactly.
//   * orc_project_f64 : the same projection in FP64 (optionally from an explicit covariance).
//   * orc_bin         : (tile | depth) keys and Gaussian-index values, sorted lexicographically.
//   * orc_composite   : per-pixel front-to-back alpha blending in FP64 (Eq. 1-2), with margin
//                       flags for pixels whose discrete decisions lie within rounding of a
//                       threshold.
//   * orc_backward    : the FP64 adjoint of the FP64 render with respect to every Gaussian
//                       parameter, plus the sum of absolute per-pixel terms for each gradient.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared.
// Plain loops throughout; OpenMP only splits independent pixels or Gaussians across threads.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// Option vector layout shared with the Python wrapper.
enum { OPT_ZNEAR = 0, OPT_LOWPASS, OPT_SIGMA_CUT, OPT_ALPHA_MIN, OPT_ALPHA_MAX, OPT_T_EPS,
       OPT_BG0, OPT_BG1, OPT_BG2, OPT_COUNT };
// Camera vector layout: T[9] row-major, t[3], fx, fy, cx, cy.
enum { CAM_T = 0, CAM_t = 9, CAM_FX = 12, CAM_FY, CAM_CX, CAM_CY, CAM_COUNT };

inline bool fin(float v) { return std::isfinite(v); }
inline bool fin(double v) { return std::isfinite(v); }

// Unit quaternion (w,x,y,z) -> rotation matrix, Hamilton convention, row-major.
// Columns of R are the ellipsoid's axes in world coordinates.
template <typename F>
void quat_to_rot(F w, F x, F y, F z, F R[9]) {
  const F one = F(1), two = F(2);
  F xx = x * x, yy = y * y, zz = z * z;
  F xy = x * y, xz = x * z, yz = y * z;
  F wx = w * x, wy = w * y, wz = w * z;
  R[0] = one - two * (yy + zz); R[1] = two * (xy - wz);       R[2] = two * (xz + wy);
  R[3] = two * (xy + wz);       R[4] = one - two * (xx + zz); R[5] = two * (yz - wx);
  R[6] = two * (xz - wy);       R[7] = two * (yz + wx);       R[8] = one - two * (xx + yy);
}

// Sigma = R diag(s^2) R^T in FP64 from a (not necessarily unit) quaternion; q = 0 is identity.
// Returns the norm of q.
double cov_from_quat_scale(const double q_in[4], const double sc[3], double R[9], double S[9]) {
  double nq = q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3];
  double len = std::sqrt(nq);
  double q[4] = {1.0, 0.0, 0.0, 0.0};
  if (nq > 0.0)
    for (int k = 0; k < 4; ++k) q[k] = q_in[k] / len;
  quat_to_rot<double>(q[0], q[1], q[2], q[3], R);
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int m = 0; m < 3; ++m) acc += R[3 * j + m] * sc[m] * sc[m] * R[3 * k + m];
      S[3 * j + k] = acc;
    }
  return len;
}

struct ScreenSplat {
  bool valid;
  double u, v, z;        // pixel centre of the mean and camera-space depth
  double a, b, c;        // screen covariance Sigma_s = [[a,b],[b,c]] including the low-pass
  double A, B, C;        // conic = inverse of Sigma_s
  double ex, ey;         // padded half extents of the sigma_cut ellipse's axis-aligned box
  int x0, x1, y0, y1;    // inclusive tile rectangle
  float zf;              // FP32 depth whose bits order the splats
};

// ---------------------------------------------------------------------------------------------
// FP32-exact projection (the binning contract). Every line is one rounded IEEE-FP32 operation,
// evaluated left to right; the build disables contraction so no step fuses.
// ---------------------------------------------------------------------------------------------
void project_one_f32(int64_t n, int64_t i, const float* mean, const float* quat, const float* scale,
                     const float* opac, const float* rgb, const float* nrm, const float* cam,
                     int W, int H, int tile, const float* opt, ScreenSplat& s, float out[9]) {
  s.valid = false;
  const float px = mean[i], py = mean[n + i], pz = mean[2 * n + i];
  float qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
  const float s0 = scale[i], s1 = scale[n + i], s2 = scale[2 * n + i];
  const float o = opac[i];
  bool ok = fin(px) && fin(py) && fin(pz) && fin(qw) && fin(qx) && fin(qy) && fin(qz) &&
            fin(s0) && fin(s1) && fin(s2) && fin(o);
  for (int k = 0; k < 3; ++k) ok = ok && fin(rgb[k * n + i]) && fin(nrm[k * n + i]);
  if (!ok) return;
  if (!(o >= opt[OPT_ALPHA_MIN])) return;  // alpha <= o can never reach the cutoff
  // (1) normalise q.
  float nq = qw * qw + qx * qx;
  nq = nq + qy * qy;
  nq = nq + qz * qz;
  if (!fin(nq)) return;
  if (nq == 0.0f) { qw = 1.0f; qx = 0.0f; qy = 0.0f; qz = 0.0f; }
  else {
    float len = std::sqrt(nq);
    qw = qw / len; qx = qx / len; qy = qy / len; qz = qz / len;
  }
  // (2) rotation.
  float R[9];
  quat_to_rot<float>(qw, qx, qy, qz, R);
  // (3) Sigma = R diag(s^2) R^T, upper triangle computed, lower mirrored.
  const float v0 = s0 * s0, v1 = s1 * s1, v2 = s2 * s2;
  float S[9];
  for (int j = 0; j < 3; ++j)
    for (int k = j; k < 3; ++k) {
      float t0 = (R[3 * j + 0] * v0) * R[3 * k + 0];
      float t1 = (R[3 * j + 1] * v1) * R[3 * k + 1];
      float t2 = (R[3 * j + 2] * v2) * R[3 * k + 2];
      float sjk = (t0 + t1) + t2;
      S[3 * j + k] = sjk;
      S[3 * k + j] = sjk;
    }
  // (4) view transform x_c = T p + t (Eq. 3).
  const float* T = cam + CAM_T;
  float xc = ((T[0] * px + T[1] * py) + T[2] * pz) + cam[CAM_t + 0];
  float yc = ((T[3] * px + T[4] * py) + T[5] * pz) + cam[CAM_t + 1];
  float zc = ((T[6] * px + T[7] * py) + T[8] * pz) + cam[CAM_t + 2];
  if (!(zc > opt[OPT_ZNEAR]) || !fin(xc) || !fin(yc) || !fin(zc)) return;
  // (5) pixel position of the mean.
  const float fx = cam[CAM_FX], fy = cam[CAM_FY];
  const float fxx = fx * xc, fyy = fy * yc;
  const float u = fxx / zc + cam[CAM_CX];
  const float v = fyy / zc + cam[CAM_CY];
  // (6) Jacobian of the perspective map at x_c (Eq. 4), no frustum clamp.
  const float zz2 = zc * zc;
  const float j00 = fx / zc, j02 = -(fxx / zz2);
  const float j11 = fy / zc, j12 = -(fyy / zz2);
  // (7) M = J T (2x3); the zero entries of J contribute no term.
  float M[6];
  for (int k = 0; k < 3; ++k) {
    M[k] = j00 * T[k] + j02 * T[6 + k];
    M[3 + k] = j11 * T[3 + k] + j12 * T[6 + k];
  }
  // (8) Sigma_s = M Sigma M^T + lowpass I.
  float P[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k)
      P[3 * r + k] = (M[3 * r + 0] * S[0 + k] + M[3 * r + 1] * S[3 + k]) + M[3 * r + 2] * S[6 + k];
  const float lp = opt[OPT_LOWPASS];
  float a = ((P[0] * M[0] + P[1] * M[1]) + P[2] * M[2]) + lp;
  float b = (P[0] * M[3] + P[1] * M[4]) + P[2] * M[5];
  float c = ((P[3] * M[3] + P[4] * M[4]) + P[5] * M[5]) + lp;
  // (9) conic, and the half extents of the axis-aligned box of the sigma_cut ellipse: the
  // ellipse x^T Sigma_s^-1 x <= sigma_cut^2 reaches sigma_cut sqrt(a) in x and sigma_cut sqrt(c)
  // in y; the extents are widened by 0.1 % and 0.01 px so that no pixel whose rounded quadratic
  // form passes the cut lies outside them.
  float det = a * c - b * b;
  if (!(det > 0.0f)) return;
  float A = c / det, Bc = -(b / det), C = a / det;
  const float cut = opt[OPT_SIGMA_CUT];
  float ex = (cut * std::sqrt(a)) * 1.001f + 0.01f;
  float ey = (cut * std::sqrt(c)) * 1.001f + 0.01f;
  if (!fin(u) || !fin(v) || !fin(A) || !fin(Bc) || !fin(C) || !fin(ex) || !fin(ey)) return;
  // (10) tile rectangle of the box [u-ex, u+ex] x [v-ey, v+ey].
  const float ts = (float)tile;
  float fx0 = std::floor((u - ex) / ts), fx1 = std::floor((u + ex) / ts);
  float fy0 = std::floor((v - ey) / ts), fy1 = std::floor((v + ey) / ts);
  const int TX = (W + tile - 1) / tile, TY = (H + tile - 1) / tile;
  if (fx1 < 0.0f || fy1 < 0.0f || fx0 > (float)(TX - 1) || fy0 > (float)(TY - 1)) return;
  s.valid = true;
  s.x0 = (int)std::max(fx0, 0.0f); s.x1 = (int)std::min(fx1, (float)(TX - 1));
  s.y0 = (int)std::max(fy0, 0.0f); s.y1 = (int)std::min(fy1, (float)(TY - 1));
  s.u = u; s.v = v; s.z = zc; s.zf = zc;
  s.a = a; s.b = b; s.c = c; s.A = A; s.B = Bc; s.C = C; s.ex = ex; s.ey = ey;
  out[0] = u; out[1] = v; out[2] = zc; out[3] = A; out[4] = Bc; out[5] = C; out[6] = ex; out[7] = ey;
  out[8] = o;
}

// Camera-space depth of step (4) of the exact FP32 sequence, from FP32 copies of the mean and
// camera: the value whose bits order the splats (reading C-8: the depth order is defined on the
// FP32 depth of the exact projection, the same order the FP32 path uses).
float depth_f32(double px, double py, double pz, const double* cam) {
  const float T6 = (float)cam[CAM_T + 6], T7 = (float)cam[CAM_T + 7], T8 = (float)cam[CAM_T + 8];
  return ((T6 * (float)px + T7 * (float)py) + T8 * (float)pz) + (float)cam[CAM_t + 2];
}

// FP64 projection; if cov6 is non-null, Sigma is taken from it (xx,xy,xz,yy,yz,zz planar).
void project_one_f64(int64_t n, int64_t i, const float* mean, const double* mean_d, const float* quat,
                     const double* quat_d, const float* scale, const double* scale_d,
                     const double* cov6, const float* opac, const double* opac_d,
                     const double* cam, int W, int H, int tile, const float* opt, ScreenSplat& s) {
  s.valid = false;
  double px = mean_d ? mean_d[i] : mean[i], py = mean_d ? mean_d[n + i] : mean[n + i],
         pz = mean_d ? mean_d[2 * n + i] : mean[2 * n + i];
  double o = opac_d ? opac_d[i] : opac[i];
  if (!fin(px) || !fin(py) || !fin(pz) || !fin(o)) return;
  if (!(o >= (double)opt[OPT_ALPHA_MIN])) return;
  double S[9];
  if (cov6) {
    double xx = cov6[i], xy = cov6[n + i], xz = cov6[2 * n + i], yy = cov6[3 * n + i],
           yz = cov6[4 * n + i], zz = cov6[5 * n + i];
    S[0] = xx; S[1] = xy; S[2] = xz; S[3] = xy; S[4] = yy; S[5] = yz; S[6] = xz; S[7] = yz; S[8] = zz;
  } else {
    double q[4], sc[3], R[9];
    for (int k = 0; k < 4; ++k) q[k] = quat_d ? quat_d[k * n + i] : quat[k * n + i];
    for (int k = 0; k < 3; ++k) sc[k] = scale_d ? scale_d[k * n + i] : scale[k * n + i];
    if (!fin(cov_from_quat_scale(q, sc, R, S))) return;
  }
  const double* T = cam + CAM_T;
  double xc = T[0] * px + T[1] * py + T[2] * pz + cam[CAM_t + 0];
  double yc = T[3] * px + T[4] * py + T[5] * pz + cam[CAM_t + 1];
  double zc = T[6] * px + T[7] * py + T[8] * pz + cam[CAM_t + 2];
  if (!(zc > (double)opt[OPT_ZNEAR])) return;
  double fx = cam[CAM_FX], fy = cam[CAM_FY];
  double u = fx * xc / zc + cam[CAM_CX], v = fy * yc / zc + cam[CAM_CY];
  double J[6] = {fx / zc, 0.0, -fx * xc / (zc * zc), 0.0, fy / zc, -fy * yc / (zc * zc)};
  double M[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int m = 0; m < 3; ++m) acc += J[3 * r + m] * T[3 * m + k];
      M[3 * r + k] = acc;
    }
  double Ss[4];
  for (int r = 0; r < 2; ++r)
    for (int cidx = 0; cidx < 2; ++cidx) {
      double acc = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) acc += M[3 * r + j] * S[3 * j + k] * M[3 * cidx + k];
      Ss[2 * r + cidx] = acc;
    }
  double lp = opt[OPT_LOWPASS];
  double a = Ss[0] + lp, b = 0.5 * (Ss[1] + Ss[2]), c = Ss[3] + lp;
  double det = a * c - b * b;
  if (!(det > 0.0)) return;
  // half extents of the sigma_cut ellipse's axis-aligned box, widened as in the FP32 sequence
  const double cut = opt[OPT_SIGMA_CUT];
  double ex = cut * std::sqrt(a) * 1.001 + 0.01, ey = cut * std::sqrt(c) * 1.001 + 0.01;
  if (!fin(u) || !fin(v) || !fin(ex) || !fin(ey)) return;
  const int TX = (W + tile - 1) / tile, TY = (H + tile - 1) / tile;
  double fx0 = std::floor((u - ex) / tile), fx1 = std::floor((u + ex) / tile);
  double fy0 = std::floor((v - ey) / tile), fy1 = std::floor((v + ey) / tile);
  if (fx1 < 0 || fy1 < 0 || fx0 > TX - 1 || fy0 > TY - 1) return;
  s.valid = true;
  s.x0 = (int)std::max(fx0, 0.0); s.x1 = (int)std::min(fx1, (double)(TX - 1));
  s.y0 = (int)std::max(fy0, 0.0); s.y1 = (int)std::min(fy1, (double)(TY - 1));
  s.u = u; s.v = v; s.z = zc; s.zf = depth_f32(px, py, pz, cam);
  s.a = a; s.b = b; s.c = c;
  s.A = c / det; s.B = -b / det; s.C = a / det; s.ex = ex; s.ey = ey;
}

inline uint32_t f32_bits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

}  // namespace

extern "C" {

// Projection of n Gaussians through one camera as the exact FP32 sequence.
// Outputs (n each): valid, u, v, z, A, B, C, ext[2][n] (ex, ey), rect[4][n] (x0,x1,y0,y1), count.
void orc_project_f32(int64_t n, const float* mean, const float* quat, const float* scale,
                     const float* opac, const float* rgb, const float* nrm, const float* cam,
                     int W, int H, int tile, const float* opt, uint8_t* valid, float* u, float* v,
                     float* z, float* A, float* B, float* C, float* ext, int32_t* rect,
                     uint32_t* count) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    ScreenSplat s;
    float o9[9];
    project_one_f32(n, i, mean, quat, scale, opac, rgb, nrm, cam, W, H, tile, opt, s, o9);
    valid[i] = s.valid ? 1 : 0;
    if (s.valid) {
      u[i] = o9[0]; v[i] = o9[1]; z[i] = o9[2]; A[i] = o9[3]; B[i] = o9[4]; C[i] = o9[5];
      ext[i] = o9[6]; ext[n + i] = o9[7];
      rect[i] = s.x0; rect[n + i] = s.x1; rect[2 * n + i] = s.y0; rect[3 * n + i] = s.y1;
      count[i] = (uint32_t)((s.x1 - s.x0 + 1) * (s.y1 - s.y0 + 1));
    } else {
      u[i] = v[i] = z[i] = A[i] = B[i] = C[i] = ext[i] = ext[n + i] = 0.0f;
      rect[i] = rect[n + i] = rect[2 * n + i] = rect[3 * n + i] = 0;
      count[i] = 0;
    }
  }
}

// FP64 projection; same outputs in double (rect and count as above). quat/scale or cov6.
void orc_project_f64(int64_t n, const double* mean, const double* quat, const double* scale,
                     const double* cov6, const double* opac, const double* cam, int W, int H,
                     int tile, const float* opt, uint8_t* valid, double* u, double* v, double* z,
                     double* A, double* B, double* C, double* ext, int32_t* rect,
                     uint32_t* count, double* cov2d /*[3][n]: a, b, c of Sigma_s*/,
                     float* zf /*[n]: the FP32 depth that orders the splats*/) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    ScreenSplat s;
    project_one_f64(n, i, nullptr, mean, nullptr, quat, nullptr, scale, cov6, nullptr, opac, cam,
                    W, H, tile, opt, s);
    valid[i] = s.valid ? 1 : 0;
    if (s.valid) {
      u[i] = s.u; v[i] = s.v; z[i] = s.z; A[i] = s.A; B[i] = s.B; C[i] = s.C;
      ext[i] = s.ex; ext[n + i] = s.ey;
      cov2d[i] = s.a; cov2d[n + i] = s.b; cov2d[2 * n + i] = s.c;
      zf[i] = s.zf;
      rect[i] = s.x0; rect[n + i] = s.x1; rect[2 * n + i] = s.y0; rect[3 * n + i] = s.y1;
      count[i] = (uint32_t)((s.x1 - s.x0 + 1) * (s.y1 - s.y0 + 1));
    } else {
      u[i] = v[i] = z[i] = A[i] = B[i] = C[i] = ext[i] = ext[n + i] = 0.0;
      cov2d[i] = cov2d[n + i] = cov2d[2 * n + i] = 0.0;
      zf[i] = 0.0f;
      rect[i] = rect[n + i] = rect[2 * n + i] = rect[3 * n + i] = 0;
      count[i] = 0;
    }
  }
}

// Sigma (planar [9][n], row-major 3x3) of n Gaussians in FP64, the covariance every FP64 path uses.
void orc_cov3d_f64(int64_t n, const double* quat, const double* scale, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    double q[4], sc[3], R[9], S[9];
    for (int k = 0; k < 4; ++k) q[k] = quat[k * n + i];
    for (int k = 0; k < 3; ++k) sc[k] = scale[k * n + i];
    cov_from_quat_scale(q, sc, R, S);
    for (int k = 0; k < 9; ++k) out[k * n + i] = S[k];
  }
}

// Keys ((cam*ntiles + ty*TX + tx) << 32) | bits(fl32 z) and values (Gaussian index) of every
// (camera, Gaussian, covered tile), sorted lexicographically by (key, value).
// Per camera c the inputs are at offset c*n: valid, zf (float), rect[4][n] (planar per camera).
// Returns M; keys/vals must hold at least sum(count).
int64_t orc_bin(int64_t n, int n_cams, int ntiles, int TX, const uint8_t* valid, const float* zf,
                const int32_t* rect, uint64_t* keys, uint32_t* vals) {
  std::vector<std::pair<uint64_t, uint32_t>> list;
  for (int c = 0; c < n_cams; ++c) {
    const uint8_t* vc = valid + (int64_t)c * n;
    const float* zc = zf + (int64_t)c * n;
    const int32_t* rc = rect + (int64_t)c * 4 * n;
    for (int64_t i = 0; i < n; ++i) {
      if (!vc[i]) continue;
      uint64_t zb = f32_bits(zc[i]);
      for (int ty = rc[2 * n + i]; ty <= rc[3 * n + i]; ++ty)
        for (int tx = rc[i]; tx <= rc[n + i]; ++tx) {
          uint64_t tile_id = (uint64_t)c * (uint64_t)ntiles + (uint64_t)(ty * TX + tx);
          list.emplace_back((tile_id << 32) | zb, (uint32_t)i);
        }
    }
  }
  std::sort(list.begin(), list.end());
  for (size_t k = 0; k < list.size(); ++k) { keys[k] = list[k].first; vals[k] = list[k].second; }
  return (int64_t)list.size();
}

// Front-to-back compositing of one camera in FP64 (Eq. 1 and 2).
// Splat arrays have n entries, all FP64: u, v, A, B, C, z, opacity, rgb[3][n], normal[3][n].
// keys/vals: this camera's sorted list (its tile ids relative to the camera: tile = key>>32 minus
// cam_tile_base). pix: optional list of pixel indices (y*W+x) to evaluate (npix entries), else all.
// Outputs are written at the pixel index (planar [3][H*W] for rgb and normal).
// flags bits: 1 = a 3-sigma test, 2 = an alpha-cutoff test, 4 = the transmittance stop lies within
// the rounding margin of its threshold. alt (optional, 5 arrays of n: u, v, A, B, C of another
// projection of the same splats, e.g. the FP64 one beside the exact FP32 one) widens every margin
// by the difference between the two projections' quadratic forms, so that a pixel where the two
// projections could take a decision differently is flagged. Returns the number of
// (pixel, list entry) visits.
int64_t orc_composite(int64_t n, const double* u, const double* v, const double* A,
                      const double* B, const double* C, const double* zdepth, const double* opac,
                      const double* rgb, const double* nrm, int64_t m, const uint64_t* keys,
                      const uint32_t* vals, uint64_t cam_tile_base, int W, int H, int tile,
                      const float* opt, const int64_t* pix, int64_t npix, double* out_rgb,
                      double* out_nrm, double* out_depth, double* out_alpha, double* out_T,
                      int32_t* out_ncontrib, uint8_t* out_flags, int64_t* out_blends,
                      const double* alt) {
  const int TX = (W + tile - 1) / tile, TY = (H + tile - 1) / tile;
  const int64_t ntiles = (int64_t)TX * TY;
  std::vector<int64_t> start(ntiles, 0), end(ntiles, 0);
  for (int64_t k = 0; k < m; ++k) {
    int64_t t = (int64_t)((keys[k] >> 32) - cam_tile_base);
    if (t < 0 || t >= ntiles) continue;
    if (k == 0 || (keys[k - 1] >> 32) != (keys[k] >> 32)) start[t] = k;
    if (k == m - 1 || (keys[k + 1] >> 32) != (keys[k] >> 32)) end[t] = k + 1;
  }
  const double cut2 = (double)opt[OPT_SIGMA_CUT] * (double)opt[OPT_SIGMA_CUT];
  const double amin = opt[OPT_ALPHA_MIN], amax = opt[OPT_ALPHA_MAX], teps = opt[OPT_T_EPS];
  const double bg[3] = {opt[OPT_BG0], opt[OPT_BG1], opt[OPT_BG2]};
  const double eps = 1e-5;  // relative rounding margin of a decision
  const int64_t npx = pix ? npix : (int64_t)W * H;
  const int64_t HW = (int64_t)W * H;
  int64_t visits = 0, blends = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : visits, blends)
  for (int64_t p = 0; p < npx; ++p) {
    const int64_t pid = pix ? pix[p] : p;
    const int x = (int)(pid % W), y = (int)(pid / W);
    const int64_t t = (int64_t)(y / tile) * TX + (x / tile);
    const double pxc = x + 0.5, pyc = y + 0.5;
    double T = 1.0, acc[7] = {0, 0, 0, 0, 0, 0, 0};
    double relT = 0.0;     // relative uncertainty of T under FP32 evaluation
    uint8_t flag = 0;
    int32_t ncontrib = 0;
    for (int64_t k = start[t]; k < end[t]; ++k) {
      ++visits;
      const uint32_t g = vals[k];
      const double dx = pxc - u[g], dy = pyc - v[g];
      const double qa = A[g] * dx * dx, qb = 2.0 * B[g] * dx * dy, qc = C[g] * dy * dy;
      const double q = qa + qb + qc;
      double dq = eps * (std::fabs(qa) + std::fabs(qb) + std::fabs(qc));
      if (alt) {
        const double dx2 = pxc - alt[g], dy2 = pyc - alt[n + g];
        const double q2 = alt[2 * n + g] * dx2 * dx2 + 2.0 * alt[3 * n + g] * dx2 * dy2 +
                          alt[4 * n + g] * dy2 * dy2;
        dq += std::fabs(q - q2);
      }
      if (std::fabs(q - cut2) <= dq) flag |= 1;
      if (!(q <= cut2)) continue;
      const double e = std::exp(-0.5 * q);
      const double araw = (double)opac[g] * e;
      const double alpha = std::min(amax, araw);
      const double da = alpha * (0.5 * dq + eps);
      if (std::fabs(alpha - amin) <= da) flag |= 2;
      if (alpha < amin) continue;
      const double w = alpha * T;
      for (int ch = 0; ch < 3; ++ch) acc[ch] += w * (double)rgb[(int64_t)ch * n + g];
      for (int ch = 0; ch < 3; ++ch) acc[3 + ch] += w * (double)nrm[(int64_t)ch * n + g];
      acc[6] += w * zdepth[g];
      T = T * (1.0 - alpha);
      ++blends;
      relT += da / (1.0 - alpha) + eps * 1e-2;
      ncontrib = (int32_t)(k - start[t] + 1);
      if (std::fabs(T - teps) <= relT * T) flag |= 4;
      if (T < teps) break;
    }
    for (int ch = 0; ch < 3; ++ch) {
      out_rgb[ch * HW + pid] = acc[ch] + T * bg[ch];
      out_nrm[ch * HW + pid] = acc[3 + ch];
    }
    out_depth[pid] = acc[6];
    out_alpha[pid] = 1.0 - T;
    out_T[pid] = T;
    out_ncontrib[pid] = ncontrib;
    out_flags[pid] = flag;
  }
  if (out_blends) *out_blends = blends;
  return visits;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// FP64 adjoint.
// ---------------------------------------------------------------------------------------------
namespace {

// Screen-space parameter gradient of one splat: u, v, A, B, C, opacity, depth feature, rgb[3],
// normal[3].
enum { SG_U = 0, SG_V, SG_A, SG_B, SG_C, SG_O, SG_Z, SG_R, SG_G, SG_BL, SG_NX, SG_NY, SG_NZ, SG_COUNT };
// World-space parameter gradient layout: mean[3], cov6[6], quat[4], scale[3], opacity, rgb[3],
// normal[3].
enum { PG_MEAN = 0, PG_COV = 3, PG_QUAT = 9, PG_SCALE = 13, PG_O = 16, PG_RGB = 17, PG_NRM = 20,
       PG_COUNT = 23 };

struct Geo {               // FP64 projection intermediates of one (camera, Gaussian)
  double q[4], qn, sc[3], R[9], S[9];
  double xc, yc, zc, M[6];
  double a, b, c, det;
  bool from_cov;
};

bool geo_f64(int64_t n, int64_t i, const double* mean, const double* quat, const double* scale,
             const double* cov6, const double* cam, Geo& G) {
  const double* T = cam + CAM_T;
  G.from_cov = cov6 != nullptr;
  if (cov6) {
    double xx = cov6[i], xy = cov6[n + i], xz = cov6[2 * n + i], yy = cov6[3 * n + i],
           yz = cov6[4 * n + i], zz = cov6[5 * n + i];
    double S[9] = {xx, xy, xz, xy, yy, yz, xz, yz, zz};
    std::memcpy(G.S, S, sizeof S);
  } else {
    for (int k = 0; k < 4; ++k) G.q[k] = quat[k * n + i];
    for (int k = 0; k < 3; ++k) G.sc[k] = scale[k * n + i];
    G.qn = cov_from_quat_scale(G.q, G.sc, G.R, G.S);
  }
  double px = mean[i], py = mean[n + i], pz = mean[2 * n + i];
  G.xc = T[0] * px + T[1] * py + T[2] * pz + cam[CAM_t + 0];
  G.yc = T[3] * px + T[4] * py + T[5] * pz + cam[CAM_t + 1];
  G.zc = T[6] * px + T[7] * py + T[8] * pz + cam[CAM_t + 2];
  double fx = cam[CAM_FX], fy = cam[CAM_FY], z = G.zc;
  double J[6] = {fx / z, 0.0, -fx * G.xc / (z * z), 0.0, fy / z, -fy * G.yc / (z * z)};
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int m = 0; m < 3; ++m) acc += J[3 * r + m] * T[3 * m + k];
      G.M[3 * r + k] = acc;
    }
  return true;
}

// Pull a screen-space gradient back to the world-space parameters (adds into pg[PG_COUNT]).
void pull_back(const Geo& G, const double* cam, const double* sg, double* pg, double lowpass) {
  const double* T = cam + CAM_T;
  const double fx = cam[CAM_FX], fy = cam[CAM_FY];
  double Ss[4] = {0, 0, 0, 0};
  for (int r = 0; r < 2; ++r)
    for (int cc = 0; cc < 2; ++cc) {
      double acc = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) acc += G.M[3 * r + j] * G.S[3 * j + k] * G.M[3 * cc + k];
      Ss[2 * r + cc] = acc;
    }
  const double a = Ss[0] + lowpass, b = 0.5 * (Ss[1] + Ss[2]), c = Ss[3] + lowpass;
  const double det = a * c - b * b, d2 = det * det;
  // conic (A,B,C) = (c, -b, a)/det
  const double gA = sg[SG_A], gB = sg[SG_B], gC = sg[SG_C];
  const double ga = gA * (-c * c / d2) + gB * (b * c / d2) + gC * (1.0 / det - a * c / d2);
  const double gb = gA * (2.0 * b * c / d2) + gB * (-1.0 / det - 2.0 * b * b / d2) + gC * (2.0 * a * b / d2);
  const double gc = gA * (1.0 / det - a * c / d2) + gB * (a * b / d2) + gC * (-a * a / d2);
  // symmetric matrix gradient of Sigma_s (b appears twice)
  const double Gs[4] = {ga, 0.5 * gb, 0.5 * gb, gc};
  // dL/dSigma = M^T Gs M ; dL/dM = 2 Gs M Sigma
  double GS[9];
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int r = 0; r < 2; ++r)
        for (int cc = 0; cc < 2; ++cc) acc += G.M[3 * r + j] * Gs[2 * r + cc] * G.M[3 * cc + k];
      GS[3 * j + k] = acc;
    }
  double GM[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int cc = 0; cc < 2; ++cc)
        for (int j = 0; j < 3; ++j) acc += 2.0 * Gs[2 * r + cc] * G.M[3 * cc + j] * G.S[3 * j + k];
      GM[3 * r + k] = acc;
    }
  // dL/dJ = dL/dM T^T
  double GJ[6];
  for (int r = 0; r < 2; ++r)
    for (int m = 0; m < 3; ++m) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += GM[3 * r + k] * T[3 * m + k];
      GJ[3 * r + m] = acc;
    }
  const double x = G.xc, y = G.yc, z = G.zc, z2 = z * z, z3 = z2 * z;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  // J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]
  gx += GJ[2] * (-fx / z2);
  gy += GJ[5] * (-fy / z2);
  gz += GJ[0] * (-fx / z2) + GJ[4] * (-fy / z2) + GJ[2] * (2.0 * fx * x / z3) + GJ[5] * (2.0 * fy * y / z3);
  // u = fx x/z + cx, v = fy y/z + cy
  gx += sg[SG_U] * fx / z;
  gz += sg[SG_U] * (-fx * x / z2);
  gy += sg[SG_V] * fy / z;
  gz += sg[SG_V] * (-fy * y / z2);
  gz += sg[SG_Z];
  for (int k = 0; k < 3; ++k) pg[PG_MEAN + k] += T[0 * 3 + k] * gx + T[1 * 3 + k] * gy + T[2 * 3 + k] * gz;
  // covariance, reported for the six unique entries (xx,xy,xz,yy,yz,zz)
  pg[PG_COV + 0] += GS[0];
  pg[PG_COV + 1] += GS[1] + GS[3];
  pg[PG_COV + 2] += GS[2] + GS[6];
  pg[PG_COV + 3] += GS[4];
  pg[PG_COV + 4] += GS[5] + GS[7];
  pg[PG_COV + 5] += GS[8];
  if (!G.from_cov) {
    // Sigma = R D R^T, D = diag(s^2): dL/ds_i = 2 s_i (R^T GS R)_ii, dL/dR = 2 GS R D
    const double* R = G.R;
    for (int m = 0; m < 3; ++m) {
      double acc = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) acc += R[3 * j + m] * GS[3 * j + k] * R[3 * k + m];
      pg[PG_SCALE + m] += 2.0 * G.sc[m] * acc;
    }
    double GR[9];
    for (int j = 0; j < 3; ++j)
      for (int m = 0; m < 3; ++m) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += GS[3 * j + k] * R[3 * k + m];
        GR[3 * j + m] = 2.0 * acc * G.sc[m] * G.sc[m];
      }
    double qh[4];
    if (G.qn == 0.0) { qh[0] = 1; qh[1] = qh[2] = qh[3] = 0; }
    else for (int k = 0; k < 4; ++k) qh[k] = G.q[k] / G.qn;
    const double w = qh[0], qx = qh[1], qy = qh[2], qz = qh[3];
    double gq[4];
    gq[0] = 2.0 * (-qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7]);
    gq[1] = 2.0 * (qy * GR[1] + qz * GR[2] + qy * GR[3] - 2.0 * qx * GR[4] - w * GR[5] + qz * GR[6] +
                   w * GR[7] - 2.0 * qx * GR[8]);
    gq[2] = 2.0 * (-2.0 * qy * GR[0] + qx * GR[1] + w * GR[2] + qx * GR[3] + qz * GR[5] - w * GR[6] +
                   qz * GR[7] - 2.0 * qy * GR[8]);
    gq[3] = 2.0 * (-2.0 * qz * GR[0] - w * GR[1] + qx * GR[2] + w * GR[3] - 2.0 * qz * GR[4] +
                   qy * GR[5] + qx * GR[6] + qy * GR[7]);
    if (G.qn > 0.0) {
      double dot = 0.0;
      for (int k = 0; k < 4; ++k) dot += qh[k] * gq[k];
      for (int k = 0; k < 4; ++k) pg[PG_QUAT + k] += (gq[k] - qh[k] * dot) / G.qn;
    }
  }
  pg[PG_O] += sg[SG_O];
  for (int k = 0; k < 3; ++k) {
    pg[PG_RGB + k] += sg[SG_R + k];
    pg[PG_NRM + k] += sg[SG_NX + k];
  }
}

}  // namespace

extern "C" {

// Pull-back alone: screen-space gradients sg[SG_COUNT][n] (u, v, A, B, C, opacity, depth, rgb,
// normal of every Gaussian's splat in one camera) to the Gaussian parameters, grad[PG_COUNT][n]
// (overwritten). Gaussians at or behind the near plane get zeros.
void orc_pull_back(int64_t n, const double* mean, const double* quat, const double* scale,
                   const double* cov6, const double* cam, const float* opt, const double* sg,
                   double* grad) {
  std::memset(grad, 0, sizeof(double) * PG_COUNT * n);
  for (int64_t i = 0; i < n; ++i) {
    Geo G;
    geo_f64(n, i, mean, quat, scale, cov6, cam, G);
    if (!(G.zc > (double)opt[OPT_ZNEAR])) continue;
    double s[SG_COUNT], pg[PG_COUNT] = {0};
    for (int k = 0; k < SG_COUNT; ++k) s[k] = sg[(size_t)k * n + i];
    pull_back(G, cam, s, pg, opt[OPT_LOWPASS]);
    for (int k = 0; k < PG_COUNT; ++k) grad[(size_t)k * n + i] = pg[k];
  }
}

// FP64 adjoint of the FP64 render of n_cams cameras. grad images: grad_rgb [C][3][H][W],
// grad_nrm [C][3][H][W], grad_depth [C][H][W] and, if not NULL, grad_alpha [C][H][W] (double; the
// alpha output is 1 - the final transmittance, the covered fraction of the pixel). Outputs: grad[PG_COUNT][n] (planar, see
// layout above) accumulated over cameras, sabs[PG_COUNT][n] the sum over pixels of the absolute
// per-pixel terms (the blend-weight part and the alpha part pulled back apart, the alpha part from
// the absolute terms of dL/dalpha: the size of what an evaluation in lower precision rounds), and sig: a 64-bit signature of the discrete decisions (which splats each
// pixel blends and where it stops), used to detect when a finite-difference step changes them.
// cov6 optional (then the quat and scale gradients are left zero). only_gauss: -1 fills sabs for
// every Gaussian, i >= 0 only for Gaussian i, -2 for none.
void orc_backward(int64_t n, const double* mean, const double* quat, const double* scale,
                  const double* cov6, const double* opac, const double* rgb, const double* nrm,
                  int n_cams, const double* cams /*[C][16]*/, int W, int H, int tile,
                  const float* opt, const double* grad_rgb, const double* grad_nrm,
                  const double* grad_depth, const double* grad_alpha, int64_t only_gauss,
                  double* grad, double* sabs, uint64_t* sig) {
  const int TX = (W + tile - 1) / tile, TY = (H + tile - 1) / tile;
  const int64_t ntiles = (int64_t)TX * TY, HW = (int64_t)W * H;
  const double cut2 = (double)opt[OPT_SIGMA_CUT] * (double)opt[OPT_SIGMA_CUT];
  const double amin = opt[OPT_ALPHA_MIN], amax = opt[OPT_ALPHA_MAX], teps = opt[OPT_T_EPS];
  const double bg[3] = {opt[OPT_BG0], opt[OPT_BG1], opt[OPT_BG2]};
  std::memset(grad, 0, sizeof(double) * PG_COUNT * n);
  std::memset(sabs, 0, sizeof(double) * PG_COUNT * n);
  uint64_t signature = 1469598103934665603ull;
  for (int cam_i = 0; cam_i < n_cams; ++cam_i) {
    const double* cam = cams + 16 * cam_i;
    std::vector<ScreenSplat> sp(n);
    for (int64_t i = 0; i < n; ++i)
      project_one_f64(n, i, nullptr, mean, nullptr, quat, nullptr, scale, cov6, nullptr, opac, cam,
                      W, H, tile, opt, sp[i]);
    std::vector<std::pair<uint64_t, uint32_t>> list;
    for (int64_t i = 0; i < n; ++i) {
      if (!sp[i].valid) continue;
      for (int ty = sp[i].y0; ty <= sp[i].y1; ++ty)
        for (int tx = sp[i].x0; tx <= sp[i].x1; ++tx)
          list.emplace_back(((uint64_t)(ty * TX + tx) << 32) | f32_bits(sp[i].zf), (uint32_t)i);
    }
    std::sort(list.begin(), list.end());
    std::vector<int64_t> start(ntiles, 0), end(ntiles, 0);
    for (size_t k = 0; k < list.size(); ++k) {
      int64_t t = (int64_t)(list[k].first >> 32);
      if (k == 0 || (list[k - 1].first >> 32) != (list[k].first >> 32)) start[t] = k;
      if (k + 1 == list.size() || (list[k + 1].first >> 32) != (list[k].first >> 32)) end[t] = k + 1;
    }
    std::vector<Geo> geo(n);
    for (int64_t i = 0; i < n; ++i)
      if (sp[i].valid) geo_f64(n, i, mean, quat, scale, cov6, cam, geo[i]);
    std::vector<double> sgrad((size_t)SG_COUNT * n, 0.0);
    // per pixel: forward to find the contributing splats, then the reverse pass
    for (int64_t pid = 0; pid < HW; ++pid) {
      const int x = (int)(pid % W), y = (int)(pid / W);
      const int64_t t = (int64_t)(y / tile) * TX + (x / tile);
      const double pxc = x + 0.5, pyc = y + 0.5;
      struct Hit { uint32_t g; double alpha, e, T, dx, dy; bool clamped; };
      std::vector<Hit> hits;
      double T = 1.0;
      int64_t stop = end[t];
      for (int64_t k = start[t]; k < end[t]; ++k) {
        const uint32_t g = list[k].second;
        const ScreenSplat& s = sp[g];
        const double dx = pxc - s.u, dy = pyc - s.v;
        const double q = s.A * dx * dx + 2.0 * s.B * dx * dy + s.C * dy * dy;
        if (!(q <= cut2)) continue;
        const double e = std::exp(-0.5 * q);
        const double araw = opac[g] * e;
        const bool clamped = araw > amax;
        const double alpha = clamped ? amax : araw;
        if (alpha < amin) continue;
        hits.push_back({g, alpha, e, T, dx, dy, clamped});
        signature = (signature ^ (uint64_t)((pid * 1000003 + k) * 2 + (clamped ? 1 : 0))) * 1099511628211ull;
        T = T * (1.0 - alpha);
        if (T < teps) { stop = k + 1; break; }
      }
      signature = (signature ^ (uint64_t)(stop + 7919 * pid)) * 1099511628211ull;
      double gch[7];
      for (int ch = 0; ch < 3; ++ch) {
        gch[ch] = grad_rgb[((int64_t)cam_i * 3 + ch) * HW + pid];
        gch[3 + ch] = grad_nrm[((int64_t)cam_i * 3 + ch) * HW + pid];
      }
      gch[6] = grad_depth[(int64_t)cam_i * HW + pid];
      const double g_cover = grad_alpha ? grad_alpha[(int64_t)cam_i * HW + pid] : 0.0;
      double behind[7] = {T * bg[0], T * bg[1], T * bg[2], 0, 0, 0, 0};
      // the same sums over absolute values, for the size of the terms that cancel in dL/dalpha
      double behind_abs[7] = {T * std::fabs(bg[0]), T * std::fabs(bg[1]), T * std::fabs(bg[2]), 0, 0, 0, 0};
      for (int64_t h = (int64_t)hits.size() - 1; h >= 0; --h) {
        const Hit& hit = hits[h];
        const uint32_t g = hit.g;
        const ScreenSplat& s = sp[g];
        double f[7] = {rgb[g], rgb[n + g], rgb[2 * n + g], nrm[g], nrm[n + g], nrm[2 * n + g], s.z};
        double px_sg[SG_COUNT] = {0};
        const double wgt = hit.T * hit.alpha;
        double dL_dalpha = 0.0, dL_dalpha_terms = 0.0;
        for (int ch = 0; ch < 7; ++ch) {
          dL_dalpha += gch[ch] * (hit.T * f[ch] - behind[ch] / (1.0 - hit.alpha));
          dL_dalpha_terms += std::fabs(gch[ch]) * (hit.T * std::fabs(f[ch]) + behind_abs[ch] / (1.0 - hit.alpha));
          behind[ch] += wgt * f[ch];
          behind_abs[ch] += wgt * std::fabs(f[ch]);
        }
        // alpha output 1 - prod_j (1 - alpha_j): its derivative in alpha_h is T_final / (1 - alpha_h)
        dL_dalpha += g_cover * T / (1.0 - hit.alpha);
        dL_dalpha_terms += std::fabs(g_cover) * T / (1.0 - hit.alpha);
        for (int ch = 0; ch < 3; ++ch) {
          px_sg[SG_R + ch] = gch[ch] * wgt;
          px_sg[SG_NX + ch] = gch[3 + ch] * wgt;
        }
        px_sg[SG_Z] = gch[6] * wgt;
        if (!hit.clamped) {
          px_sg[SG_O] = dL_dalpha * hit.e;
          const double dL_dq = dL_dalpha * (-0.5 * hit.alpha);
          px_sg[SG_A] = dL_dq * hit.dx * hit.dx;
          px_sg[SG_B] = dL_dq * 2.0 * hit.dx * hit.dy;
          px_sg[SG_C] = dL_dq * hit.dy * hit.dy;
          px_sg[SG_U] = dL_dq * (-2.0 * (s.A * hit.dx + s.B * hit.dy));
          px_sg[SG_V] = dL_dq * (-2.0 * (s.B * hit.dx + s.C * hit.dy));
        }
        for (int k = 0; k < SG_COUNT; ++k) sgrad[(size_t)k * n + g] += px_sg[k];
        if (only_gauss == -1 || (int64_t)g == only_gauss) {
          // size of this pixel's terms: the blend-weight part as it is, and the alpha part with
          // dL/dalpha replaced by the sum of the absolute values of its terms (front colour
          // against the part behind, which cancel where the splat hardly changes the pixel)
          double sg_w[SG_COUNT] = {0}, sg_a[SG_COUNT] = {0};
          for (int k = SG_Z; k < SG_COUNT; ++k) sg_w[k] = px_sg[k];
          if (!hit.clamped) {
            const double dq = dL_dalpha_terms * (-0.5 * hit.alpha);
            sg_a[SG_O] = dL_dalpha_terms * hit.e;
            sg_a[SG_A] = dq * hit.dx * hit.dx;
            sg_a[SG_B] = dq * 2.0 * hit.dx * hit.dy;
            sg_a[SG_C] = dq * hit.dy * hit.dy;
            sg_a[SG_U] = dq * (-2.0 * (s.A * hit.dx + s.B * hit.dy));
            sg_a[SG_V] = dq * (-2.0 * (s.B * hit.dx + s.C * hit.dy));
          }
          double pw[PG_COUNT] = {0}, pa[PG_COUNT] = {0};
          pull_back(geo[g], cam, sg_w, pw, opt[OPT_LOWPASS]);
          pull_back(geo[g], cam, sg_a, pa, opt[OPT_LOWPASS]);
          for (int k = 0; k < PG_COUNT; ++k) sabs[(size_t)k * n + g] += std::fabs(pw[k]) + std::fabs(pa[k]);
        }
      }
    }
    for (int64_t i = 0; i < n; ++i) {
      if (!sp[i].valid) continue;
      double sg[SG_COUNT], pg[PG_COUNT] = {0};
      for (int k = 0; k < SG_COUNT; ++k) sg[k] = sgrad[(size_t)k * n + i];
      pull_back(geo[i], cam, sg, pg, opt[OPT_LOWPASS]);
      for (int k = 0; k < PG_COUNT; ++k) grad[(size_t)k * n + i] += pg[k];
    }
  }
  *sig = signature;
}

}  // extern "C"
