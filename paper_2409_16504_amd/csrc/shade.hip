// Late shading of a rendered frame (Section 3.1: the blended normal map shaded by a pixel
// shader). Blinn-Phong with one directional light: the rendered colour is the premultiplied
// albedo of the covered fraction alpha, the normal map is normalised per pixel, the view
// direction is the pixel's ray back to the camera. One thread per pixel; HBM-bound (28 bytes read,
// 12 written per pixel).

#include "pcs_internal.hpp"

namespace pcs {

namespace {

__global__ __launch_bounds__(256) void k_shade(int W, int H, const DevCamera* __restrict__ cams,
                                               const float* __restrict__ rgb,
                                               const float* __restrict__ nrm,
                                               const float* __restrict__ alpha, DevLight L,
                                               float* __restrict__ out) {
  const int64_t HW = (int64_t)W * H;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (p >= HW) return;
  const int x = (int)(p % W), y = (int)(p / W);
  const DevCamera& cam = cams[c];
  const int64_t c3 = (int64_t)c * 3 * HW;
  const float a = alpha[(int64_t)c * HW + p];
  const float T = 1.0f - a;
  const float f0 = rgb[c3 + p] - T * L.bg[0], f1 = rgb[c3 + HW + p] - T * L.bg[1],
              f2 = rgb[c3 + 2 * HW + p] - T * L.bg[2];
  float nx = nrm[c3 + p], ny = nrm[c3 + HW + p], nz = nrm[c3 + 2 * HW + p];
  const float nl = sqrtf(nx * nx + ny * ny + nz * nz);
  const bool has = nl > 0.0f;
  const float inv = has ? 1.0f / nl : 0.0f;
  nx *= inv; ny *= inv; nz *= inv;
  // pixel ray in camera coordinates, to world by the transposed rotation, towards the camera
  const float rx = ((float)x + 0.5f - cam.cx) / cam.fx, ry = ((float)y + 0.5f - cam.cy) / cam.fy;
  float vx = -(cam.T[0] * rx + cam.T[3] * ry + cam.T[6]);
  float vy = -(cam.T[1] * rx + cam.T[4] * ry + cam.T[7]);
  float vz = -(cam.T[2] * rx + cam.T[5] * ry + cam.T[8]);
  const float vi = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
  vx *= vi; vy *= vi; vz *= vi;
  float hx = L.dir[0] + vx, hy = L.dir[1] + vy, hz = L.dir[2] + vz;
  const float hl = sqrtf(hx * hx + hy * hy + hz * hz);
  const float hi = hl > 0.0f ? 1.0f / hl : 0.0f;
  hx *= hi; hy *= hi; hz *= hi;
  const float ndl = fmaxf(nx * L.dir[0] + ny * L.dir[1] + nz * L.dir[2], 0.0f);
  const float ndh = fmaxf(nx * hx + ny * hy + nz * hz, 0.0f);
  const float spec = has ? exp2f(L.shininess * log2f(ndh)) : 0.0f;   // ndh^shininess, 0^s = 0
  const float kd = L.ambient + L.diffuse * ndl;
  const float ks = a * L.specular * spec;
  out[c3 + p] = (f0 * kd + ks) * L.color[0] + T * L.bg[0];
  out[c3 + HW + p] = (f1 * kd + ks) * L.color[1] + T * L.bg[1];
  out[c3 + 2 * HW + p] = (f2 * kd + ks) * L.color[2] + T * L.bg[2];
}

}  // namespace

hipError_t launch_shade(int W, int H, int n_cams, const DevCamera* cams, const float* rgb,
                        const float* nrm, const float* alpha, const DevLight& L, float* out,
                        hipStream_t s) {
  const int64_t HW = (int64_t)W * H;
  if (HW == 0 || n_cams == 0) return hipSuccess;
  hipLaunchKernelGGL(k_shade, dim3((unsigned)((HW + 255) / 256), (unsigned)n_cams), dim3(256), 0, s, W, H,
                     cams, rgb, nrm, alpha, L, out);
  return hipGetLastError();
}

}  // namespace pcs
