// Projection of every (camera, Gaussian): EWA screen covariance, conic, 3-sigma extent, tile
// rectangle (Section 3.1, Eq. 3-4), plus the splat record the compositor stages.
//
// The arithmetic up to the tile rectangle is a fixed IEEE-FP32 operation sequence: each line
// below is one correctly rounded operation evaluated left to right, and this file is compiled
// without multiply-add contraction. Binning depends only on these values, so the (tile, depth)
// key lists are reproducible bit for bit by any implementation of the same sequence.
//
// One thread per (camera, Gaussian); the planar inputs make every load a coalesced 4-byte stream.

#include <algorithm>

#include "projection.hpp"

namespace pcs {

namespace {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

__global__ void k_fill_f32(float* __restrict__ p, float value, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

__device__ __forceinline__ bool fin(float x) { return isfinite(x); }

// Frame words written by block (0, 0) of the projection: the error word and the instance total
// reset, and (ARG_CAMS) the cameras of the kernel arguments copied to cams_out for the later kernels.
template <bool ARG_CAMS>
__device__ __forceinline__ void frame_words(const CamBatch& arg_cams, DevCamera* __restrict__ cams_out,
                                            uint32_t* __restrict__ err, uint64_t* __restrict__ total) {
  if (blockIdx.x != 0 || blockIdx.y != 0) return;
  const int t = threadIdx.x;
  if (t == 0 && err) *err = 0u;
  if (t == 0 && total) *total = 0u;
  if constexpr (ARG_CAMS) {
    constexpr int kWords = (int)(sizeof(DevCamera) / 4);
    if (t < (int)gridDim.y * kWords)
      reinterpret_cast<uint32_t*>(cams_out)[t] = reinterpret_cast<const uint32_t*>(arg_cams.c)[t];
  }
}

// ARG_CAMS: the cameras come as kernel arguments (at most kArgCams), else from cams.
template <bool ARG_CAMS>
__global__ __launch_bounds__(256) void k_project(
    int64_t n, DevCamera* __restrict__ cams, DevOptions opt,
    const float* __restrict__ mean, const float* __restrict__ quat,
    const float* __restrict__ scale, const float* __restrict__ opac,
    const float* __restrict__ rgb, const float* __restrict__ nrm, float4* __restrict__ rec,
    uint32_t* __restrict__ zbits_out, uint2* __restrict__ rect, bool narrow_rect,
    uint32_t* __restrict__ zrange,
    unsigned long long* __restrict__ count_slots, ClearSpans clear, CamBatch arg_cams,
    uint32_t* __restrict__ err, uint64_t* __restrict__ total) {
  clear_spans(clear, ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x,
              (int64_t)gridDim.x * gridDim.y * blockDim.x);
  frame_words<ARG_CAMS>(arg_cams, cams, err, total);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  const DevCamera& cam = ARG_CAMS ? arg_cams.c[c] : cams[c];
  const int64_t out = (int64_t)c * n + i;
  bool visible = false;
  uint32_t zbits = 0, my_count = 0;
  if (i < n) {
    const float px = mean[i], py = mean[n + i], pz = mean[2 * n + i];
    const float qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
    const float s0 = scale[i], s1 = scale[n + i], s2 = scale[2 * n + i];
    const float o = opac[i];
    const float cr = rgb[i], cg = rgb[n + i], cb = rgb[2 * n + i];
    const float nx = nrm[i], ny = nrm[n + i], nz = nrm[2 * n + i];
    bool ok = fin(px) && fin(py) && fin(pz) && fin(qw) && fin(qx) && fin(qy) && fin(qz) &&
              fin(s0) && fin(s1) && fin(s2) && fin(o) && fin(cr) && fin(cg) && fin(cb) &&
              fin(nx) && fin(ny) && fin(nz) && (o >= opt.alpha_min);
    ProjGeo G;
    ok = proj_geometry(px, py, pz, qw, qx, qy, qz, s0, s1, s2, cam, opt.lowpass, G) && ok;
    const float zc = G.zc, u = G.u, v = G.v2;
    ok = ok && (zc > opt.z_near) && fin(G.xc) && fin(G.yc) && fin(zc);
    ok = ok && (G.det > 0.0f);
    const float A = G.c / G.det, B = -(G.b / G.det), C = G.a / G.det;
    // half extents of the axis-aligned box of the sigma_cut ellipse (it reaches sigma_cut sqrt(a)
    // in x and sigma_cut sqrt(c) in y), widened so that pixels outside the box fail the
    // sigma_cut test by a wide margin whatever the rounding of the quadratic form; the box bins
    // the splat and culls it in compositing
    const float ex = (opt.sigma_cut * sqrtf(G.a)) * 1.001f + 0.01f;
    const float ey = (opt.sigma_cut * sqrtf(G.c)) * 1.001f + 0.01f;
    ok = ok && fin(u) && fin(v) && fin(A) && fin(B) && fin(C) && fin(ex) && fin(ey);
    // tile rectangle of the box [u - ex, u + ex] x [v - ey, v + ey]
    const int TX = (cam.W + kTile - 1) / kTile, TY = (cam.H + kTile - 1) / kTile;
    const float ts = (float)kTile;
    const float fx0 = floorf((u - ex) / ts), fx1 = floorf((u + ex) / ts);
    const float fy0 = floorf((v - ey) / ts), fy1 = floorf((v + ey) / ts);
    ok = ok && !(fx1 < 0.0f || fy1 < 0.0f || fx0 > (float)(TX - 1) || fy0 > (float)(TY - 1));
    if (ok) {
      const int x0 = (int)fmaxf(fx0, 0.0f), x1 = (int)fminf(fx1, (float)(TX - 1));
      const int y0 = (int)fmaxf(fy0, 0.0f), y1 = (int)fminf(fy1, (float)(TY - 1));
      visible = true;
      zbits = __float_as_uint(zc);
      my_count = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
      zbits_out[out] = zbits;
      store_rect(rect, out, narrow_rect, (uint32_t)x0, (uint32_t)(x1 + 1), (uint32_t)y0,
                 (uint32_t)(y1 + 1));
      float4* r = rec + out * kRecFloat4;
      r[0] = make_float4(u, v, o, zc);
      r[1] = make_float4(A, B, C, ex);
      r[2] = make_float4(cr, cg, cb, ey);
      r[3] = make_float4(nx, ny, nz, 0.0f);
    } else {
      zbits_out[out] = 0u;                 // a visible depth is above z_near > 0: never zero bits
      store_rect(rect, out, narrow_rect, 0u, 0u, 0u, 0u);
    }
  }
  // depth-bit range and instance total of the block: block reduction, then one atomic each into
  // one of kZSlots slots (spreading the atomics; the depth-key pass folds the slots)
  __shared__ uint32_t s_lo[4], s_hi[4];
  __shared__ unsigned long long s_cnt[4];
  uint32_t lo = visible ? zbits : 0xFFFFFFFFu, hi = visible ? zbits : 0u;
  unsigned long long cnt = my_count;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, kWave));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, kWave));
    cnt += __shfl_xor(cnt, o, kWave);
  }
  const int wave = threadIdx.x / kWave;
  if (lane_id() == 0) { s_lo[wave] = lo; s_hi[wave] = hi; s_cnt[wave] = cnt; }
  __syncthreads();
  if (threadIdx.x == 0) {
    lo = min(min(s_lo[0], s_lo[1]), min(s_lo[2], s_lo[3]));
    hi = max(max(s_hi[0], s_hi[1]), max(s_hi[2], s_hi[3]));
    cnt = (s_cnt[0] + s_cnt[1]) + (s_cnt[2] + s_cnt[3]);
    if (hi != 0u) {
      const int slot = (blockIdx.x + blockIdx.y * 7) % kZSlots;
      atomicMin(&zrange[slot], lo);
      atomicMax(&zrange[kZSlots + slot], hi);
      atomicAdd(&count_slots[slot], cnt);
    }
  }
}

// Resets the small words (when small is set) and copies n of the batch's cameras to dst.
__global__ __launch_bounds__(256) void k_init_small(uint32_t* __restrict__ small, CamBatch cams, int n,
                                                    DevCamera* __restrict__ dst, uint32_t* __restrict__ err) {
  const int i = threadIdx.x;
  constexpr int kWords = (int)(sizeof(DevCamera) / 4);
  if (i < n * kWords)
    reinterpret_cast<uint32_t*>(dst)[i] = reinterpret_cast<const uint32_t*>(cams.c)[i];
  if (err && i == 0) *err = 0u;                               // the frame's error word
  if (!small) return;
  if (i < 2) small[i] = 0u;                                   // instance total (u64)
  if (i < kZSlots) {
    small[2 + i] = 0xFFFFFFFFu;                               // depth-bit minima
    small[2 + kZSlots + i] = 0u;                              // depth-bit maxima
  }
  if (i < 2 * kZSlots) small[kCountWord + i] = 0u;           // partial instance counts (u64)
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_init_small(uint32_t* small, const DevCamera* cams, int n_cams, DevCamera* dst,
                             hipStream_t s, uint32_t* err) {
  static_assert(kArgCams * sizeof(DevCamera) / 4 <= 256 && 2 * kZSlots <= 256, "one 256-thread block");
  for (int c0 = 0; c0 == 0 || c0 < n_cams; c0 += kArgCams) {
    CamBatch b{};
    const int nb = std::min(kArgCams, n_cams - c0);
    for (int k = 0; k < nb; ++k) b.c[k] = cams[c0 + k];
    hipLaunchKernelGGL(k_init_small, dim3(1), dim3(256), 0, s, c0 == 0 ? small : nullptr, b,
                       std::max(nb, 0), dst + c0, c0 == 0 ? err : nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_project(int64_t n, int n_cams, DevCamera* cams, const DevOptions& opt,
                          const pcs_gaussians& g, float4* rec, uint32_t* zbits, uint2* rect,
                          bool narrow_rect, uint32_t* zrange, unsigned long long* count_slots,
                          const ClearSpans& clear, hipStream_t s, const CamBatch* arg_cams,
                          uint32_t* err, uint64_t* total) {
  if (n <= 0 || n_cams <= 0) return hipSuccess;
  if (arg_cams && n_cams > kArgCams) return hipErrorInvalidValue;
  static_assert(kArgCams * sizeof(DevCamera) / 4 <= 256, "block (0, 0) copies the cameras");
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_cams);
  const CamBatch none{};
  if (arg_cams)
    hipLaunchKernelGGL(k_project<true>, grid, dim3(256), 0, s, n, cams, opt, g.mean, g.quat, g.scale,
                       g.opacity, g.rgb, g.normal, rec, zbits, rect, narrow_rect, zrange, count_slots,
                       clear, *arg_cams, err, total);
  else
    hipLaunchKernelGGL(k_project<false>, grid, dim3(256), 0, s, n, cams, opt, g.mean, g.quat, g.scale,
                       g.opacity, g.rgb, g.normal, rec, zbits, rect, narrow_rect, zrange, count_slots,
                       clear, none, err, total);
  return hipGetLastError();
}

}  // namespace pcs
