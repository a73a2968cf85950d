// kNN-PCA surfel ellipsoids: the plain-path estimate of every point's Gaussian.
//
// For each point: its k nearest points (itself included; ties by index), their covariance about
// their mean, the eigen-decomposition of that 3x3 matrix (cyclic Jacobi), scales
// s_i = kappa sqrt(lambda_i) with s_3 >= floor * s_2, the least-variance axis as the normal
// (oriented away from the cloud centroid) and the axes as a rotation quaternion.
//
// Neighbour search uses a dense uniform grid built by counting sort (cell histogram, exclusive
// scan, scatter). Points are processed in cell order so the 64 queries of a wavefront read the
// same cells; each query visits Chebyshev rings of cells around its own cell and stops once the
// k-th best distance is strictly below the distance to the unvisited region, so the result is the
// exact kNN set for any cell size.

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "pcs_internal.hpp"

namespace pcs {

namespace {

struct GridInfo {
  float ox, oy, oz;     // origin (minimum corner)
  float cell;           // cell edge
  float inv_cell;
  int gx, gy, gz;       // cells per axis
  int64_t ncells;
};

__device__ __forceinline__ uint32_t float_to_ordered(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Bounding box (ordered-uint min/max) and coordinate sums (FP64) of the cloud.
__global__ __launch_bounds__(256) void k_bounds(const float* __restrict__ xyz, int64_t n,
                                                uint32_t* __restrict__ box /*[6]*/,
                                                double* __restrict__ sum /*[3]*/) {
  __shared__ uint32_t s_lo[3][4], s_hi[3][4];
  __shared__ double s_sum[3][4];
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float v = xyz[a * n + i];
      const uint32_t o = float_to_ordered(v);
      lo[a] = min(lo[a], o);
      hi[a] = max(hi[a], o);
      acc[a] += (double)v;
    }
  }
  const int lane = lane_id(), wave = threadIdx.x / kWave;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      lo[a] = min(lo[a], (uint32_t)__shfl_xor((int)lo[a], o, kWave));
      hi[a] = max(hi[a], (uint32_t)__shfl_xor((int)hi[a], o, kWave));
      acc[a] += __shfl_xor(acc[a], o, kWave);
    }
    if (lane == 0) { s_lo[a][wave] = lo[a]; s_hi[a][wave] = hi[a]; s_sum[a][wave] = acc[a]; }
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    uint32_t l = s_lo[a][0], h = s_hi[a][0];
    double s = s_sum[a][0];
    for (int w = 1; w < 4; ++w) { l = min(l, s_lo[a][w]); h = max(h, s_hi[a][w]); s += s_sum[a][w]; }
    atomicMin(&box[a], l);
    atomicMax(&box[3 + a], h);
    unsafeAtomicAdd(&sum[a], s);
  }
}

__device__ __forceinline__ void cell_of(const GridInfo& G, float x, float y, float z, int& cx,
                                        int& cy, int& cz) {
  cx = min(max((int)floorf((x - G.ox) * G.inv_cell), 0), G.gx - 1);
  cy = min(max((int)floorf((y - G.oy) * G.inv_cell), 0), G.gy - 1);
  cz = min(max((int)floorf((z - G.oz) * G.inv_cell), 0), G.gz - 1);
}

__global__ __launch_bounds__(256) void k_cell_count(const float* __restrict__ xyz, int64_t n,
                                                    GridInfo G, uint32_t* __restrict__ cell_id,
                                                    uint32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int cx, cy, cz;
  cell_of(G, xyz[i], xyz[n + i], xyz[2 * n + i], cx, cy, cz);
  const uint32_t c = (uint32_t)(((int64_t)cz * G.gy + cy) * G.gx + cx);
  cell_id[i] = c;
  atomicAdd(&counts[c], 1u);
}

__global__ __launch_bounds__(256) void k_cell_scatter(const float* __restrict__ xyz, int64_t n,
                                                      const uint32_t* __restrict__ cell_id,
                                                      const uint32_t* __restrict__ cell_start,
                                                      uint32_t* __restrict__ cursor,
                                                      float4* __restrict__ sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = cell_id[i];
  const uint32_t pos = cell_start[c] + atomicAdd(&cursor[c], 1u);
  sorted[pos] = make_float4(xyz[i], xyz[n + i], xyz[2 * n + i], __uint_as_float((uint32_t)i));
}

// Insert (d, id) into the ascending list (bd, bi) of K entries, dropping the largest.
template <int K>
__device__ __forceinline__ void topk_insert(float (&bd)[K], uint32_t (&bi)[K], float d, uint32_t id) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool less = d < bd[j] || (d == bd[j] && id < bi[j]);
    const float td = less ? bd[j] : d;
    const uint32_t ti = less ? bi[j] : id;
    bd[j] = less ? d : bd[j];
    bi[j] = less ? id : bi[j];
    d = td;
    id = ti;
  }
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix: A (6 unique: 00,01,02,11,12,22)
// -> eigenvalues w[3], eigenvectors as columns of V (row-major).
__device__ __forceinline__ void jacobi3(float a00, float a01, float a02, float a11, float a12,
                                        float a22, float w[3], float V[9]) {
  float A[3][3] = {{a00, a01, a02}, {a01, a11, a12}, {a02, a12, a22}};
  float v[3][3] = {{1.f, 0.f, 0.f}, {0.f, 1.f, 0.f}, {0.f, 0.f, 1.f}};
  for (int sweep = 0; sweep < 8; ++sweep) {
    const float off = fabsf(A[0][1]) + fabsf(A[0][2]) + fabsf(A[1][2]);
    const float diag = fabsf(A[0][0]) + fabsf(A[1][1]) + fabsf(A[2][2]);
    if (off <= 1e-9f * diag || off == 0.0f) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const float apq = A[p][q];
      if (apq == 0.0f) continue;
      const float theta = (A[q][q] - A[p][p]) / (2.0f * apq);
      const float t = copysignf(1.0f, theta) / (fabsf(theta) + sqrtf(theta * theta + 1.0f));
      const float c = 1.0f / sqrtf(t * t + 1.0f), s = t * c;
      // A <- J^T A J with the rotation in the (p, q) plane
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float vkp = v[k][p], vkq = v[k][q];
        v[k][p] = c * vkp - s * vkq;
        v[k][q] = s * vkp + c * vkq;
      }
    }
  }
  w[0] = A[0][0]; w[1] = A[1][1]; w[2] = A[2][2];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) V[3 * r + c] = v[r][c];
}

template <int K>
__global__ __launch_bounds__(256) void k_knn_pca(const float4* __restrict__ sorted,
                                                 const float* __restrict__ xyz, int64_t n, int k,
                                                 GridInfo G, const uint32_t* __restrict__ cell_start,
                                                 const double* __restrict__ sum, float kappa,
                                                 float floor_ratio, float* __restrict__ quat,
                                                 float* __restrict__ scale,
                                                 float* __restrict__ normal,
                                                 float* __restrict__ nn_dist) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float4 P = sorted[s];
  const uint32_t self = __float_as_uint(P.w);
  float bd[K];
  uint32_t bi[K];
#pragma unroll
  for (int j = 0; j < K; ++j) { bd[j] = FLT_MAX; bi[j] = 0xFFFFFFFFu; }
  float thr = FLT_MAX;            // k-th best (distance, index) so far
  uint32_t thr_i = 0xFFFFFFFFu;
  int cx, cy, cz;
  cell_of(G, P.x, P.y, P.z, cx, cy, cz);
  const int max_ring = max(max(G.gx, G.gy), G.gz);
  for (int r = 0; r <= max_ring; ++r) {
    for (int dz = -r; dz <= r; ++dz) {
      const int z = cz + dz;
      if (z < 0 || z >= G.gz) continue;
      for (int dy = -r; dy <= r; ++dy) {
        const int y = cy + dy;
        if (y < 0 || y >= G.gy) continue;
        // inside the ring's shell only the x = +-r cells are new unless this row is on a face
        const bool face = (dz == -r || dz == r || dy == -r || dy == r);
        const int step = (face || r == 0) ? 1 : 2 * r;
        for (int dx = -r; dx <= r; dx += step) {
          const int x = cx + dx;
          if (x < 0 || x >= G.gx) continue;
          const int64_t c = ((int64_t)z * G.gy + y) * G.gx + x;
          const uint32_t b = cell_start[c], e = cell_start[c + 1];
          for (uint32_t j = b; j < e; ++j) {
            const float4 Q = sorted[j];
            const float ex = Q.x - P.x, ey = Q.y - P.y, ez = Q.z - P.z;
            const float d = ex * ex + ey * ey + ez * ez;
            const uint32_t id = __float_as_uint(Q.w);
            if (d < thr || (d == thr && id < thr_i)) {
              topk_insert<K>(bd, bi, d, id);
              if (k == K) { thr = bd[K - 1]; thr_i = bi[K - 1]; }
              else {
#pragma unroll
                for (int q = 0; q < K; ++q)
                  if (q == k - 1) { thr = bd[q]; thr_i = bi[q]; }
              }
            }
          }
        }
      }
    }
    // every unvisited point lies at least `bnd` away: the distance from P to the boundary of the
    // visited (2r+1)^3 block (cells beyond the grid edge hold no points)
    const bool lo_x = cx - r <= 0, hi_x = cx + r >= G.gx - 1;
    const bool lo_y = cy - r <= 0, hi_y = cy + r >= G.gy - 1;
    const bool lo_z = cz - r <= 0, hi_z = cz + r >= G.gz - 1;
    if (lo_x && hi_x && lo_y && hi_y && lo_z && hi_z) break;        // whole grid visited
    float bnd = FLT_MAX;
    if (!lo_x) bnd = fminf(bnd, P.x - (G.ox + (float)(cx - r) * G.cell));
    if (!hi_x) bnd = fminf(bnd, (G.ox + (float)(cx + r + 1) * G.cell) - P.x);
    if (!lo_y) bnd = fminf(bnd, P.y - (G.oy + (float)(cy - r) * G.cell));
    if (!hi_y) bnd = fminf(bnd, (G.oy + (float)(cy + r + 1) * G.cell) - P.y);
    if (!lo_z) bnd = fminf(bnd, P.z - (G.oz + (float)(cz - r) * G.cell));
    if (!hi_z) bnd = fminf(bnd, (G.oz + (float)(cz + r + 1) * G.cell) - P.z);
    bnd = fmaxf(bnd, 0.0f);
    if (thr < bnd * bnd * (1.0f - 1e-5f)) break;
  }
  if (nn_dist) nn_dist[self] = sqrtf(bd[1]);   // nearest other point (self is one of the first two)
  // neighbourhood mean and covariance (two passes, coordinates relative to P)
  const float inv_k = 1.0f / (float)k;
  float mx = 0.f, my = 0.f, mz = 0.f;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (q < k) {
      const uint32_t id = bi[q];
      mx += xyz[id] - P.x;
      my += xyz[n + id] - P.y;
      mz += xyz[2 * n + id] - P.z;
    }
  }
  mx *= inv_k; my *= inv_k; mz *= inv_k;
  float c00 = 0.f, c01 = 0.f, c02 = 0.f, c11 = 0.f, c12 = 0.f, c22 = 0.f;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (q < k) {
      const uint32_t id = bi[q];
      const float ex = (xyz[id] - P.x) - mx, ey = (xyz[n + id] - P.y) - my, ez = (xyz[2 * n + id] - P.z) - mz;
      c00 += ex * ex; c01 += ex * ey; c02 += ex * ez;
      c11 += ey * ey; c12 += ey * ez; c22 += ez * ez;
    }
  }
  c00 *= inv_k; c01 *= inv_k; c02 *= inv_k; c11 *= inv_k; c12 *= inv_k; c22 *= inv_k;
  float w[3], V[9];
  jacobi3(c00, c01, c02, c11, c12, c22, w, V);
  // order eigenpairs by descending eigenvalue
  int o0 = 0, o1 = 1, o2 = 2;
  if (w[o0] < w[o1]) { int t = o0; o0 = o1; o1 = t; }
  if (w[o1] < w[o2]) { int t = o1; o1 = o2; o2 = t; }
  if (w[o0] < w[o1]) { int t = o0; o0 = o1; o1 = t; }
  const float l0 = fmaxf(w[o0], 0.0f), l1 = fmaxf(w[o1], 0.0f), l2 = fmaxf(w[o2], 0.0f);
  const float s0 = kappa * sqrtf(l0), s1 = kappa * sqrtf(l1);
  const float s2 = fmaxf(kappa * sqrtf(l2), floor_ratio * s1);
  float e1[3] = {V[o0], V[3 + o0], V[6 + o0]};
  float e2[3] = {V[o1], V[3 + o1], V[6 + o1]};
  float nn[3] = {V[o2], V[3 + o2], V[6 + o2]};
  const float inv_n = 1.0f / (float)n;
  const float gx = (float)(sum[0]) * inv_n, gy = (float)(sum[1]) * inv_n, gz = (float)(sum[2]) * inv_n;
  if (nn[0] * (P.x - gx) + nn[1] * (P.y - gy) + nn[2] * (P.z - gz) < 0.0f) {
    nn[0] = -nn[0]; nn[1] = -nn[1]; nn[2] = -nn[2];
  }
  const float det = e1[0] * (e2[1] * nn[2] - e2[2] * nn[1]) - e1[1] * (e2[0] * nn[2] - e2[2] * nn[0]) +
                    e1[2] * (e2[0] * nn[1] - e2[1] * nn[0]);
  if (det < 0.0f) { e2[0] = -e2[0]; e2[1] = -e2[1]; e2[2] = -e2[2]; }
  // rotation with columns (e1, e2, n) -> unit quaternion (Shepperd), w >= 0
  const float R00 = e1[0], R10 = e1[1], R20 = e1[2];
  const float R01 = e2[0], R11 = e2[1], R21 = e2[2];
  const float R02 = nn[0], R12 = nn[1], R22 = nn[2];
  float qw, qx, qy, qz;
  const float tr = R00 + R11 + R22;
  if (tr > 0.0f) {
    const float t = sqrtf(tr + 1.0f) * 2.0f;
    qw = 0.25f * t; qx = (R21 - R12) / t; qy = (R02 - R20) / t; qz = (R10 - R01) / t;
  } else if (R00 > R11 && R00 > R22) {
    const float t = sqrtf(1.0f + R00 - R11 - R22) * 2.0f;
    qw = (R21 - R12) / t; qx = 0.25f * t; qy = (R01 + R10) / t; qz = (R02 + R20) / t;
  } else if (R11 > R22) {
    const float t = sqrtf(1.0f + R11 - R00 - R22) * 2.0f;
    qw = (R02 - R20) / t; qx = (R01 + R10) / t; qy = 0.25f * t; qz = (R12 + R21) / t;
  } else {
    const float t = sqrtf(1.0f + R22 - R00 - R11) * 2.0f;
    qw = (R10 - R01) / t; qx = (R02 + R20) / t; qy = (R12 + R21) / t; qz = 0.25f * t;
  }
  const float ql = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float sg = (qw < 0.0f ? -1.0f : 1.0f) / ql;
  quat[self] = qw * sg;
  quat[n + self] = qx * sg;
  quat[2 * n + self] = qy * sg;
  quat[3 * n + self] = qz * sg;
  scale[self] = s0;
  scale[n + self] = s1;
  scale[2 * n + self] = s2;
  normal[self] = nn[0];
  normal[n + self] = nn[1];
  normal[2 * n + self] = nn[2];
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

constexpr int64_t kMaxCells = int64_t(1) << 24;

}  // namespace

// Scratch layout: [box 6 x u32 | pad | sums 3 x f64 | pad] 128 B, cell_id[n], sorted[n] (float4),
// counts[kMaxCells + 1], cell_start[kMaxCells + 1], scan scratch.
size_t knn_scratch_bytes(int64_t n) {
  return 128 + (size_t)n * 4 + 64 + (size_t)n * 16 + 2 * ((size_t)kMaxCells + 64) * 4 +
         scan_scratch_bytes(kMaxCells + 1) + 256;
}

hipError_t launch_knn_pca(const float* xyz, int64_t n, int k, float kappa, float floor_ratio,
                          float* quat, float* scale, float* normal, float* nn_dist, void* scratch,
                          size_t scratch_bytes, uint32_t* host_pinned, hipStream_t s) {
  if (scratch_bytes < knn_scratch_bytes(n)) return hipErrorInvalidValue;
  char* base = reinterpret_cast<char*>(scratch);
  uint32_t* box = reinterpret_cast<uint32_t*>(base);
  double* sums = reinterpret_cast<double*>(base + 32);
  uint32_t* cell_id = reinterpret_cast<uint32_t*>(base + 128);
  float4* sorted = reinterpret_cast<float4*>(base + 128 + ((n * 4 + 63) / 64) * 64);
  uint32_t* counts = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(sorted) + n * 16);
  uint32_t* cell_start = counts + kMaxCells + 64;
  void* scan_scr = cell_start + kMaxCells + 64;
  hipError_t e = launch_fill_u32(box, 0xFFFFFFFFu, 3, s);
  if (e == hipSuccess) e = launch_fill_u32(box + 3, 0u, 3, s);
  if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(sums), 0u, 6, s);
  if (e != hipSuccess) return e;
  const unsigned bb = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_bounds, dim3(bb), dim3(256), 0, s, xyz, n, box, sums);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(host_pinned, box, 24, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  auto ord = [](uint32_t u) {
    const uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
  };
  const float lo[3] = {ord(host_pinned[0]), ord(host_pinned[1]), ord(host_pinned[2])};
  const float hi[3] = {ord(host_pinned[3]), ord(host_pinned[4]), ord(host_pinned[5])};
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a])) return hipErrorInvalidValue;
  double ext[3], emax = 0.0;
  for (int a = 0; a < 3; ++a) {
    ext[a] = (double)hi[a] - (double)lo[a];
    emax = std::max(emax, ext[a]);
  }
  if (emax <= 0.0) emax = 1.0;
  double vol = 1.0;
  for (int a = 0; a < 3; ++a) vol *= std::max(ext[a], 1e-3 * emax);
  double cell = std::cbrt(vol / (double)n);
  cell = std::max(cell, emax / 1024.0);
  GridInfo G{};
  for (;;) {
    G.gx = (int)std::floor(ext[0] / cell) + 1;
    G.gy = (int)std::floor(ext[1] / cell) + 1;
    G.gz = (int)std::floor(ext[2] / cell) + 1;
    G.ncells = (int64_t)G.gx * G.gy * G.gz;
    if (G.ncells <= kMaxCells) break;
    cell *= 1.25;
  }
  G.ox = lo[0]; G.oy = lo[1]; G.oz = lo[2];
  G.cell = (float)cell;
  G.inv_cell = (float)(1.0 / cell);
  if ((e = launch_fill_u32(counts, 0u, G.ncells + 1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_count, dim3(blocks_for(n, 256)), dim3(256), 0, s, xyz, n, G, cell_id, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint64_t* total = reinterpret_cast<uint64_t*>(base + 64);
  if ((e = launch_scan(counts, nullptr, nullptr, nullptr, cell_start, G.ncells + 1, total, scan_scr, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(counts, 0u, G.ncells + 1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, xyz, n, cell_id,
                     cell_start, counts, sorted);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (k <= 16) {
    hipLaunchKernelGGL(k_knn_pca<16>, dim3(blocks_for(n, 256)), dim3(256), 0, s, sorted, xyz, n, k, G,
                       cell_start, sums, kappa, floor_ratio, quat, scale, normal, nn_dist);
  } else {
    hipLaunchKernelGGL(k_knn_pca<32>, dim3(blocks_for(n, 256)), dim3(256), 0, s, sorted, xyz, n, k, G,
                       cell_start, sums, kappa, floor_ratio, quat, scale, normal, nn_dist);
  }
  return hipGetLastError();
}

}  // namespace pcs
