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

// Bounding box (ordered-uint min/max) and coordinate sums (FP64) of the cloud, in two steps
// without atomics: every block writes its partial (lo[3], hi[3], sum[3]), one block combines them.
struct BoundsPart {
  uint32_t lo[3], hi[3];
  double sum[3];
};

__global__ __launch_bounds__(256) void k_bounds(const float* __restrict__ xyz, int64_t n,
                                                BoundsPart* __restrict__ part) {
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
    double sm = s_sum[a][0];
    for (int w = 1; w < 4; ++w) { l = min(l, s_lo[a][w]); h = max(h, s_hi[a][w]); sm += s_sum[a][w]; }
    part[blockIdx.x].lo[a] = l;
    part[blockIdx.x].hi[a] = h;
    part[blockIdx.x].sum[a] = sm;
  }
}

// One block of 256 threads combines the blocks' partials into box[6] and sum[3].
__global__ __launch_bounds__(256) void k_bounds_final(const BoundsPart* __restrict__ part, int parts,
                                                      uint32_t* __restrict__ box, double* __restrict__ sum) {
  __shared__ uint32_t s_lo[3][4], s_hi[3][4];
  __shared__ double s_sum[3][4];
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
  double acc[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < parts; b += blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = min(lo[a], part[b].lo[a]);
      hi[a] = max(hi[a], part[b].hi[a]);
      acc[a] += part[b].sum[a];
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
    double sm = s_sum[a][0];
    for (int w = 1; w < 4; ++w) { l = min(l, s_lo[a][w]); h = max(h, s_hi[a][w]); sm += s_sum[a][w]; }
    box[a] = l;
    box[3 + a] = h;
    sum[a] = sm;
  }
}

constexpr int64_t kMaxCells = int64_t(1) << 24;

// Cubic cells of edge `cell` from the minimum corner (ox, oy, oz) over extents (ex, ey, ez); the
// edge grows by 1.25 until the grid has at most kMaxCells cells.
__host__ __device__ inline GridInfo grid_for(float ox, float oy, float oz, double ex, double ey,
                                             double ez, double cell) {
  GridInfo G{};
  for (;;) {
    G.gx = (int)floor(ex / cell) + 1;
    G.gy = (int)floor(ey / cell) + 1;
    G.gz = (int)floor(ez / cell) + 1;
    G.ncells = (int64_t)G.gx * G.gy * G.gz;
    if (G.ncells <= kMaxCells) break;
    cell *= 1.25;
  }
  G.ox = ox; G.oy = oy; G.oz = oz;
  G.cell = (float)cell;
  G.inv_cell = (float)(1.0 / cell);
  return G;
}

__device__ __forceinline__ void cell_of(const GridInfo& G, float x, float y, float z, int& cx,
                                        int& cy, int& cz) {
  cx = min(max((int)floorf((x - G.ox) * G.inv_cell), 0), G.gx - 1);
  cy = min(max((int)floorf((y - G.oy) * G.inv_cell), 0), G.gy - 1);
  cz = min(max((int)floorf((z - G.oz) * G.inv_cell), 0), G.gz - 1);
}

// Cell of every point and the cells' point counts.
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

// Scatter every point into its cell's slot range; cell_id[i] is replaced by the point's position
// in the cell-sorted array (each thread rewrites only its own entry).
__global__ __launch_bounds__(256) void k_cell_scatter(const float* __restrict__ xyz, int64_t n,
                                                      uint32_t* __restrict__ cell_id,
                                                      const uint32_t* __restrict__ cell_start,
                                                      uint32_t* __restrict__ cursor,
                                                      float4* __restrict__ sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = cell_id[i];
  const uint32_t pos = cell_start[c] + atomicAdd(&cursor[c], 1u);
  sorted[pos] = make_float4(xyz[i], xyz[n + i], xyz[2 * n + i], __uint_as_float((uint32_t)i));
  cell_id[i] = pos;
}

// A candidate is the 64-bit key (squared distance bits << 32 | point index): squared distances are
// non-negative, so unsigned key order is (distance, index) order, the tie rule of the kNN set.
__device__ __forceinline__ uint64_t knn_key(float d, uint32_t id) {
  return ((uint64_t)__float_as_uint(d) << 32) | id;
}

// Insert a key into the ascending list of K keys, dropping the largest.
template <int K>
__device__ __forceinline__ void topk_insert(uint64_t (&bk)[K], uint64_t key) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool less = key < bk[j];
    const uint64_t t = less ? bk[j] : key;
    bk[j] = less ? key : bk[j];
    key = t;
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

// Block search: a query's first candidates are the points of the 3x3x3 cells around its own, read
// as nine runs of the cell-sorted array (the three cells of a row are adjacent in it). Inserting
// every candidate that beats the running k-th best would run the K-step insertion for nearly every
// candidate (some lane of the wavefront always has one to insert), so the block is read twice:
// first into a per-query histogram of squared distance (kHistBins - 1 bins over [0, cell^2), the
// last for the rest; 16-bit counts, two per word), then keeping the positions of the candidates in
// the bins up to the one that holds the k-th smallest, at most kList of them, which alone are
// inserted. A bin index is a monotone function of the squared distance, so every candidate left
// out is strictly farther than every one kept and the kept ones contain the k nearest (ties
// included). When the kept set would not fit (or the block holds 2^16 points or more), every
// candidate of the block is inserted directly.
constexpr int kHistBins = 16;
constexpr int kList = 31;
constexpr int kSearchThreads = 256;

template <int K>
__global__ __launch_bounds__(kSearchThreads) void k_knn_pca(const float4* __restrict__ sorted,
                                                 const uint32_t* __restrict__ pos_of, int64_t n, int k,
                                                 GridInfo G,
                                                 const uint32_t* __restrict__ cell_start,
                                                 const double* __restrict__ sum, float kappa,
                                                 float floor_ratio, float4* __restrict__ stage) {
  // per-lane columns (lane fastest): each query owns column `lane` of its wavefront's arrays
  __shared__ uint32_t s_hist[kSearchThreads / kWave][kHistBins / 2][kWave];
  __shared__ uint32_t s_list[kSearchThreads / kWave][kList + 1][kWave];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  uint32_t* hist = &s_hist[wave][0][lane];
  uint32_t* list = &s_list[wave][0][lane];
  const float4 P = sorted[s];
  uint64_t bk[K];
#pragma unroll
  for (int j = 0; j < K; ++j) bk[j] = ~0ull;
  uint64_t thr = ~0ull;           // k-th best key so far
  // visit the points [b, e) of the cell-sorted array, kBatch loads in flight at a time; positions
  // past e re-read e - 1 and are visited as invalid (no branches: the visitors mask their effect)
  constexpr int kBatch = 8;
  auto walk = [&](uint32_t b, uint32_t e, auto&& visit) {
    for (uint32_t j = b; j < e; j += kBatch) {
      float4 Q[kBatch];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) Q[i] = sorted[min(j + (uint32_t)i, e - 1u)];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) visit(Q[i], j + (uint32_t)i, j + (uint32_t)i < e);
    }
  };
  auto insert = [&](uint64_t key) {
    if (key < thr) {
      topk_insert<K>(bk, key);
      if (k == K) thr = bk[K - 1];
      else {
#pragma unroll
        for (int q = 0; q < K; ++q)
          if (q == k - 1) thr = bk[q];
      }
    }
  };
  int cx, cy, cz;
  cell_of(G, P.x, P.y, P.z, cx, cy, cz);
  // the nine runs of the 3x3x3 block (empty for rows outside the grid)
  uint32_t rb[9], re[9];
  {
    const int x0 = max(cx - 1, 0), x1 = min(cx + 1, G.gx - 1);
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const int z = cz + r / 3 - 1, y = cy + r % 3 - 1;
      const bool ok = z >= 0 && z < G.gz && y >= 0 && y < G.gy;
      const int64_t row = ((int64_t)(ok ? z : cz) * G.gy + (ok ? y : cy)) * G.gx;
      rb[r] = ok ? cell_start[row + x0] : 0u;
      re[r] = ok ? cell_start[row + x1 + 1] : 0u;
    }
  }
  uint32_t total = 0;
#pragma unroll
  for (int r = 0; r < 9; ++r) total += re[r] - rb[r];
  const float hscale = (float)(kHistBins - 1) * (G.inv_cell * G.inv_cell);
  auto bin_of = [&](float d2) { return (uint32_t)fminf(d2 * hscale, (float)(kHistBins - 1)); };
  // the bin that holds the k-th smallest squared distance, and how many lie up to it
  uint32_t last_bin = kHistBins - 1;
  uint32_t kept = total;
  if (total < 65536u) {
#pragma unroll
    for (int b = 0; b < kHistBins / 2; ++b) hist[b * kWave] = 0u;
#pragma unroll
    for (int r = 0; r < 9; ++r)
      walk(rb[r], re[r], [&](float4 Q, uint32_t, bool valid) {
        const float ex = Q.x - P.x, ey = Q.y - P.y, ez = Q.z - P.z;
        const uint32_t b = bin_of(ex * ex + ey * ey + ez * ez);
        atomicAdd(&hist[(b & (kHistBins / 2 - 1)) * kWave], valid ? 1u << ((b & (kHistBins / 2)) << 1) : 0u);
      });
    uint32_t run = 0;
    bool found = false;
#pragma unroll
    for (int b = 0; b < kHistBins; ++b) {
      run += (hist[(b & (kHistBins / 2 - 1)) * kWave] >> ((b & (kHistBins / 2)) << 1)) & 0xFFFFu;
      if (!found && run >= (uint32_t)k) { found = true; last_bin = (uint32_t)b; kept = run; }
    }
  }
  if (kept <= (uint32_t)kList) {
    uint32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r)
      walk(rb[r], re[r], [&](float4 Q, uint32_t j, bool valid) {
        // written at slot cnt always, kept only if it counts (slot kList takes the others)
        const float ex = Q.x - P.x, ey = Q.y - P.y, ez = Q.z - P.z;
        list[cnt * kWave] = j;
        cnt += (valid && bin_of(ex * ex + ey * ey + ez * ez) <= last_bin) ? 1u : 0u;
      });
#pragma unroll 1
    for (uint32_t i = 0; i < cnt; i += kBatch) {
      float4 Q[kBatch];
#pragma unroll
      for (int t = 0; t < kBatch; ++t) Q[t] = sorted[list[min(i + (uint32_t)t, cnt - 1u) * kWave]];
#pragma unroll
      for (int t = 0; t < kBatch; ++t) {
        if (i + (uint32_t)t >= cnt) break;
        const float ex = Q[t].x - P.x, ey = Q[t].y - P.y, ez = Q[t].z - P.z;
        insert(knn_key(ex * ex + ey * ey + ez * ez, __float_as_uint(Q[t].w)));
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < 9; ++r)
      walk(rb[r], re[r], [&](float4 Q, uint32_t, bool valid) {
        const float ex = Q.x - P.x, ey = Q.y - P.y, ez = Q.z - P.z;
        insert(valid ? knn_key(ex * ex + ey * ey + ez * ez, __float_as_uint(Q.w)) : ~0ull);
      });
  }
  // Chebyshev rings r >= 2 (rare): every unvisited point lies at least `bnd` away, the distance
  // from P to the boundary of the visited (2r+1)^3 block (cells beyond the grid edge hold no points)
  const int max_ring = max(max(G.gx, G.gy), G.gz);
  for (int r = 1; r <= max_ring; ++r) {
    if (r >= 2) {
      for (int dz = -r; dz <= r; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= G.gz) continue;
        for (int dy = -r; dy <= r; ++dy) {
          const int y = cy + dy;
          if (y < 0 || y >= G.gy) continue;
          // inside the ring's shell only the x = +-r cells are new unless this row is on a face
          const bool face = (dz == -r || dz == r || dy == -r || dy == r);
          const int step = face ? 1 : 2 * r;
          for (int dx = -r; dx <= r; dx += step) {
            const int x = cx + dx;
            if (x < 0 || x >= G.gx) continue;
            const int64_t c = ((int64_t)z * G.gy + y) * G.gx + x;
            const uint32_t b = cell_start[c], e = cell_start[c + 1];
            for (uint32_t j = b; j < e; ++j) {
              const float4 Q = sorted[j];
              const float ex = Q.x - P.x, ey = Q.y - P.y, ez = Q.z - P.z;
              insert(knn_key(ex * ex + ey * ey + ez * ez, __float_as_uint(Q.w)));
            }
          }
        }
      }
    }
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
    if (__uint_as_float((uint32_t)(thr >> 32)) < bnd * bnd * (1.0f - 1e-5f)) break;
  }
  const float nn1 = sqrtf(__uint_as_float((uint32_t)(bk[1] >> 32)));   // nearest other point (self is one of the first two)
  // neighbourhood mean and covariance about it (two passes, coordinates relative to P): each of
  // the k neighbours is one 16-byte record of the cell-sorted array (near each other and near the
  // wavefront's other queries), found through the point -> position map
  const float inv_k = 1.0f / (float)k;
  uint32_t pos[K];
#pragma unroll
  for (int q = 0; q < K; ++q) pos[q] = q < k ? pos_of[(uint32_t)bk[q]] : (uint32_t)s;
  float mx = 0.f, my = 0.f, mz = 0.f;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (q < k) {
      const float4 Q = sorted[pos[q]];
      mx += Q.x - P.x; my += Q.y - P.y; mz += Q.z - P.z;
    }
  }
  mx *= inv_k; my *= inv_k; mz *= inv_k;
  float c00 = 0.f, c01 = 0.f, c02 = 0.f, c11 = 0.f, c12 = 0.f, c22 = 0.f;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (q < k) {
      const float4 Q = sorted[pos[q]];
      const float ex = (Q.x - P.x) - mx, ey = (Q.y - P.y) - my, ez = (Q.z - P.z) - mz;
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
  // the query's record in cell order (stores of consecutive lanes are adjacent); a second kernel
  // moves it to the point's index
  float4* rec = stage + 3 * s;
  rec[0] = make_float4(qw * sg, qx * sg, qy * sg, qz * sg);
  rec[1] = make_float4(s0, s1, s2, nn1);
  rec[2] = make_float4(nn[0], nn[1], nn[2], 0.0f);
}

// Every point's outputs from its record: one gathered 48-byte record, planar stores in index
// order.
__global__ __launch_bounds__(256) void k_knn_unpermute(const float4* __restrict__ stage,
                                                       const uint32_t* __restrict__ pos_of, int64_t n,
                                                       float* __restrict__ quat, float* __restrict__ scale,
                                                       float* __restrict__ normal, float* __restrict__ nn_dist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4* rec = stage + 3 * (int64_t)pos_of[i];
  const float4 a = rec[0], b = rec[1], c = rec[2];
  quat[i] = a.x;
  quat[n + i] = a.y;
  quat[2 * n + i] = a.z;
  quat[3 * n + i] = a.w;
  scale[i] = b.x;
  scale[n + i] = b.y;
  scale[2 * n + i] = b.z;
  normal[i] = c.x;
  normal[n + i] = c.y;
  normal[2 * n + i] = c.z;
  if (nn_dist) nn_dist[i] = b.w;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// Scratch layout: a 256-byte header [box 6 x u32 | pad | sums 3 x f64 | scan total (u64)], the
// blocks' bounds partials (1024 x 48 B), cell_id[n], sorted[n] (float4), the results in cell order
// (3 float4 per point), counts[kMaxCells + 1], cell_start[kMaxCells + 1], scan scratch.
constexpr int kBoundsBlocks = 1024;
constexpr size_t kHeader = 256;
constexpr size_t kPartBytes = kBoundsBlocks * sizeof(BoundsPart);

size_t knn_scratch_bytes(int64_t n) {
  return kHeader + kPartBytes + (size_t)n * 4 + 64 + (size_t)n * 16 + (size_t)n * 48 + 2 * ((size_t)kMaxCells + 64) * 4 +
         scan_scratch_bytes(kMaxCells + 1) + 256;
}

hipError_t launch_knn_pca(const float* xyz, int64_t n, int k, float kappa, float floor_ratio,
                          float* quat, float* scale, float* normal, float* nn_dist, void* scratch,
                          size_t scratch_bytes, uint32_t* host_pinned, hipStream_t s) {
  if (scratch_bytes < knn_scratch_bytes(n)) return hipErrorInvalidValue;
  char* base = reinterpret_cast<char*>(scratch);
  uint32_t* box = reinterpret_cast<uint32_t*>(base);
  double* sums = reinterpret_cast<double*>(base + 32);
  uint64_t* total = reinterpret_cast<uint64_t*>(base + 64);
  BoundsPart* parts = reinterpret_cast<BoundsPart*>(base + kHeader);
  uint32_t* cell_id = reinterpret_cast<uint32_t*>(base + kHeader + kPartBytes);
  float4* sorted = reinterpret_cast<float4*>(reinterpret_cast<char*>(cell_id) + ((n * 4 + 63) / 64) * 64);
  float4* stage = sorted + n;
  uint32_t* counts = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(stage) + n * 48);
  uint32_t* cell_start = counts + kMaxCells + 64;
  void* scan_scr = cell_start + kMaxCells + 64;
  hipError_t e = hipSuccess;
  const int bb = (int)std::min<int64_t>(kBoundsBlocks, (n + 255) / 256);
  hipLaunchKernelGGL(k_bounds, dim3(bb), dim3(256), 0, s, xyz, n, parts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(256), 0, s, parts, bb, box, sums);
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
  // about one point per cell if the cloud filled its box
  const GridInfo G = grid_for(lo[0], lo[1], lo[2], ext[0], ext[1], ext[2],
                              std::max(std::cbrt(vol / (double)n), emax / 1024.0));
  if ((e = launch_fill_u32(counts, 0u, G.ncells + 1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_count, dim3(blocks_for(n, 256)), dim3(256), 0, s, xyz, n, G, cell_id, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_scan(counts, nullptr, nullptr, nullptr, cell_start, G.ncells + 1, total, scan_scr, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(counts, 0u, G.ncells + 1, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, xyz, n, cell_id,
                     cell_start, counts, sorted);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (k <= 16) {
    hipLaunchKernelGGL(k_knn_pca<16>, dim3(blocks_for(n, kSearchThreads)), dim3(kSearchThreads), 0, s, sorted,
                       cell_id, n, k, G, cell_start, sums, kappa, floor_ratio, stage);
  } else {
    hipLaunchKernelGGL(k_knn_pca<32>, dim3(blocks_for(n, kSearchThreads)), dim3(kSearchThreads), 0, s, sorted,
                       cell_id, n, k, G, cell_start, sums, kappa, floor_ratio, stage);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_knn_unpermute, dim3(blocks_for(n, 256)), dim3(256), 0, s, stage, cell_id, n, quat, scale,
                     normal, nn_dist);
  return hipGetLastError();
}

}  // namespace pcs
