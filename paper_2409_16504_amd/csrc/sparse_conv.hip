// Sparse point-to-ellipsoid estimator (Section 3.2; the configuration-4 network): voxelisation,
// kernel map, submanifold 3x3x3 convolution on BF16 MFMA with FP32 accumulation (forward, data
// gradient, weight gradient) and the per-voxel head with its activations.
//
//  * voxelise: the grid coordinate of every point (a grid of up to 1024^3 voxels over [-1,1]^3) is
//    a 30-bit key; a radix sort of
//    (key, point) groups the points of a voxel, a scan of key changes numbers the voxels in key
//    order, one thread per voxel averages colour and coordinate residual; an open-addressing hash
//    of the keys answers the 27 neighbour queries of every voxel (the kernel map).
//  * convolution: output-stationary gather-GEMM. A block owns 256 output voxels (64 per
//    wavefront, four 16-row MFMA tiles); for each of the 27 offsets the offset's weights are
//    staged in LDS, each lane gathers 8 BF16 input channels of its row's neighbour (zeros where
//    the neighbour is absent) and v_mfma_f32_16x16x32_bf16 accumulates in FP32. Bias and ReLU are
//    fused into the epilogue, which rounds to BF16.
//  * data gradient: the same kernel with weights W'_k = W_{26-k}^T (submanifold maps are
//    symmetric: j = nbr_k(i) <=> i = nbr_{26-k}(j), so dx_j = sum_k W_{26-k} dy_{nbr_k(j)}).
//  * weight gradient: dW_k = sum_i x_{nbr_k(i)} dy_i^T as an MFMA reduction over voxels; each
//    block stages 64 voxels of dy and of the gathered inputs transposed in LDS, accumulates its
//    voxel range in registers and adds its partial matrix once with float atomics.

#include "pcs_internal.hpp"

namespace pcs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;   // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);                                           // nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, sizeof r);
  return r;
}

__device__ __forceinline__ uint32_t hash_slot(uint32_t key, int log2cap) {
  return (key * 0x9E3779B1u) >> (32 - log2cap);
}

// ---- voxelisation -----------------------------------------------------------------------------
// Voxel key (x << 2b) | (y << b) | z with b = log2(grid): lexicographic (x, y, z) order in 3b bits,
// so the sort runs ceil(3b / 8) passes.
__global__ void k_vox_key(const float* __restrict__ xyz, int64_t n, int grid, int b,
                          uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float g = floorf((xyz[a * n + i] + 1.0f) * (0.5f * (float)grid));
    c[a] = (uint32_t)fminf(fmaxf(g, 0.0f), (float)(grid - 1));
  }
  keys[i] = (c[0] << (2 * b)) | (c[1] << b) | c[2];
  vals[i] = (uint32_t)i;
}

__global__ void k_vox_flag(const uint32_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  flag[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1u : 0u;
}

__global__ void k_vox_start(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ excl,
                            int64_t n, uint32_t* __restrict__ start) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (flag[j]) start[excl[j]] = (uint32_t)j;
}

// One thread per voxel: coordinates, mean colour, residual and position (features, BF16, 32
// channels: rgb, residual, absolute position in [-1, 1]^3, zero padding), point -> voxel map and
// hash insertion.
__global__ void k_vox_reduce(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ order,
                             const uint32_t* __restrict__ start, int64_t V, int64_t n,
                             const float* __restrict__ xyz, const float* __restrict__ rgb, int grid, int gb,
                             int32_t* __restrict__ coords, uint16_t* __restrict__ feat,
                             int32_t* __restrict__ point_voxel, uint32_t* __restrict__ hkeys,
                             int32_t* __restrict__ hvals, int log2cap) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const uint32_t b = start[v], e = (v + 1 < V) ? start[v + 1] : (uint32_t)n;
  const uint32_t key = keys[b];
  const int cx = (int)(key >> (2 * gb)), cy = (int)(key >> gb) & (grid - 1), cz = (int)key & (grid - 1);
  coords[v] = cx;
  coords[V + v] = cy;
  coords[2 * V + v] = cz;
  if (!feat) {
    // a pooled level: the parents' features come from their children, not from these points
    for (uint32_t j = b; j < e; ++j) point_voxel[order[j]] = (int32_t)v;
  } else {
    float s[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (uint32_t j = b; j < e; ++j) {
      const uint32_t i = order[j];
      point_voxel[i] = (int32_t)v;
      s[0] += rgb[i];
      s[1] += rgb[n + i];
      s[2] += rgb[2 * n + i];
      const float half = 0.5f * (float)grid;
      const float px = xyz[i], py = xyz[n + i], pz = xyz[2 * n + i];
      s[3] += (px + 1.0f) * half - ((float)cx + 0.5f);
      s[4] += (py + 1.0f) * half - ((float)cy + 0.5f);
      s[5] += (pz + 1.0f) * half - ((float)cz + 0.5f);
      s[6] += px;
      s[7] += py;
      s[8] += pz;
    }
    const float inv = 1.0f / (float)(e - b);
    uint16_t f[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) f[c] = c < 9 ? f32_to_bf16(s[c] * inv) : (uint16_t)0;
    uint4* dst = reinterpret_cast<uint4*>(feat + v * 32);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint4 w;
      w.x = f[8 * q + 0] | ((uint32_t)f[8 * q + 1] << 16);
      w.y = f[8 * q + 2] | ((uint32_t)f[8 * q + 3] << 16);
      w.z = f[8 * q + 4] | ((uint32_t)f[8 * q + 5] << 16);
      w.w = f[8 * q + 6] | ((uint32_t)f[8 * q + 7] << 16);
      dst[q] = w;
    }
  }
  // insert into the hash table under the 10-bit-field key the kernel map looks up (keys are
  // unique; linear probing always finds a free slot because the table holds at most half its
  // capacity)
  const uint32_t k32 = ((uint32_t)cx << 20) | ((uint32_t)cy << 10) | (uint32_t)cz;
  const uint32_t mask = (1u << log2cap) - 1u;
  uint32_t slot = hash_slot(k32, log2cap);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const uint32_t prev = atomicCAS(&hkeys[slot], kEmptyKey, k32);
    if (prev == kEmptyKey) {
      hvals[slot] = (int32_t)v;
      break;
    }
    slot = (slot + 1) & mask;
  }
}

// The 27 neighbours of every voxel by hash lookup. The first probe of all 27 keys is issued at
// once (27 loads in flight per thread), and so are the value loads of the hits; only keys whose
// first slot holds another key probe on (linear probing, the table at most half full).
__global__ __launch_bounds__(256) void k_kernel_map(const int32_t* __restrict__ coords, int64_t V, int grid,
                                                    const uint32_t* __restrict__ hkeys,
                                                    const int32_t* __restrict__ hvals, int log2cap,
                                                    int32_t* __restrict__ nbr) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int cx = coords[v], cy = coords[V + v], cz = coords[2 * V + v];
  const uint32_t mask = (1u << log2cap) - 1u;
  uint32_t key[27], slot[27], hk[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) {
    const int x = cx + (k / 9) - 1, y = cy + ((k / 3) % 3) - 1, z = cz + (k % 3) - 1;
    const bool in = x >= 0 && x < grid && y >= 0 && y < grid && z >= 0 && z < grid;
    key[k] = in ? (((uint32_t)x << 20) | ((uint32_t)y << 10) | (uint32_t)z) : kEmptyKey;
    slot[k] = in ? hash_slot(key[k], log2cap) : 0u;
  }
#pragma unroll
  for (int k = 0; k < 27; ++k) hk[k] = key[k] != kEmptyKey ? hkeys[slot[k]] : kEmptyKey;
  // keys whose first slot holds another key probe on (rare)
#pragma unroll
  for (int k = 0; k < 27; ++k) {
    if (key[k] == kEmptyKey) continue;
    for (uint32_t probe = 1; hk[k] != key[k] && hk[k] != kEmptyKey && probe <= mask; ++probe) {
      slot[k] = (slot[k] + 1) & mask;
      hk[k] = hkeys[slot[k]];
    }
  }
  int32_t found[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) found[k] = (key[k] != kEmptyKey && hk[k] == key[k]) ? hvals[slot[k]] : -1;
#pragma unroll
  for (int k = 0; k < 27; ++k) nbr[(int64_t)k * V + v] = found[k];
}

// ---- convolution ------------------------------------------------------------------------------
constexpr int kConvWaves = 4;                  // wavefronts per block
constexpr int kConvTiles = 1;                  // 16-row MFMA tiles per wavefront
// y[v][o] = relu?(bias[o] + sum_k sum_c W[k][o][c] x[nbr_k(v)][c]) over n_off offsets (27 for a
// submanifold 3x3x3 convolution, 8 for a stride-2 transposed 2x2x2 one); wt is [n_off][COUT][CIN]
// BF16 and nbr is [n_off][V]. HALVES: the input rows are the concatenation of x ([V][CIN / 2]) and
// x2 ([V][CIN / 2]) along the channels, read where they lie.
template <int CIN, int COUT, int MB, bool HALVES>
__global__ __launch_bounds__(256) void k_subm_conv(const uint16_t* __restrict__ x,
                                                   const uint16_t* __restrict__ wt,
                                                   const float* __restrict__ bias,
                                                   const int32_t* __restrict__ nbr, int64_t V,
                                                   int relu, uint16_t* __restrict__ y, int n_off,
                                                   const uint16_t* __restrict__ x2) {
  constexpr int KC = CIN / 32;       // K chunks of 32 channels
  constexpr int NB = COUT / 16;      // 16-column output blocks
  constexpr int LDW = CIN + 8;       // padded LDS row (avoids bank conflicts)
  __shared__ uint16_t s_w[COUT * LDW];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int64_t vbase = (int64_t)blockIdx.x * (kConvWaves * 16 * MB) + wave * (16 * MB);
  const int row = lane % 16, grp = lane / 16;
  f32x4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Software pipeline over the offsets: offset k + 1's weight slice (16 bytes per thread per pass,
  // kWQ passes), neighbour indices and gathered input rows are loaded into registers while offset
  // k's products run, so each offset waits on LDS only.
  constexpr int kWQ = (COUT * CIN / 8 + 255) / 256;
  uint4 wreg[kWQ];
  uint4 arow[MB][KC];
  static_assert(!HALVES || KC % 2 == 0, "the halves are whole 32-channel chunks");
  constexpr int LDX = HALVES ? CIN / 2 : CIN;       // row stride of x (and of x2)
  auto load_offset = [&](int k) {
    const uint4* wsrc = reinterpret_cast<const uint4*>(wt + (int64_t)k * COUT * CIN);
#pragma unroll
    for (int i = 0; i < kWQ; ++i) {
      const int q = tid + i * 256;
      wreg[i] = q < COUT * CIN / 8 ? wsrc[q] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int64_t v = vbase + mb * 16 + row;
      const int32_t j = v < V ? nbr[(int64_t)k * V + v] : -1;
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const bool second = HALVES && kc >= KC / 2;
        const uint16_t* piece = (second ? x2 : x) + (int64_t)j * LDX + (second ? kc - KC / 2 : kc) * 32 + grp * 8;
        arow[mb][kc] = j >= 0 ? *reinterpret_cast<const uint4*>(piece) : make_uint4(0u, 0u, 0u, 0u);
      }
    }
  };
  if (n_off > 0) load_offset(0);
  for (int k = 0; k < n_off; ++k) {
    __syncthreads();                                   // the last offset's LDS reads are done
    // stage W_k into LDS: COUT x CIN BF16
#pragma unroll
    for (int i = 0; i < kWQ; ++i) {
      const int q = tid + i * 256;
      if (q < COUT * CIN / 8) {
        const int o = (q * 8) / CIN, c = (q * 8) % CIN;
        *reinterpret_cast<uint4*>(&s_w[o * LDW + c]) = wreg[i];
      }
    }
    uint4 acur[MB][KC];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) acur[mb][kc] = arow[mb][kc];
    if (k + 1 < n_off) load_offset(k + 1);
    __syncthreads();
    bf16x8 bfr[KC][NB];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bfr[kc][nb] = as_bf16x8(*reinterpret_cast<const uint4*>(&s_w[(nb * 16 + row) * LDW + kc * 32 + grp * 8]));
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const bf16x8 af = as_bf16x8(acur[mb][kc]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[kc][nb], acc[mb][nb], 0, 0, 0);
      }
  }
  // epilogue: lane holds rows 4*grp + r of column row of each 16x16 block
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int o = nb * 16 + row;
      const float bo = bias ? bias[o] : 0.0f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t v = vbase + mb * 16 + grp * 4 + r;
        if (v < V) {
          float val = acc[mb][nb][r] + bo;
          if (relu) val = fmaxf(val, 0.0f);
          y[v * COUT + o] = f32_to_bf16(val);
        }
      }
    }
}

// wt_t[s][c][o] = wt[flip ? n_off - 1 - s : s][o][c]: weights of a data-gradient convolution
// (flipped for the symmetric submanifold map, not for the transposed convolution's own tables).
__global__ void k_weight_t(const uint16_t* __restrict__ wt, int n_off, int cin, int cout, int flip,
                           uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_off * cin * cout;
  if (i >= total) return;
  const int s = (int)(i / ((int64_t)cin * cout));
  const int rem = (int)(i % ((int64_t)cin * cout));
  const int c = rem / cout, o = rem % cout;
  out[i] = wt[((int64_t)(flip ? n_off - 1 - s : s) * cout + o) * cin + c];
}

// ---- pooling and upsampling tables (the encoder's 2x2x2 average pooling, the decoder's
// transposed convolution pruned to the encoder's occupancy) --------------------------------------
// World-space centre of every voxel of a G^3 grid over [-1,1]^3: voxelising the centres on the grid
// of half the resolution gives the parent voxels (c >> 1, exactly: every step is exact in FP32).
__global__ void k_voxel_centres(const int32_t* __restrict__ coords, int64_t V, int grid,
                                float* __restrict__ xyz) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const float h = 2.0f / (float)grid;
#pragma unroll
  for (int a = 0; a < 3; ++a) xyz[a * V + v] = ((float)coords[a * V + v] + 0.5f) * h - 1.0f;
}

// Upsampling tables: child j (coordinates c) sits at offset k = 4 (cx & 1) + 2 (cy & 1) + (cz & 1)
// of its parent p; fwd[k][j] = p at that offset and -1 at the other seven, bwd[k][p] = j (-1 where
// the parent has no child at offset k; bwd is filled with -1 beforehand).
__global__ void k_up_tables(const int32_t* __restrict__ child_coords, const int32_t* __restrict__ parent_of,
                            int64_t Vc, int64_t Vp, int32_t* __restrict__ fwd, int32_t* __restrict__ bwd) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Vc) return;
  const int k = 4 * (child_coords[j] & 1) + 2 * (child_coords[Vc + j] & 1) + (child_coords[2 * Vc + j] & 1);
  const int32_t p = parent_of[j];
#pragma unroll
  for (int o = 0; o < 8; ++o) fwd[(int64_t)o * Vc + j] = o == k ? p : -1;
  bwd[(int64_t)k * Vp + p] = (int32_t)j;
}

// parent_feat[p] = mean of its children's features (BF16 in and out, FP32 sums); the children of p
// are order[start[p] .. start[p + 1]) (the parent voxelisation's grouping).
__global__ void k_pool_features(const uint32_t* __restrict__ order, const uint32_t* __restrict__ start,
                                int64_t Vp, int64_t Vc, const uint16_t* __restrict__ child, int C,
                                uint16_t* __restrict__ parent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (parent, 8-channel group)
  const int groups = C / 8;
  if (i >= Vp * groups) return;
  const int64_t p = i / groups;
  const int g = (int)(i % groups);
  const uint32_t b = start[p], e = p + 1 < Vp ? start[p + 1] : (uint32_t)Vc;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (uint32_t q = b; q < e; ++q) {
    const uint4 w = *reinterpret_cast<const uint4*>(child + (int64_t)order[q] * C + g * 8);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[2 * t] += bf16_to_f32((uint16_t)(ws[t] & 0xFFFFu));
      acc[2 * t + 1] += bf16_to_f32((uint16_t)(ws[t] >> 16));
    }
  }
  const float inv = 1.0f / (float)(e - b);
  uint4 o;
  uint32_t* os = reinterpret_cast<uint32_t*>(&o);
#pragma unroll
  for (int t = 0; t < 4; ++t)
    os[t] = f32_to_bf16(acc[2 * t] * inv) | ((uint32_t)f32_to_bf16(acc[2 * t + 1] * inv) << 16);
  *reinterpret_cast<uint4*>(parent + p * C + g * 8) = o;
}

// Adjoint of the mean: d_child[j] = d_parent[p(j)] / (children of p(j)).
__global__ void k_pool_features_bwd(const int32_t* __restrict__ parent_of, const uint32_t* __restrict__ start,
                                    int64_t Vp, int64_t Vc, const uint16_t* __restrict__ dparent, int C,
                                    uint16_t* __restrict__ dchild) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Vc * C) return;
  const int64_t j = i / C;
  const int c = (int)(i % C);
  const int32_t p = parent_of[j];
  const uint32_t b = start[p], e = p + 1 < Vp ? start[p + 1] : (uint32_t)Vc;
  dchild[i] = f32_to_bf16(bf16_to_f32(dparent[(int64_t)p * C + c]) / (float)(e - b));
}

// dy_masked = dy * (y > 0) (ReLU derivative), BF16.
__global__ void k_relu_mask(const uint16_t* __restrict__ y, const uint16_t* __restrict__ dy,
                            int64_t count, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  out[i] = bf16_to_f32(y[i]) > 0.0f ? dy[i] : (uint16_t)0;
}

// Bias gradient: db[o] += sum_v dy[v][o] (block partial sums, one atomic per block and channel).
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t* __restrict__ dy, int64_t V,
                                                   int cout, float* __restrict__ db) {
  __shared__ float s[256];
  const int tid = threadIdx.x;
  const int o = tid % cout, lane_set = tid / cout, sets = 256 / cout;
  float acc = 0.f;
  for (int64_t v = (int64_t)blockIdx.x * sets + lane_set; v < V; v += (int64_t)gridDim.x * sets)
    acc += bf16_to_f32(dy[v * cout + o]);
  s[tid] = acc;
  __syncthreads();
  if (tid < cout) {
    float t = 0.f;
    for (int q = 0; q < sets; ++q) t += s[q * cout + tid];
    atomicAdd(&db[tid], t);
  }
}

// dW[k][o][c] += sum_v dy[v][o] x[nbr_k(v)][c]; blockIdx.y = k. D (COUT x CIN) = dY^T X_k with
// the voxel dimension as the MFMA reduction axis, staged transposed through LDS 64 voxels at a time.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_subm_conv_dw(const uint16_t* __restrict__ x,
                                                      const uint16_t* __restrict__ dy,
                                                      const int32_t* __restrict__ nbr, int64_t V,
                                                      int64_t chunk, float* __restrict__ dw) {
  constexpr int MB = COUT / 16, NB = CIN / 16, TILES = MB * NB, PER_WAVE = (TILES + 3) / 4;
  constexpr int LDT = 64 + 8;        // padded rows of the transposed chunks
  __shared__ uint16_t s_dyT[COUT * LDT];
  __shared__ uint16_t s_xT[CIN * LDT];
  const int k = blockIdx.y;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int row = lane % 16, grp = lane / 16;
  f32x4 acc[PER_WAVE];
#pragma unroll
  for (int t = 0; t < PER_WAVE; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t v0 = (int64_t)blockIdx.x * chunk;
  const int64_t v1 = min(V, v0 + chunk);
  for (int64_t vb = v0; vb < v1; vb += 64) {
    __syncthreads();
    // stage: thread -> (voxel slot, 8-channel group)
    for (int q = tid; q < 64 * (COUT / 8); q += 256) {
      const int slot = q / (COUT / 8), cg = (q % (COUT / 8)) * 8;
      const int64_t v = vb + slot;
      uint4 w = make_uint4(0u, 0u, 0u, 0u);
      if (v < v1) w = *reinterpret_cast<const uint4*>(dy + v * COUT + cg);
      const uint16_t* h = reinterpret_cast<const uint16_t*>(&w);
#pragma unroll
      for (int e = 0; e < 8; ++e) s_dyT[(cg + e) * LDT + slot] = h[e];
    }
    for (int q = tid; q < 64 * (CIN / 8); q += 256) {
      const int slot = q / (CIN / 8), cg = (q % (CIN / 8)) * 8;
      const int64_t v = vb + slot;
      uint4 w = make_uint4(0u, 0u, 0u, 0u);
      if (v < v1) {
        const int32_t j = nbr[(int64_t)k * V + v];
        if (j >= 0) w = *reinterpret_cast<const uint4*>(x + (int64_t)j * CIN + cg);
      }
      const uint16_t* h = reinterpret_cast<const uint16_t*>(&w);
#pragma unroll
      for (int e = 0; e < 8; ++e) s_xT[(cg + e) * LDT + slot] = h[e];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER_WAVE; ++t) {
      const int tile = wave * PER_WAVE + t;
      if (tile < TILES) {
        const int mb = tile / NB, nb = tile % NB;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const bf16x8 af = as_bf16x8(*reinterpret_cast<const uint4*>(&s_dyT[(mb * 16 + row) * LDT + ks * 32 + grp * 8]));
          const bf16x8 bf = as_bf16x8(*reinterpret_cast<const uint4*>(&s_xT[(nb * 16 + row) * LDT + ks * 32 + grp * 8]));
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[t], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < PER_WAVE; ++t) {
    const int tile = wave * PER_WAVE + t;
    if (tile < TILES) {
      const int mb = tile / NB, nb = tile % NB;
      const int c = nb * 16 + row;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = mb * 16 + grp * 4 + r;
        const float val = acc[t][r];
        if (val != 0.0f) unsafeAtomicAdd(&dw[((int64_t)k * COUT + o) * CIN + c], val);
      }
    }
  }
}

// ---- head -------------------------------------------------------------------------------------
constexpr int kHeadIn = 32, kHeadOut = 11;

struct HeadOut {
  float scale[3], q[4], qn, opacity, drgb[3];
};

__device__ __forceinline__ void head_voxel(const uint16_t* __restrict__ f, const float* s_wh,
                                           const float* s_bh, float voxel, float raw[kHeadOut],
                                           HeadOut& h) {
  float fv[kHeadIn];
  const uint4* src = reinterpret_cast<const uint4*>(f);
#pragma unroll
  for (int q = 0; q < kHeadIn / 8; ++q) {
    const uint4 w = src[q];
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      fv[8 * q + 2 * e] = bf16_to_f32((uint16_t)(ws[e] & 0xFFFF));
      fv[8 * q + 2 * e + 1] = bf16_to_f32((uint16_t)(ws[e] >> 16));
    }
  }
#pragma unroll
  for (int o = 0; o < kHeadOut; ++o) {
    float a = s_bh[o];
#pragma unroll
    for (int c = 0; c < kHeadIn; ++c) a = fmaf(s_wh[o * kHeadIn + c], fv[c], a);
    raw[o] = a;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) h.scale[a] = voxel * __expf(raw[a]);
  const float q0 = raw[3] + 1.0f, q1 = raw[4], q2 = raw[5], q3 = raw[6];
  h.qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const float iq = h.qn > 0.0f ? 1.0f / h.qn : 0.0f;
  h.q[0] = h.qn > 0.0f ? q0 * iq : 1.0f;
  h.q[1] = q1 * iq; h.q[2] = q2 * iq; h.q[3] = q3 * iq;
  h.opacity = 1.0f / (1.0f + __expf(-raw[7]));
  h.drgb[0] = raw[8]; h.drgb[1] = raw[9]; h.drgb[2] = raw[10];
}

// Per point: its voxel's scale, rotation and opacity, colour = point colour + residual, and the
// normal = rotated axis of the smallest scale oriented away from the centroid.
__global__ __launch_bounds__(256) void k_head_forward(
    const uint16_t* __restrict__ feat, const float* __restrict__ wh, const float* __restrict__ bh,
    const int32_t* __restrict__ point_voxel, const float* __restrict__ xyz,
    const float* __restrict__ rgb, const float* __restrict__ centroid, int64_t n, float voxel,
    float* __restrict__ quat, float* __restrict__ scale, float* __restrict__ opac,
    float* __restrict__ out_rgb, float* __restrict__ normal) {
  __shared__ float s_wh[kHeadOut * kHeadIn], s_bh[kHeadOut];
  for (int i = threadIdx.x; i < kHeadOut * kHeadIn; i += blockDim.x) s_wh[i] = wh[i];
  if (threadIdx.x < kHeadOut) s_bh[threadIdx.x] = bh[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t v = point_voxel[i];
  float raw[kHeadOut];
  HeadOut h;
  head_voxel(feat + (int64_t)v * kHeadIn, s_wh, s_bh, voxel, raw, h);
#pragma unroll
  for (int a = 0; a < 4; ++a) quat[a * n + i] = h.q[a];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    scale[a * n + i] = h.scale[a];
    out_rgb[a * n + i] = rgb[a * n + i] + h.drgb[a];
  }
  opac[i] = h.opacity;
  // rotation column of the smallest scale
  const int m = (h.scale[0] <= h.scale[1] && h.scale[0] <= h.scale[2]) ? 0 : (h.scale[1] <= h.scale[2] ? 1 : 2);
  const float w = h.q[0], x = h.q[1], y = h.q[2], z = h.q[3];
  float nx, ny, nz;
  if (m == 0) { nx = 1 - 2 * (y * y + z * z); ny = 2 * (x * y + w * z); nz = 2 * (x * z - w * y); }
  else if (m == 1) { nx = 2 * (x * y - w * z); ny = 1 - 2 * (x * x + z * z); nz = 2 * (y * z + w * x); }
  else { nx = 2 * (x * z + w * y); ny = 2 * (y * z - w * x); nz = 1 - 2 * (x * x + y * y); }
  const float dx = xyz[i] - centroid[0], dy = xyz[n + i] - centroid[1], dz = xyz[2 * n + i] - centroid[2];
  if (nx * dx + ny * dy + nz * dz < 0.0f) { nx = -nx; ny = -ny; nz = -nz; }
  normal[i] = nx; normal[n + i] = ny; normal[2 * n + i] = nz;
}

// Per voxel: gradients of its points' (quat, scale, opacity, rgb) summed (points are contiguous in
// voxel order), chained through the activations to raw, then to the features and head weights.
// The normal is not differentiated (the training loss supervises colour only).
__global__ __launch_bounds__(256) void k_head_backward(
    const uint16_t* __restrict__ feat, const float* __restrict__ wh, const float* __restrict__ bh,
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ start, int64_t V, int64_t n,
    float voxel, const float* __restrict__ d_quat, const float* __restrict__ d_scale,
    const float* __restrict__ d_opac, const float* __restrict__ d_rgb, uint16_t* __restrict__ d_feat,
    float* __restrict__ d_wh, float* __restrict__ d_bh) {
  __shared__ float s_wh[kHeadOut * kHeadIn], s_bh[kHeadOut];
  __shared__ float s_dwh[kHeadOut * kHeadIn], s_dbh[kHeadOut];
  for (int i = threadIdx.x; i < kHeadOut * kHeadIn; i += blockDim.x) { s_wh[i] = wh[i]; s_dwh[i] = 0.f; }
  if (threadIdx.x < kHeadOut) { s_bh[threadIdx.x] = bh[threadIdx.x]; s_dbh[threadIdx.x] = 0.f; }
  __syncthreads();
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < V) {
    float raw[kHeadOut];
    HeadOut h;
    head_voxel(feat + v * kHeadIn, s_wh, s_bh, voxel, raw, h);
    float gq[4] = {0.f, 0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, go = 0.f, gc[3] = {0.f, 0.f, 0.f};
    const uint32_t b = start[v], e = (v + 1 < V) ? start[v + 1] : (uint32_t)n;
    for (uint32_t j = b; j < e; ++j) {
      const uint32_t i = order[j];
#pragma unroll
      for (int a = 0; a < 4; ++a) gq[a] += d_quat[a * n + i];
#pragma unroll
      for (int a = 0; a < 3; ++a) { gs[a] += d_scale[a * n + i]; gc[a] += d_rgb[a * n + i]; }
      go += d_opac[i];
    }
    float graw[kHeadOut];
#pragma unroll
    for (int a = 0; a < 3; ++a) graw[a] = gs[a] * h.scale[a];
    const float dot = h.q[0] * gq[0] + h.q[1] * gq[1] + h.q[2] * gq[2] + h.q[3] * gq[3];
    const float iq = h.qn > 0.0f ? 1.0f / h.qn : 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) graw[3 + a] = (gq[a] - h.q[a] * dot) * iq;
    graw[7] = go * h.opacity * (1.0f - h.opacity);
#pragma unroll
    for (int a = 0; a < 3; ++a) graw[8 + a] = gc[a];
    float fv[kHeadIn];
    const uint16_t* fr = feat + v * kHeadIn;
#pragma unroll
    for (int c = 0; c < kHeadIn; ++c) fv[c] = bf16_to_f32(fr[c]);
#pragma unroll
    for (int c = 0; c < kHeadIn; ++c) {
      float a = 0.f;
#pragma unroll
      for (int o = 0; o < kHeadOut; ++o) a = fmaf(s_wh[o * kHeadIn + c], graw[o], a);
      d_feat[v * kHeadIn + c] = f32_to_bf16(a);
    }
#pragma unroll
    for (int o = 0; o < kHeadOut; ++o) {
      if (graw[o] == 0.0f) continue;
      atomicAdd(&s_dbh[o], graw[o]);
#pragma unroll
      for (int c = 0; c < kHeadIn; ++c) atomicAdd(&s_dwh[o * kHeadIn + c], graw[o] * fv[c]);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHeadOut * kHeadIn; i += blockDim.x)
    if (s_dwh[i] != 0.0f) unsafeAtomicAdd(&d_wh[i], s_dwh[i]);
  if (threadIdx.x < kHeadOut && s_dbh[threadIdx.x] != 0.0f) unsafeAtomicAdd(&d_bh[threadIdx.x], s_dbh[threadIdx.x]);
}

// ---- the UNet's head (Section 3.2): a shared MLP per point ------------------------------------
// Input of point i: the 32 decoder features of its voxel and its own coordinate residual (in voxel
// edges, as the voxelisation computes it), 35 values; ReLU hidden layer of 32; 14 outputs
// (offset 3, log-scale 3, rotation 4, opacity 1, normal 3), activated per point.
constexpr int kMlpFeat = 32, kMlpIn = 35, kMlpHidden = 32, kMlpOut = 14;

__device__ __forceinline__ void load_feat32(const uint16_t* __restrict__ f, float* fv) {
  const uint4* q4 = reinterpret_cast<const uint4*>(f);
#pragma unroll
  for (int q = 0; q < kMlpFeat / 8; ++q) {
    const uint4 w = q4[q];
    const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      fv[8 * q + 2 * t] = __uint_as_float(u[t] << 16);
      fv[8 * q + 2 * t + 1] = __uint_as_float(u[t] & 0xFFFF0000u);
    }
  }
}

// The MLP input of point i in voxel v.
__device__ __forceinline__ void point_input(const uint16_t* __restrict__ feat, const int32_t* __restrict__ coords,
                                            int64_t V, const float* __restrict__ xyz, int64_t n, int64_t i,
                                            int32_t v, float half, float (&in)[kMlpIn]) {
  load_feat32(feat + (int64_t)v * kMlpFeat, in);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    in[kMlpFeat + k] = (xyz[k * n + i] + 1.0f) * half - ((float)coords[k * V + v] + 0.5f);
}

__device__ __forceinline__ void mlp_forward(const float (&in)[kMlpIn], const float* s_w1, const float* s_b1,
                                            const float* s_w2, const float* s_b2, float (&h)[kMlpHidden],
                                            float (&raw)[kMlpOut]) {
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) raw[o] = s_b2[o];
#pragma unroll 4
  for (int j = 0; j < kMlpHidden; ++j) {
    float a = s_b1[j];
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) a = fmaf(s_w1[j * kMlpIn + c], in[c], a);
    a = fmaxf(a, 0.0f);
    h[j] = a;
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) raw[o] = fmaf(s_w2[o * kMlpHidden + j], a, raw[o]);
  }
}

struct MlpAct {
  float delta[3], th[3], scale[3], q[4], qn, opacity, n[3], nn;
};

__device__ __forceinline__ MlpAct mlp_activate(const float* r, float voxel) {
  MlpAct a;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a.th[k] = tanhf(r[k]);
    a.delta[k] = voxel * a.th[k];
    a.scale[k] = voxel * __expf(r[3 + k]);
  }
  const float q0 = r[6] + 1.0f, q1 = r[7], q2 = r[8], q3 = r[9];
  a.qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const float iq = a.qn > 0.0f ? 1.0f / a.qn : 0.0f;
  a.q[0] = a.qn > 0.0f ? q0 * iq : 1.0f;
  a.q[1] = q1 * iq; a.q[2] = q2 * iq; a.q[3] = q3 * iq;
  a.opacity = 1.0f / (1.0f + __expf(-r[10]));
  a.nn = sqrtf(r[11] * r[11] + r[12] * r[12] + r[13] * r[13]);
  const float in = a.nn > 0.0f ? 1.0f / a.nn : 0.0f;
  a.n[0] = r[11] * in; a.n[1] = r[12] * in; a.n[2] = r[13] * in;
  return a;
}

// Gradient of the raw outputs from point i's upstream gradients through the activations.
__device__ __forceinline__ void mlp_act_grad(const MlpAct& a, float voxel, int64_t i, int64_t n,
                                             const float* __restrict__ d_mean, const float* __restrict__ d_quat,
                                             const float* __restrict__ d_scale, const float* __restrict__ d_opac,
                                             const float* __restrict__ d_normal, float (&g)[kMlpOut]) {
  float gm[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, go = 0.f;
  float gn[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d_mean) gm[k] = d_mean[k * n + i];
    if (d_scale) gs[k] = d_scale[k * n + i];
    if (d_normal) gn[k] = d_normal[k * n + i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (d_quat) gq[k] = d_quat[k * n + i];
  if (d_opac) go = d_opac[i];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g[k] = gm[k] * voxel * (1.0f - a.th[k] * a.th[k]);
    g[3 + k] = gs[k] * a.scale[k];
  }
  const float dq = a.q[0] * gq[0] + a.q[1] * gq[1] + a.q[2] * gq[2] + a.q[3] * gq[3];
  const float iq = a.qn > 0.0f ? 1.0f / a.qn : 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) g[6 + k] = (gq[k] - a.q[k] * dq) * iq;
  g[10] = go * a.opacity * (1.0f - a.opacity);
  const float dn = a.n[0] * gn[0] + a.n[1] * gn[1] + a.n[2] * gn[2];
  const float in = a.nn > 0.0f ? 1.0f / a.nn : 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) g[11 + k] = (gn[k] - a.n[k] * dn) * in;
}

// The hidden layer's gradient (after the ReLU) from the raw outputs' gradient.
__device__ __forceinline__ void mlp_hidden_grad(const float (&h)[kMlpHidden], const float (&g)[kMlpOut],
                                                const float* s_w2, float (&gh)[kMlpHidden]) {
#pragma unroll
  for (int j = 0; j < kMlpHidden; ++j) {
    float t = 0.f;
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) t = fmaf(s_w2[o * kMlpHidden + j], g[o], t);
    gh[j] = h[j] > 0.0f ? t : 0.0f;
  }
}

#define PCS_MLP_WEIGHTS_TO_LDS(NT)                                                                  \
  __shared__ float s_w1[kMlpHidden * kMlpIn], s_b1[kMlpHidden], s_w2[kMlpOut * kMlpHidden], s_b2[kMlpOut]; \
  for (int t_ = threadIdx.x; t_ < kMlpHidden * kMlpIn; t_ += (NT)) s_w1[t_] = w1[t_];              \
  for (int t_ = threadIdx.x; t_ < kMlpOut * kMlpHidden; t_ += (NT)) s_w2[t_] = w2[t_];             \
  if (threadIdx.x < kMlpHidden) s_b1[threadIdx.x] = b1[threadIdx.x];                               \
  if (threadIdx.x < kMlpOut) s_b2[threadIdx.x] = b2[threadIdx.x];                                  \
  __syncthreads();

// One thread per point: the MLP on its input, activated; mean = point + offset, colour = the
// point's own.
__global__ __launch_bounds__(256) void k_mlp_points(const uint16_t* __restrict__ feat, const int32_t* __restrict__ coords,
                                                    int64_t V, const int32_t* __restrict__ point_voxel,
                                                    const float* __restrict__ w1, const float* __restrict__ b1,
                                                    const float* __restrict__ w2, const float* __restrict__ b2,
                                                    const float* __restrict__ xyz, const float* __restrict__ rgb,
                                                    int64_t n, int grid, float* __restrict__ mean,
                                                    float* __restrict__ quat, float* __restrict__ scale,
                                                    float* __restrict__ opac, float* __restrict__ out_rgb,
                                                    float* __restrict__ normal) {
  PCS_MLP_WEIGHTS_TO_LDS(256)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float half = 0.5f * (float)grid, voxel = 2.0f / (float)grid;
  float in[kMlpIn], h[kMlpHidden], r[kMlpOut];
  point_input(feat, coords, V, xyz, n, i, point_voxel[i], half, in);
  mlp_forward(in, s_w1, s_b1, s_w2, s_b2, h, r);
  const MlpAct a = mlp_activate(r, voxel);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    mean[k * n + i] = xyz[k * n + i] + a.delta[k];
    scale[k * n + i] = a.scale[k];
    out_rgb[k * n + i] = rgb[k * n + i];
    normal[k * n + i] = a.n[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) quat[k * n + i] = a.q[k];
  opac[i] = a.opacity;
}

// Weight gradients of the head: one row per point, points taken in voxel order (row p is point
// order[p]), kMlpBwdThreads rows per block. Each thread recomputes its point's input, hidden layer
// and outputs, keeps the input, the hidden values and both layers' output gradients in LDS, and
// stores the hidden-layer gradient to gh[p][32] for the feature gradients. The weight gradients are
// the block's sums of outer products, one weight element per thread at a time, added once per block.
constexpr int kMlpBwdThreads = 128;
constexpr int kMlpRowIn = 37, kMlpRow = 33;      // padded LDS rows
__global__ __launch_bounds__(kMlpBwdThreads) void k_mlp_wgrad(
    const uint16_t* __restrict__ feat, const int32_t* __restrict__ coords, int64_t V,
    const int32_t* __restrict__ point_voxel, const uint32_t* __restrict__ order, const float* __restrict__ w1,
    const float* __restrict__ b1, const float* __restrict__ w2, const float* __restrict__ b2,
    const float* __restrict__ xyz, int64_t n, int grid, const float* __restrict__ d_mean,
    const float* __restrict__ d_quat, const float* __restrict__ d_scale, const float* __restrict__ d_opac,
    const float* __restrict__ d_normal, float* __restrict__ gh_out, float* __restrict__ d_w1,
    float* __restrict__ d_b1, float* __restrict__ d_w2, float* __restrict__ d_b2) {
  PCS_MLP_WEIGHTS_TO_LDS(kMlpBwdThreads)
  __shared__ float s_f[kMlpBwdThreads * kMlpRowIn], s_h[kMlpBwdThreads * kMlpRow];
  __shared__ float s_gh[kMlpBwdThreads * kMlpRow], s_g[kMlpBwdThreads * 15];
  const int tid = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * kMlpBwdThreads + tid;
  float* F = s_f + tid * kMlpRowIn;
  float* Hh = s_h + tid * kMlpRow;
  float* GH = s_gh + tid * kMlpRow;
  float* G = s_g + tid * 15;
  if (p < n) {
    const int64_t i = order[p];
    const float half = 0.5f * (float)grid, voxel = 2.0f / (float)grid;
    float in[kMlpIn], h[kMlpHidden], r[kMlpOut], g[kMlpOut], gh[kMlpHidden];
    point_input(feat, coords, V, xyz, n, i, point_voxel[i], half, in);
    mlp_forward(in, s_w1, s_b1, s_w2, s_b2, h, r);
    const MlpAct a = mlp_activate(r, voxel);
    mlp_act_grad(a, voxel, i, n, d_mean, d_quat, d_scale, d_opac, d_normal, g);
    mlp_hidden_grad(h, g, s_w2, gh);
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) F[c] = in[c];
#pragma unroll
    for (int j = 0; j < kMlpHidden; ++j) { Hh[j] = h[j]; GH[j] = gh[j]; }
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) G[o] = g[o];
    float4* dst = reinterpret_cast<float4*>(gh_out + p * kMlpHidden);
#pragma unroll
    for (int j = 0; j < kMlpHidden; j += 4) dst[j / 4] = make_float4(gh[j], gh[j + 1], gh[j + 2], gh[j + 3]);
  } else {
    // rows past the last point add nothing to the sums
    for (int c = 0; c < kMlpRowIn; ++c) F[c] = 0.f;
    for (int c = 0; c < kMlpRow; ++c) { Hh[c] = 0.f; GH[c] = 0.f; }
    for (int o = 0; o < 15; ++o) G[o] = 0.f;
  }
  __syncthreads();
  // dW2[o][j] = sum G[o] H[j], dW1[j][c] = sum GH[j] F[c], and the biases
  constexpr int kW2 = kMlpOut * kMlpHidden, kW1 = kMlpHidden * kMlpIn;
  for (int el = tid; el < kW2 + kW1 + kMlpOut + kMlpHidden; el += kMlpBwdThreads) {
    float acc = 0.f;
    if (el < kW2) {
      const int o = el / kMlpHidden, j = el % kMlpHidden;
      for (int u = 0; u < kMlpBwdThreads; ++u) acc = fmaf(s_g[u * 15 + o], s_h[u * kMlpRow + j], acc);
      if (acc != 0.0f) unsafeAtomicAdd(&d_w2[el], acc);
    } else if (el < kW2 + kW1) {
      const int e2 = el - kW2, j = e2 / kMlpIn, c = e2 % kMlpIn;
      for (int u = 0; u < kMlpBwdThreads; ++u) acc = fmaf(s_gh[u * kMlpRow + j], s_f[u * kMlpRowIn + c], acc);
      if (acc != 0.0f) unsafeAtomicAdd(&d_w1[e2], acc);
    } else if (el < kW2 + kW1 + kMlpOut) {
      const int o = el - kW2 - kW1;
      for (int u = 0; u < kMlpBwdThreads; ++u) acc += s_g[u * 15 + o];
      if (acc != 0.0f) unsafeAtomicAdd(&d_b2[o], acc);
    } else {
      const int j = el - kW2 - kW1 - kMlpOut;
      for (int u = 0; u < kMlpBwdThreads; ++u) acc += s_gh[u * kMlpRow + j];
      if (acc != 0.0f) unsafeAtomicAdd(&d_b1[j], acc);
    }
  }
}

// Feature gradients of the head: one thread per voxel sums the hidden-layer gradients of its points
// (rows start[v] .. start[v+1] of gh, voxel order) and maps the sum through the feature columns of
// the first layer: d feat = W1[:, :32]^T sum_i gh_i (the residual columns give no feature gradient).
__global__ __launch_bounds__(256) void k_mlp_dfeat(const float* __restrict__ gh, const uint32_t* __restrict__ start,
                                                   int64_t V, int64_t n, const float* __restrict__ w1,
                                                   uint16_t* __restrict__ d_feat) {
  __shared__ float s_w1[kMlpHidden * kMlpIn];
  for (int t = threadIdx.x; t < kMlpHidden * kMlpIn; t += 256) s_w1[t] = w1[t];
  __syncthreads();
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  float sgh[kMlpHidden];
#pragma unroll
  for (int j = 0; j < kMlpHidden; ++j) sgh[j] = 0.0f;
  const uint32_t b = start[v], e = v + 1 < V ? start[v + 1] : (uint32_t)n;
  for (uint32_t p = b; p < e; ++p) {
    const float4* row = reinterpret_cast<const float4*>(gh + (int64_t)p * kMlpHidden);
#pragma unroll
    for (int j = 0; j < kMlpHidden; j += 4) {
      const float4 t = row[j / 4];
      sgh[j] += t.x; sgh[j + 1] += t.y; sgh[j + 2] += t.z; sgh[j + 3] += t.w;
    }
  }
#pragma unroll
  for (int c = 0; c < kMlpFeat; c += 8) {
    float df[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) df[t] = 0.0f;
#pragma unroll
    for (int j = 0; j < kMlpHidden; ++j)
#pragma unroll
      for (int t = 0; t < 8; ++t) df[t] = fmaf(s_w1[j * kMlpIn + c + t], sgh[j], df[t]);
    uint4 w;
    w.x = f32_to_bf16(df[0]) | ((uint32_t)f32_to_bf16(df[1]) << 16);
    w.y = f32_to_bf16(df[2]) | ((uint32_t)f32_to_bf16(df[3]) << 16);
    w.z = f32_to_bf16(df[4]) | ((uint32_t)f32_to_bf16(df[5]) << 16);
    w.w = f32_to_bf16(df[6]) | ((uint32_t)f32_to_bf16(df[7]) << 16);
    *reinterpret_cast<uint4*>(d_feat + v * kMlpFeat + c) = w;
  }
}

__global__ __launch_bounds__(256) void k_centroid(const float* __restrict__ xyz, int64_t n,
                                                  double* __restrict__ sum) {
  __shared__ double s[3][256];
  double a[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int c = 0; c < 3; ++c) a[c] += xyz[c * n + i];
  for (int c = 0; c < 3; ++c) s[c][threadIdx.x] = a[c];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 3; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) unsafeAtomicAdd(&sum[threadIdx.x], s[threadIdx.x][0]);
}

__global__ void k_centroid_finish(const double* __restrict__ sum, int64_t n, float* __restrict__ c) {
  if (threadIdx.x < 3) c[threadIdx.x] = (float)(sum[threadIdx.x] / (double)n);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---- host launchers -----------------------------------------------------------------------------
int grid_bits(int grid) {
  int b = 0;
  while ((1 << b) < grid) ++b;
  return b;
}

hipError_t launch_vox_keys(const float* xyz, int64_t n, int grid, uint32_t* keys, uint32_t* vals,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_vox_key, dim3(blocks_for(n, 256)), dim3(256), 0, s, xyz, n, grid, grid_bits(grid), keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_vox_flags(const uint32_t* keys, int64_t n, uint32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_vox_flag, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys, n, flag);
  return hipGetLastError();
}

hipError_t launch_vox_build(const uint32_t* keys, const uint32_t* order, const uint32_t* flag,
                            const uint32_t* excl, int64_t n, int64_t V, const float* xyz,
                            const float* rgb, int grid, uint32_t* start, int32_t* coords,
                            uint16_t* feat, int32_t* point_voxel, uint32_t* hkeys, int32_t* hvals,
                            int log2cap, int32_t* nbr, hipStream_t s) {
  hipError_t e = launch_fill_u32(hkeys, kEmptyKey, int64_t(1) << log2cap, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vox_start, dim3(blocks_for(n, 256)), dim3(256), 0, s, flag, excl, n, start);
  hipLaunchKernelGGL(k_vox_reduce, dim3(blocks_for(V, 256)), dim3(256), 0, s, keys, order, start, V, n,
                     xyz, rgb, grid, grid_bits(grid), coords, feat, point_voxel, hkeys, hvals, log2cap);
  hipLaunchKernelGGL(k_kernel_map, dim3(blocks_for(V, 256)), dim3(256), 0, s, coords, V, grid, hkeys,
                     hvals, log2cap, nbr);
  return hipGetLastError();
}

// 128 channels enter the decoder's convolutions (skip connections concatenated) and leave their
// data gradients; 128 -> 128 is not needed
bool conv_shape_supported(int cin, int cout) {
  return (cin == 32 || cin == 64 || cin == 128) && (cout == 32 || cout == 64 || cout == 128) &&
         !(cin == 128 && cout == 128);
}

hipError_t launch_subm_conv(const uint16_t* x, int cin, const uint16_t* wt, const float* bias, int cout,
                            const int32_t* nbr, int64_t V, int relu, uint16_t* y, hipStream_t s, int n_off,
                            const uint16_t* x2, int c1) {
  if (V == 0) return hipSuccess;
  if (x2 && (c1 * 2 != cin || c1 % 32 != 0)) return hipErrorInvalidValue;
  // one 16-row MFMA tile per wavefront, four wavefronts per block: 64 voxels per block spread
  // even a coarse UNet level over the chip (four row tiles per wavefront, which share the weight
  // fragments, were slower at every level size measured, 26k to 333k voxels)
  const dim3 grid(blocks_for(V, kConvWaves * 16 * kConvTiles)), block(kConvWaves * kWave);
#define PCS_CONV(CI, CO)                                                                              \
  if (cin == CI && cout == CO && !x2) {                                                               \
    hipLaunchKernelGGL((k_subm_conv<CI, CO, kConvTiles, false>), grid, block, 0, s, x, wt, bias, nbr, V, \
                       relu, y, n_off, nullptr);                                                      \
    return hipGetLastError();                                                                         \
  }
#define PCS_CONV_CAT(CI, CO)                                                                          \
  if (cin == CI && cout == CO && x2) {                                                                \
    hipLaunchKernelGGL((k_subm_conv<CI, CO, kConvTiles, true>), grid, block, 0, s, x, wt, bias, nbr, V,  \
                       relu, y, n_off, x2);                                                           \
    return hipGetLastError();                                                                         \
  }
  PCS_CONV(32, 32) PCS_CONV(32, 64) PCS_CONV(64, 32) PCS_CONV(64, 64) PCS_CONV(128, 32) PCS_CONV(128, 64)
  PCS_CONV(32, 128) PCS_CONV(64, 128)
  PCS_CONV_CAT(64, 32) PCS_CONV_CAT(64, 64) PCS_CONV_CAT(64, 128) PCS_CONV_CAT(128, 32) PCS_CONV_CAT(128, 64)
#undef PCS_CONV_CAT
#undef PCS_CONV
  return hipErrorInvalidValue;
}

hipError_t launch_weight_t(const uint16_t* wt, int n_off, int cin, int cout, bool flip, uint16_t* out,
                           hipStream_t s) {
  const int64_t total = (int64_t)n_off * cin * cout;
  hipLaunchKernelGGL(k_weight_t, dim3(blocks_for(total, 256)), dim3(256), 0, s, wt, n_off, cin, cout,
                     flip ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_voxel_centres(const int32_t* coords, int64_t V, int grid, float* xyz, hipStream_t s) {
  if (V == 0) return hipSuccess;
  hipLaunchKernelGGL(k_voxel_centres, dim3(blocks_for(V, 256)), dim3(256), 0, s, coords, V, grid, xyz);
  return hipGetLastError();
}

hipError_t launch_up_tables(const int32_t* child_coords, const int32_t* parent_of, int64_t Vc, int64_t Vp,
                            int32_t* fwd, int32_t* bwd, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(bwd), 0xFFFFFFFFu, 8 * Vp, s);
  if (e != hipSuccess || Vc == 0) return e;
  hipLaunchKernelGGL(k_up_tables, dim3(blocks_for(Vc, 256)), dim3(256), 0, s, child_coords, parent_of, Vc, Vp,
                     fwd, bwd);
  return hipGetLastError();
}

hipError_t launch_pool_features(const uint32_t* order, const uint32_t* start, int64_t Vp, int64_t Vc,
                                const uint16_t* child, int C, uint16_t* parent, hipStream_t s) {
  if (Vp == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_features, dim3(blocks_for(Vp * (C / 8), 256)), dim3(256), 0, s, order, start, Vp,
                     Vc, child, C, parent);
  return hipGetLastError();
}

hipError_t launch_pool_features_bwd(const int32_t* parent_of, const uint32_t* start, int64_t Vp, int64_t Vc,
                                    const uint16_t* dparent, int C, uint16_t* dchild, hipStream_t s) {
  if (Vc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_features_bwd, dim3(blocks_for(Vc * C, 256)), dim3(256), 0, s, parent_of, start, Vp,
                     Vc, dparent, C, dchild);
  return hipGetLastError();
}

hipError_t launch_relu_mask(const uint16_t* y, const uint16_t* dy, int64_t count, uint16_t* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_relu_mask, dim3(blocks_for(count, 256)), dim3(256), 0, s, y, dy, count, out);
  return hipGetLastError();
}

hipError_t launch_bias_grad(const uint16_t* dy, int64_t V, int cout, float* db, hipStream_t s) {
  if (V == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(512, (V + 255) / 256);
  hipLaunchKernelGGL(k_bias_grad, dim3(blocks), dim3(256), 0, s, dy, V, cout, db);
  return hipGetLastError();
}

hipError_t launch_subm_conv_dw(const uint16_t* x, int cin, const uint16_t* dy, int cout,
                               const int32_t* nbr, int64_t V, float* dw, hipStream_t s, int n_off) {
  if (V == 0) return hipSuccess;
  // ~32 voxel ranges per offset: enough blocks to fill the GPU, few atomics per weight
  const int64_t ranges = std::min<int64_t>(32, (V + 63) / 64);
  const int64_t chunk = ((V + ranges - 1) / ranges + 63) / 64 * 64;
  const dim3 grid((unsigned)((V + chunk - 1) / chunk), (unsigned)n_off), block(256);
#define PCS_CONV_DW(CI, CO)                                                                    \
  if (cin == CI && cout == CO) {                                                               \
    hipLaunchKernelGGL((k_subm_conv_dw<CI, CO>), grid, block, 0, s, x, dy, nbr, V, chunk, dw); \
    return hipGetLastError();                                                                  \
  }
  PCS_CONV_DW(32, 32) PCS_CONV_DW(32, 64) PCS_CONV_DW(64, 32) PCS_CONV_DW(64, 64) PCS_CONV_DW(128, 32)
  PCS_CONV_DW(128, 64) PCS_CONV_DW(32, 128) PCS_CONV_DW(64, 128)
#undef PCS_CONV_DW
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_points(const uint16_t* feat, const int32_t* coords, int64_t V, const int32_t* point_voxel,
                             const float* w1, const float* b1, const float* w2, const float* b2,
                             const float* xyz, const float* rgb, int64_t n, int grid, float* mean, float* quat,
                             float* scale, float* opac, float* out_rgb, float* normal, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_points, dim3(blocks_for(n, 256)), dim3(256), 0, s, feat, coords, V, point_voxel, w1,
                     b1, w2, b2, xyz, rgb, n, grid, mean, quat, scale, opac, out_rgb, normal);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const uint16_t* feat, const int32_t* coords, int64_t V, const int32_t* point_voxel,
                               const uint32_t* order, const uint32_t* start, const float* w1, const float* b1,
                               const float* w2, const float* b2, const float* xyz, int64_t n, int grid,
                               const float* d_mean, const float* d_quat, const float* d_scale,
                               const float* d_opac, const float* d_normal, float* gh, uint16_t* d_feat,
                               float* d_w1, float* d_b1, float* d_w2, float* d_b2, hipStream_t s) {
  if (V == 0 || n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks_for(n, kMlpBwdThreads)), dim3(kMlpBwdThreads), 0, s, feat, coords,
                     V, point_voxel, order, w1, b1, w2, b2, xyz, n, grid, d_mean, d_quat, d_scale, d_opac, d_normal,
                     gh, d_w1, d_b1, d_w2, d_b2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_dfeat, dim3(blocks_for(V, 256)), dim3(256), 0, s, gh, start, V, n, w1, d_feat);
  return hipGetLastError();
}

hipError_t launch_centroid(const float* xyz, int64_t n, double* sum, float* c, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(sum), 0u, 6, s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)std::min<int64_t>(256, (n + 255) / 256);
  if (n > 0) hipLaunchKernelGGL(k_centroid, dim3(blocks), dim3(256), 0, s, xyz, n, sum);
  hipLaunchKernelGGL(k_centroid_finish, dim3(1), dim3(64), 0, s, sum, std::max<int64_t>(n, 1), c);
  return hipGetLastError();
}

hipError_t launch_head_forward(const uint16_t* feat, const float* wh, const float* bh,
                               const int32_t* point_voxel, const float* xyz, const float* rgb,
                               const float* centroid, int64_t n, float voxel, float* quat, float* scale,
                               float* opac, float* out_rgb, float* normal, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_head_forward, dim3(blocks_for(n, 256)), dim3(256), 0, s, feat, wh, bh, point_voxel,
                     xyz, rgb, centroid, n, voxel, quat, scale, opac, out_rgb, normal);
  return hipGetLastError();
}

hipError_t launch_head_backward(const uint16_t* feat, const float* wh, const float* bh,
                                const uint32_t* order, const uint32_t* start, int64_t V, int64_t n,
                                float voxel, const float* d_quat, const float* d_scale,
                                const float* d_opac, const float* d_rgb, uint16_t* d_feat, float* d_wh,
                                float* d_bh, hipStream_t s) {
  if (V == 0) return hipSuccess;
  hipLaunchKernelGGL(k_head_backward, dim3(blocks_for(V, 256)), dim3(256), 0, s, feat, wh, bh, order, start,
                     V, n, voxel, d_quat, d_scale, d_opac, d_rgb, d_feat, d_wh, d_bh);
  return hipGetLastError();
}

}  // namespace pcs
