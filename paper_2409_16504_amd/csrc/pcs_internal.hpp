// Internal declarations shared by the HIP translation units of libpcsplat.so (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pcsplat.h"

namespace pcs {

constexpr int kTile = 16;          // screen tile edge in pixels
constexpr int kTilePixels = kTile * kTile;
constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kRecFloat4 = 4;      // splat record: 4 x float4 = 64 bytes

// Camera as the kernels see it.
struct DevCamera {
  float T[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t W, H;
  int32_t pad[2];
};

struct DevOptions {
  float z_near, lowpass, sigma_cut, alpha_min, alpha_max, t_eps;
  float bg[3];
};

// Splat record written by the projection for every visible (camera, Gaussian), read by
// compositing and its adjoint:
//   r0 = (u, v, opacity, z)   r1 = (A, B, C, ex)   r2 = (r, g, b, ey)   r3 = (nx, ny, nz, 0)
// where (A, B, C) is the conic (inverse screen covariance) and (ex, ey) the padded half extents
// of the bounding box of the sigma_cut ellipse.
// Binning inputs per (camera, Gaussian): the fp32 bits of the depth (0 for a culled splat) and the
// tile rectangle (x0 | x_end << 16, y0 | y_end << 16), ends exclusive (zero for a culled splat).
// When the frame has at most kNarrowRectTiles tile columns and rows, the rectangle is stored in
// one word instead (x0 | x_end << 8 | y0 << 16 | y_end << 24): binning reads the rectangles in
// depth order, one random 4-byte read per splat rather than 8.
constexpr int kNarrowRectTiles = 255;
__device__ __forceinline__ void store_rect(uint2* rect, int64_t i, bool narrow, uint32_t x0,
                                           uint32_t x_end, uint32_t y0, uint32_t y_end) {
  if (narrow)
    reinterpret_cast<uint32_t*>(rect)[i] = x0 | (x_end << 8) | (y0 << 16) | (y_end << 24);
  else
    rect[i] = make_uint2(x0 | (x_end << 16), y0 | (y_end << 16));
}
// The rectangle in its wide form, whichever form it was stored in.
__device__ __forceinline__ uint2 load_rect(const uint2* rect, int64_t i, bool narrow) {
  if (!narrow) return rect[i];
  const uint32_t c = reinterpret_cast<const uint32_t*>(rect)[i];
  return make_uint2((c & 0xFFu) | (((c >> 8) & 0xFFu) << 16), ((c >> 16) & 0xFFu) | ((c >> 24) << 16));
}

// ---- wave64 helpers -------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive prefix sum across the wave (Hillis-Steele with cross-lane shuffles).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t t = __shfl_up(v, o, kWave);
    if (l >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_inclusive_scan64(uint64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint64_t t = __shfl_up(v, o, kWave);
    if (l >= o) v += t;
  }
  return v;
}

// Sum across the wave using row-local DPP shifts and four lane reads; every lane gets the total.
__device__ __forceinline__ float wave_sum(float v) {
  // row_shr:1,2,4,8 within 16-lane rows (bound_ctrl so shifted-in lanes read 0)
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 15));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 31));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 47));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  return (r0 + r1) + (r2 + r3);
}

// Wave-wide sums of 16 per-lane values v[0..15] (padding with zeros is free), left in four lanes:
// lane 16 R + 15 holds in out[j] the sum of v[4 R + j] (R = 0..3). Two lane-half exchanges
// (v_permlane32_swap: the upper 32 lanes of the first operand trade places with the lower 32 of
// the second; v_permlane16_swap: the same for odd and even 16-lane rows) each fold half of the
// values into the other half of the lanes, then row_shr prefix sums finish every row.
__device__ __forceinline__ void wave_sum16_rows(const float (&v)[16], float (&out)[4]) {
  float q[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]),
                                                    false, false);
    q[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);   // lanes 0-31: v[i], 32-63: v[i + 8]
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(q[i]), __float_as_uint(q[i + 4]),
                                                    false, false);
    float x = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // row R: v[4 R + i]
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xF, 0xF, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x112, 0xF, 0xF, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xF, 0xF, true));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xF, 0xF, true));
    out[i] = x;
  }
}

// Bits of a frame's error word (device, one per render state): a look-back that waited too long
// (a broken launch), and more tile instances than a fixed capacity holds. Kernels that consume the
// failed stage's output return at once.
constexpr uint32_t kErrSpin = 1u;
constexpr uint32_t kErrCapacity = 2u;

// Zeroing folded into a kernel that runs anyway: every thread of the grid clears the words
// i = its global index, + the grid size, ... of each span (a span of count 0 is skipped).
struct ClearSpans {
  uint32_t* p[3] = {nullptr, nullptr, nullptr};
  int64_t count[3] = {0, 0, 0};
};
__device__ __forceinline__ void clear_spans(const ClearSpans& c, int64_t gid, int64_t gsize) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
    for (int64_t i = gid; i < c.count[k]; i += gsize) c.p[k][i] = 0u;
}

// Late-shading parameters on the device: unit direction towards the light, light colour,
// Blinn-Phong coefficients, background colour.
struct DevLight {
  float dir[3], color[3];
  float ambient, diffuse, specular, shininess;
  float bg[3];
};

// ---- launchers (stream-ordered, return the launch error) ------------------------------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float value, int64_t n, hipStream_t s);

// Depth-bit range slots: zrange[0..kZSlots) minima, zrange[kZSlots..2 kZSlots) maxima.
constexpr int kZSlots = 64;
// small[0..1] a u64 total written by the scan, small[2..2+2 kZSlots) depth-bit range slots,
// small[kCountWord..) kZSlots u64 partial instance counts, small[kDepthWord..+3) the depth sort's
// pass count, depth bits and minimum depth bits (written on the device). The range slots and
// counts (kSlotWords from word 2) are reset for the next frame by the frame's tile-order kernel,
// after their only reader, or by launch_init_small.
constexpr int kCountWord = 2 + 2 * kZSlots;
constexpr int kDepthWord = kCountWord + 2 * kZSlots;
constexpr int kVoxErrWord = kDepthWord + 3;   // error word of a voxelisation
constexpr int kSmallWords = kDepthWord + 4;
constexpr int kSlotWords = kDepthWord - 2;
// Cameras travel to the device as kernel arguments, kArgCams per launch.
constexpr int kArgCams = 8;
struct CamBatch {
  DevCamera c[kArgCams];
};
// Resets the frame's error word (err, may be null) and, when small is set, the instance total and
// the projection slots; writes the batch of up to kArgCams cameras into dst. Needed only where the
// frame cannot do this itself: more than kArgCams cameras, no Gaussians, or slots whose last
// frame did not reach its tile order.
hipError_t launch_init_small(uint32_t* small, const DevCamera* cams, int n_cams, DevCamera* dst,
                             hipStream_t s, uint32_t* err = nullptr);
// zrange / count_slots: the projection slots (reset beforehand). arg_cams (may be null; else
// n_cams <= kArgCams): the cameras as kernel arguments, which the projection reads instead of
// cams and also writes to cams for the later kernels. err, total (may be null): the frame's error
// word and the instance total, reset (nothing in the frame writes them before the projection ends).
hipError_t launch_project(int64_t n, int n_cams, DevCamera* cams, const DevOptions& opt,
                          const pcs_gaussians& g, float4* rec, uint32_t* zbits, uint2* rect,
                          bool narrow_rect, uint32_t* zrange, unsigned long long* count_slots,
                          const ClearSpans& clear, hipStream_t s, const CamBatch* arg_cams = nullptr,
                          uint32_t* err = nullptr, uint64_t* total = nullptr);

// Exclusive scan of n u32 values in[gather[j]] (no gather: in[j]); writes out[n] and *total (u64).
// gather is gather1 when sel is set and *sel is odd, else gather0. Scratch from scan_scratch_bytes.
size_t scan_scratch_bytes(int64_t n);
// err (may be null): set to kErrSpin if a look-back wait runs out its bound (spin_limit rounds,
// 0 = the default).
hipError_t launch_scan(const uint32_t* in, const uint32_t* gather0, const uint32_t* gather1,
                       const uint32_t* sel, uint32_t* out, int64_t n, uint64_t* total, void* scratch,
                       hipStream_t s, bool scratch_cleared = false, uint32_t* err = nullptr,
                       uint32_t spin_limit = 0);
// Words of scan scratch that must be zero before a scan of n values.
int64_t scan_clear_words(int64_t n);

// Depth key per (camera, Gaussian) entry and its index as the value, and the keys' four digit
// histograms into hist_copies (kTileHistWords, kTileHistCopies partial copies, zeroed beforehand),
// for a launch_sort with them as ext_hist. The depth-bit range comes from the projection's slots on the device; info[0..3)
// receives the pass count, depth bits and minimum depth bits. The sum of the projection's
// kZSlots count slots goes to host_word[0] (pinned, coherent host memory) as seq << 32 | total,
// the total capped at 2^32 - 1, and the depth bits to host_word[1] as seq << 32 | bits.
hipError_t launch_depth_keys_hist(int64_t m, const uint32_t* zbits,
                                  const unsigned long long* count_slots,
                                  unsigned long long* host_word, uint32_t seq, const uint32_t* zrange,
                                  uint32_t* info, uint32_t* keys, uint32_t* vals, uint32_t* hist_copies,
                                  hipStream_t s);

// Tile-digit histograms counted by binning: kTileHistCopies partial copies of
// [kTileHistPasses][256] counters, summed by the tile sort.
constexpr int kTileHistCopies = 32;
constexpr int kTileHistPasses = 4;
constexpr int64_t kTileHistWords = (int64_t)kTileHistCopies * kTileHistPasses * 256;

// Binning fused with the prefix sum of the tile counts in depth order: the (camera, Gaussian)
// entries in the depth order (order1 when *passes is odd, where the depth sort ended, else
// order0) get their offsets from a decoupled look-back scan, and every block then writes its
// entries' tile keys (global tile ids, row-major within a rectangle) and Gaussian indices at
// those offsets, counting the keys' 8-bit digits into hist (kTileHistWords, zeroed beforehand)
// for the tile sort (launch_sort with ext_hist). scan_scratch must be cleared (scan_clear_words);
// *total receives the instance count. rect holds the rectangles in their narrow form when
// narrow_rect is set (store_rect).
// err: the frame's error word (binning returns at once if it is set; a look-back that waits
// more than spin_limit rounds, 0 = the default bound, sets kErrSpin and goes on). capacity: keys
// and values are written only below it (more instances set kErrCapacity; *total still receives
// the full count).
hipError_t launch_scan_binning(int64_t n, int n_cams, int TX, int64_t tiles_per_cam,
                               const uint32_t* order0, const uint32_t* order1,
                               const uint32_t* passes, const uint2* rect, bool narrow_rect,
                               void* scan_scratch, uint64_t* total, uint32_t* keys, uint32_t* vals,
                               int tile_bits,
                               uint32_t* hist, const ClearSpans& clear, hipStream_t s, uint32_t* err,
                               uint32_t spin_limit, uint64_t capacity);

// Stable LSD radix sort of (key, value) pairs over key bits [0, bits), K = uint32_t or uint64_t;
// keys must have no bit set at or above `bits` (the ranking skips those bits).
// Ping-pongs between (k0,v0) and (k1,v1); returns in *result_in_alt whether the sorted data ended
// in (k1,v1).
size_t sort_scratch_bytes(int64_t m);
// live_passes (device, may be null): passes at or beyond *live_passes return at once, so the data
// ends in (k1,v1) when *live_passes is odd; *result_in_alt then describes the host's pass count.
// [pass_begin, pass_end) launches only those passes (pass_end < 0: all): a sort may be launched in
// pieces on one stream, the set-up (clear, histogram) going with the piece that starts at pass 0.
// ranges (32-bit keys below n_tiles, zeroed beforehand): the last pass also records every key's
// run as ranges[key] = ~start, ranges[n_tiles + key] = end (launch_tile_order turns the starts
// back into plain ones).
// err (may be null): the passes return at once if it is set, and a look-back that waits more than
// spin_limit rounds (0 = the default bound) sets kErrSpin. m_dev (may be null): the element count
// is read on the device (at most m, which then sizes the launch). wide (32-bit keys): scatter
// partitions run as 1024 threads x 4 keys instead of 512 x 8 (same partitions, same result; faster
// for the depth sort of a frame's splats, slower for the tile sort of its instances).
template <typename K>
hipError_t launch_sort(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t m, int bits, void* scratch,
                       hipStream_t s, bool* result_in_alt, const uint32_t* live_passes = nullptr,
                       bool scratch_cleared = false, bool hist_ready = false,
                       const uint32_t* ext_hist = nullptr, int pass_begin = 0, int pass_end = -1,
                       uint32_t* ranges = nullptr, int64_t n_tiles = 0, uint32_t* err = nullptr,
                       uint32_t spin_limit = 0, const uint64_t* m_dev = nullptr, bool wide = false);
// Words at the start of sort scratch that must be zero before a sort of m pairs (cleared by the
// sort itself unless the caller has cleared them and says so).
int64_t sort_clear_words(int64_t m);

// ranges must be zero (cleared by the caller, e.g. folded into binning); starts are written
// complemented, like the sort's (launch_tile_order turns them back).
hipError_t launch_ranges(const uint32_t* keys, int64_t m, int64_t n_tiles, uint32_t* ranges,
                         hipStream_t s, const uint64_t* m_dev = nullptr, const uint32_t* err = nullptr);

// Permutation of the tiles for compositing: longest lists first, empty tiles last. Reads the
// complemented starts and leaves plain ones. report (pinned host memory, may be null) receives
// seq << 32 | the frame's error word; if that word is set, every tile's run is left empty instead
// (the order is then the identity), so that compositing and its adjoint read nothing the failed
// stage produced.
// slots (may be null): the projection slots (kSlotWords words), reset for the next frame.
hipError_t launch_tile_order(uint32_t* ranges, int64_t n_tiles, uint32_t* order, hipStream_t s,
                             const uint32_t* err = nullptr, unsigned long long* report = nullptr,
                             uint32_t seq = 0, uint32_t* slots = nullptr);

hipError_t launch_canonical_keys(const uint32_t* keys, const uint32_t* vals, int64_t m, int64_t n,
                                 int64_t tiles_per_cam, const float4* rec, uint64_t* out,
                                 hipStream_t s);

// ev_start / ev_stop, when given, receive the compositing kernel's own start and end times.
hipError_t launch_composite(int64_t n, int n_cams, int W, int H, const float4* rec,
                            const uint32_t* vals, const uint32_t* ranges, const uint32_t* order,
                            const DevOptions& opt, const pcs_images& out, float* t_final,
                            int32_t* n_contrib, hipStream_t s, hipEvent_t ev_start = nullptr,
                            hipEvent_t ev_stop = nullptr);

// Backward: per-(camera, Gaussian) screen-space gradient accumulators, [C*n][16] (one 64-byte
// line per splat, so a splat's partials from one wavefront go out as one atomic request):
// u, v, A, B, C, opacity, depth, r, g, b, nx, ny, nz, three unused.
constexpr int kScreenGrads = 13;
constexpr int kScreenStride = 16;
hipError_t launch_composite_backward(int64_t n, int n_cams, int W, int H, const float4* rec,
                                     const uint32_t* vals, const uint32_t* ranges,
                                     const uint32_t* order, const DevOptions& opt, const float* t_final,
                                     const int32_t* n_contrib, const pcs_images& grad_out,
                                     float* sgrad, hipStream_t s);
hipError_t launch_project_backward(int64_t n, int n_cams, const DevCamera* cams,
                                   const DevOptions& opt, const pcs_gaussians& g,
                                   const float* sgrad, const pcs_grads& grads, hipStream_t s);

// Synchronises the stream once (bounding box readback through host_pinned, >= 24 bytes).
hipError_t launch_knn_pca(const float* xyz, int64_t n, int k, float kappa, float floor_ratio,
                          float* quat, float* scale, float* normal, float* nn_dist, void* scratch,
                          size_t scratch_bytes, uint32_t* host_pinned, hipStream_t s);
size_t knn_scratch_bytes(int64_t n);

// ---- sparse estimator ---------------------------------------------------------------------------
// log2 of a power-of-two grid: the width of each coordinate field of a voxel key
int grid_bits(int grid);
hipError_t launch_vox_keys(const float* xyz, int64_t n, int grid, uint32_t* keys, uint32_t* vals,
                           hipStream_t s);
hipError_t launch_vox_flags(const uint32_t* keys, int64_t n, uint32_t* flag, hipStream_t s);
hipError_t launch_vox_build(const uint32_t* keys, const uint32_t* order, const uint32_t* flag,
                            const uint32_t* excl, int64_t n, int64_t V, const float* xyz,
                            const float* rgb, int grid, uint32_t* start, int32_t* coords,
                            uint16_t* feat, int32_t* point_voxel, uint32_t* hkeys, int32_t* hvals,
                            int log2cap, int32_t* nbr, hipStream_t s);
bool conv_shape_supported(int cin, int cout);
// y = relu?(bias + sum over n_off offsets of W_k x[nbr_k]): 27 offsets for the submanifold
// convolution, 8 for the transposed stride-2 convolution (with its upsampling table). x2 (may be
// null): the input is [x | x2] along the channels in equal halves, x[V][c1] and x2[V][c1] with
// c1 = cin / 2 a multiple of 32 (hipErrorInvalidValue otherwise).
hipError_t launch_subm_conv(const uint16_t* x, int cin, const uint16_t* wt, const float* bias, int cout,
                            const int32_t* nbr, int64_t V, int relu, uint16_t* y, hipStream_t s,
                            int n_off = 27, const uint16_t* x2 = nullptr, int c1 = 0);
// out[s][c][o] = wt[flip ? n_off - 1 - s : s][o][c]
hipError_t launch_weight_t(const uint16_t* wt, int n_off, int cin, int cout, bool flip, uint16_t* out,
                           hipStream_t s);
hipError_t launch_voxel_centres(const int32_t* coords, int64_t V, int grid, float* xyz, hipStream_t s);
hipError_t launch_up_tables(const int32_t* child_coords, const int32_t* parent_of, int64_t Vc, int64_t Vp,
                            int32_t* fwd, int32_t* bwd, hipStream_t s);
hipError_t launch_pool_features(const uint32_t* order, const uint32_t* start, int64_t Vp, int64_t Vc,
                                const uint16_t* child, int C, uint16_t* parent, hipStream_t s);
hipError_t launch_pool_features_bwd(const int32_t* parent_of, const uint32_t* start, int64_t Vp, int64_t Vc,
                                    const uint16_t* dparent, int C, uint16_t* dchild, hipStream_t s);
hipError_t launch_mlp_points(const uint16_t* feat, const int32_t* coords, int64_t V, const int32_t* point_voxel,
                             const float* w1, const float* b1, const float* w2, const float* b2,
                             const float* xyz, const float* rgb, int64_t n, int grid, float* mean, float* quat,
                             float* scale, float* opac, float* out_rgb, float* normal, hipStream_t s);
hipError_t launch_mlp_backward(const uint16_t* feat, const int32_t* coords, int64_t V, const int32_t* point_voxel,
                               const uint32_t* order, const uint32_t* start, const float* w1, const float* b1,
                               const float* w2, const float* b2, const float* xyz, int64_t n, int grid,
                               const float* d_mean, const float* d_quat, const float* d_scale,
                               const float* d_opac, const float* d_normal, float* gh, uint16_t* d_feat,
                               float* d_w1, float* d_b1, float* d_w2, float* d_b2, hipStream_t s);
hipError_t launch_relu_mask(const uint16_t* y, const uint16_t* dy, int64_t count, uint16_t* out,
                            hipStream_t s);
hipError_t launch_bias_grad(const uint16_t* dy, int64_t V, int cout, float* db, hipStream_t s);
hipError_t launch_subm_conv_dw(const uint16_t* x, int cin, const uint16_t* dy, int cout,
                               const int32_t* nbr, int64_t V, float* dw, hipStream_t s, int n_off = 27);
hipError_t launch_centroid(const float* xyz, int64_t n, double* sum, float* c, hipStream_t s);
hipError_t launch_head_forward(const uint16_t* feat, const float* wh, const float* bh,
                               const int32_t* point_voxel, const float* xyz, const float* rgb,
                               const float* centroid, int64_t n, float voxel, float* quat,
                               float* scale, float* opac, float* out_rgb, float* normal, hipStream_t s);
hipError_t launch_head_backward(const uint16_t* feat, const float* wh, const float* bh,
                                const uint32_t* order, const uint32_t* start, int64_t V, int64_t n,
                                float voxel, const float* d_quat, const float* d_scale,
                                const float* d_opac, const float* d_rgb, uint16_t* d_feat, float* d_wh,
                                float* d_bh, hipStream_t s);

// Late shading of rendered frames: out[C][3][H][W] from rgb/normal [C][3][H][W], alpha [C][H][W].
hipError_t launch_shade(int W, int H, int n_cams, const DevCamera* cams, const float* rgb,
                        const float* nrm, const float* alpha, const DevLight& L, float* out,
                        hipStream_t s);

// LDS read-bandwidth probe: `blocks` blocks each reading 16-byte LDS words; lds_probe_bytes gives
// the bytes read. sink: blocks * 256 floats (never written in practice).
hipError_t launch_lds_probe(int blocks, int iters, float* sink, hipStream_t s);
int64_t lds_probe_bytes(int blocks, int iters);

}  // namespace pcs
