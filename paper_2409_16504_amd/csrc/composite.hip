// Per-tile front-to-back compositing (Section 3.1, Eq. 1-2) and its adjoint.
//
// Forward: one single-wavefront block per 8x8 quadrant of a 16x16 screen tile, tiles taken longest
// list first. The wavefront streams the tile's depth-sorted list in batches of 64 records (one per
// lane, the next batch fetched into registers while the current one is composited), keeps the
// records whose ellipse bounding box reaches its quadrant, compacted into LDS in list order, and
// walks them: every pixel tests the 3-sigma ellipse, evaluates alpha = o * exp(-q/2), and blends
// RGB, normal and depth until its transmittance drops below t_eps. Records are kept only if their
// box reaches the rectangle of the quadrant's pixels that are still blending, which shrinks as
// pixels finish. The quadrants of a tile run independently, so none waits for another and each
// stops as soon as its own pixels are done.
//
// The adjoint uses the same quadrant wavefronts and walks the list back to front from the
// quadrant's furthest last contributor, recovering each pixel's transmittance by division, keeps a
// running sum of what lies behind each splat, and reduces each splat's 13 screen-space partials
// across the wavefront (lane-half exchanges leave them in four lanes) before one atomic add per
// value.

#include <hip/hip_ext.h>

#include "projection.hpp"

namespace pcs {

namespace {

constexpr int kGroup = 4;             // reaching splats whose quadratic forms are evaluated together
constexpr float kNegHalfLog2e = -0.72134752044448170f;   // -log2(e) / 2

// Pixel of a thread: wavefront w owns the 8x8 quadrant (w & 1, w >> 1) of the 16x16 tile.
struct TilePixel {
  int x, y;             // pixel
  float qx0, qy0;       // centre of the quadrant's first pixel
};

__device__ __forceinline__ TilePixel tile_pixel(int tx, int ty, int tid) {
  const int wave = tid / kWave, lane = tid % kWave;
  TilePixel p;
  const int bx = tx * kTile + (wave & 1) * 8, by = ty * kTile + (wave >> 1) * 8;
  p.x = bx + (lane & 7);
  p.y = by + (lane >> 3);
  p.qx0 = (float)bx + 0.5f;
  p.qy0 = (float)by + 0.5f;
  return p;
}

// Block b of the forward pass composites quadrant (b / 8) % 4 of the tile at position
// (b / 32) * 8 + b % 8 of the order: the four quadrants of a tile are blocks b, b + 8, b + 16,
// b + 24, which the dispatcher deals to the same XCD (blocks go round-robin over the 8 XCDs), so
// they share the tile's records in one L2. Returns false for positions past the last tile.
__device__ __forceinline__ bool quadrant_of_block(int64_t b, int64_t total_tiles, int64_t& pos,
                                                  int& quad) {
  pos = (b / 32) * 8 + b % 8;
  quad = (int)((b / 8) % 4);
  return pos < total_tiles;
}

// Bounding rectangle (pixel centres) of the lanes set in an 8x8 quadrant's lane mask.
struct ActiveRect {
  float x0, x1, y0, y1;
};

__device__ __forceinline__ ActiveRect active_rect(uint64_t live, float qx0, float qy0) {
  uint64_t cols = live | (live >> 32);
  cols |= cols >> 16;
  cols |= cols >> 8;
  const uint32_t colmask = (uint32_t)cols & 0xFFu;
  uint64_t rows = live | (live >> 4);
  rows |= rows >> 2;
  rows |= rows >> 1;
  rows &= 0x0101010101010101ull;                      // bit 8 r set: row r has a live lane
  ActiveRect r;
  r.x0 = qx0 + (float)__builtin_ctz(colmask);
  r.x1 = qx0 + (float)(31 - __builtin_clz(colmask));
  r.y0 = qy0 + (float)(__builtin_ctzll(rows) >> 3);
  r.y1 = qy0 + (float)((63 - __builtin_clzll(rows)) >> 3);
  return r;
}

// Does the splat's padded ellipse bounding box reach a pixel centre of the rectangle?
__device__ __forceinline__ bool touches_rect(float u, float v, float ex, float ey, const ActiveRect& r) {
  const float gx = fmaxf(fmaxf(r.x0 - u, u - r.x1), 0.0f);
  const float gy = fmaxf(fmaxf(r.y0 - v, v - r.y1), 0.0f);
  return gx <= ex && gy <= ey;
}

// Blend-order form of a record, written by the lane that keeps it:
//   f0 = (u, v, k A, 2 k B)   f1 = (k C, log2 o, thr, z)   f2 = (r, g, b, list position + 1)
//   f3 = (nx, ny, nz, 0)
// with k = -log2(e) / 2, so that s = k q comes out of the quadratic form directly and
// alpha = o e^(-q/2) = 2^(s + log2 o). thr = max(k sigma_cut^2, log2 alpha_min - log2 o): s >= thr
// is the 3-sigma test (q <= sigma_cut^2) and the alpha cut-off together (alpha_max >= alpha_min).
// For o = 0 the difference is NaN or +inf and fmaxf leaves the 3-sigma test or never, as the
// sequential test would (a zero-alpha blend counts only when alpha_min = 0).
__device__ __forceinline__ void blend_form(const float4& r0, const float4& r1, const float4& r2,
                                           const float4& r3, int32_t pos, float k_cut2, float l2amin,
                                           float4& f0, float4& f1, float4& f2, float4& f3) {
  const float l2o = __log2f(r0.z);
  f0 = make_float4(r0.x, r0.y, kNegHalfLog2e * r1.x, (2.0f * kNegHalfLog2e) * r1.y);
  f1 = make_float4(kNegHalfLog2e * r1.z, l2o, fmaxf(k_cut2, l2amin - l2o), r0.w);
  f2 = make_float4(r2.x, r2.y, r2.z, __int_as_float(pos));
  f3 = make_float4(r3.x, r3.y, r3.z, 0.0f);
}

// k q of a blend form at the pixel centre (px, py), with the offsets it used. Compositing and its
// adjoint evaluate this same operation sequence, so they take the same blend decisions.
__device__ __forceinline__ float blend_kq(const float4& f0, const float4& f1, float px, float py,
                                          float& dx, float& dy) {
  dx = px - f0.x;
  dy = py - f0.y;
  return fmaf(dx, fmaf(f0.z, dx, f0.w * dy), (f1.x * dy) * dy);
}

__global__ __launch_bounds__(kWave) void k_composite(
    int64_t n, int W, int H, int TX, int64_t tiles_per_cam, int64_t total_tiles,
    const float4* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, DevOptions opt,
    float* __restrict__ out_rgb,
    float* __restrict__ out_nrm, float* __restrict__ out_depth, float* __restrict__ out_alpha,
    float* __restrict__ t_final, int32_t* __restrict__ n_contrib) {
  // blend forms of a batch's kept records, plus kGroup slots past the last one whose threshold
  // is NaN
  __shared__ float4 s_f0[kWave + kGroup], s_f1[kWave + kGroup], s_f2[kWave + kGroup], s_f3[kWave + kGroup];
  int64_t opos;
  int quad;
  if (!quadrant_of_block(blockIdx.x, total_tiles, opos, quad)) return;
  const int64_t tile = order[opos];         // longest lists first
  const int64_t cam = tile / tiles_per_cam;
  const int64_t t = tile - cam * tiles_per_cam;
  const int tx = (int)(t % TX), ty = (int)(t / TX);
  const int lane = threadIdx.x;
  const TilePixel P = tile_pixel(tx, ty, quad * kWave + lane);
  const bool inside = P.x < W && P.y < H;
  const float pxf = (float)P.x + 0.5f, pyf = (float)P.y + 0.5f;
  const uint32_t start = ranges[tile], end = ranges[total_tiles + tile];
  const float k_cut2 = kNegHalfLog2e * (opt.sigma_cut * opt.sigma_cut);
  const float amax = fmaxf(opt.alpha_max, opt.alpha_max);    // canonical once, not per use
  // alpha_max below alpha_min: no alpha passes the cut-off
  const float l2amin = opt.alpha_max < opt.alpha_min ? __builtin_inff() : __log2f(opt.alpha_min);
  const float4* rec_cam = rec + cam * n * kRecFloat4;
  const uint64_t lt = lanemask_lt();
  // A pixel blends while T >= t_eps (t_eps <= 1, so it starts blending): the blend that takes T
  // below t_eps is its last, and after it T, the sums and the last contributor stay as they are.
  // Pixels outside the image start at T = 0 and never blend.
  float T = inside ? 1.0f : 0.0f;
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f, acc4 = 0.f, acc5 = 0.f, acc6 = 0.f;
  int32_t last = 0;
  // one record per lane; the next batch's records and the batch after's splat indices travel in
  // registers while the current batch is composited, so each batch waits on one round trip. The
  // loads are unconditional (positions past the list re-read its last entry; the position test
  // below drops them), which keeps the prefetched values in registers.
  // every slot starts finite (zeros), so a slot after the last kept record, read with zero
  // weight, leaves the sums exact
  {
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    s_f0[lane] = z4; s_f2[lane] = z4; s_f3[lane] = z4;
    if (lane < kGroup) { s_f0[kWave + lane] = z4; s_f2[kWave + lane] = z4; s_f3[kWave + lane] = z4; }
  }
  const uint32_t lastpos = end > start ? end - 1 : start;
  float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0, p2 = p0, p3 = p0;
  uint32_t vnext = 0;
  if (end > start) {
    const float4* r = rec_cam + (int64_t)min(vals[min(start + lane, lastpos)], (uint32_t)(n - 1)) * kRecFloat4;
    p0 = r[0]; p1 = r[1]; p2 = r[2]; p3 = r[3];
    vnext = vals[min(start + kWave + lane, lastpos)];
  }
  for (uint32_t b = start; b < end; b += kWave) {
    const uint64_t live = __ballot(T >= opt.t_eps);
    if (live == 0ull) break;                          // every pixel of the quadrant is done
    // keep the records whose padded ellipse box reaches a pixel that is still blending, compacted
    // in list order; the live pixels' bounding rectangle comes from the stop mask (lane = 8 y + x):
    // rows are its non-zero bytes, columns the OR of its bytes
    const ActiveRect ar = active_rect(live, P.qx0, P.qy0);
    const bool rel = b + lane < end && touches_rect(p0.x, p0.y, p1.w, p2.w, ar);
    const uint64_t relmask = __ballot(rel);
    if (rel) {
      const int slot = __popcll(relmask & lt);
      float4 f0, f1, f2, f3;
      blend_form(p0, p1, p2, p3, (int32_t)(b - start) + lane + 1, k_cut2, l2amin, f0, f1, f2, f3);
      s_f0[slot] = f0; s_f1[slot] = f1; s_f2[slot] = f2; s_f3[slot] = f3;
    }
    // the kGroup slots after the last kept record can never blend (NaN threshold: s >= thr
    // fails); their other fields are finite (earlier records or the initial zeros)
    if (lane < kGroup) s_f1[__popcll(relmask) + lane] = make_float4(0.f, 0.f, __int_as_float(0x7fc00000), 0.f);
    {
      const float4* r = rec_cam + (int64_t)min(vnext, (uint32_t)(n - 1)) * kRecFloat4;
      p0 = r[0]; p1 = r[1]; p2 = r[2]; p3 = r[3];
      vnext = vals[min(b + 2 * kWave + lane, lastpos)];
    }
    __syncthreads();                                  // one wavefront: orders the LDS writes
    const int nrel = __popcll(relmask);
    for (int k0 = 0; k0 < nrel; k0 += kGroup) {
      // the group's alphas first: they do not depend on T, so the in-order blends below run
      // from registers
      float aa[kGroup];
      float4 c2[kGroup], c3[kGroup];
      float zz[kGroup];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const int k = k0 + j;
        const float4 f0 = s_f0[k];
        const float4 f1 = s_f1[k];
        c2[j] = s_f2[k];
        c3[j] = s_f3[k];
        zz[j] = f1.w;
        float dx, dy;
        const float sq = blend_kq(f0, f1, pxf, pyf, dx, dy);
        const float a = fminf(amax, __builtin_amdgcn_exp2f(sq + f1.y));
        aa[j] = sq >= f1.z ? a : -0.0f;               // -0: no blend, and w = -0 says so
      }
      // blends in list order without branches: a record that does not blend, or a pixel that
      // has stopped, gives w = -0, which leaves T and the sums as they are; w >= +0 marks a blend
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const float a = aa[j];
        const bool go = T >= opt.t_eps;
        const float w = go ? a * T : -0.0f;
        acc0 = fmaf(w, c2[j].x, acc0);
        acc1 = fmaf(w, c2[j].y, acc1);
        acc2 = fmaf(w, c2[j].z, acc2);
        acc3 = fmaf(w, c3[j].x, acc3);
        acc4 = fmaf(w, c3[j].y, acc4);
        acc5 = fmaf(w, c3[j].z, acc5);
        acc6 = fmaf(w, zz[j], acc6);
        T = go ? T * (1.0f - a) : T;
        const bool blended = __builtin_amdgcn_classf(w, 0x3C0);   // +0, +denormal, +normal, +inf
        last = blended ? __float_as_int(c2[j].w) : last;
      }
    }
    __syncthreads();                                  // reads done before the next batch lands
  }
  if (!inside) return;
  const int64_t HW = (int64_t)W * H;
  const int64_t pix = (int64_t)P.y * W + P.x;
  const int64_t c3 = cam * 3 * HW;
  out_rgb[c3 + pix] = acc0 + T * opt.bg[0];
  out_rgb[c3 + HW + pix] = acc1 + T * opt.bg[1];
  out_rgb[c3 + 2 * HW + pix] = acc2 + T * opt.bg[2];
  if (out_nrm) {
    out_nrm[c3 + pix] = acc3;
    out_nrm[c3 + HW + pix] = acc4;
    out_nrm[c3 + 2 * HW + pix] = acc5;
  }
  if (out_depth) out_depth[cam * HW + pix] = acc6;
  if (out_alpha) out_alpha[cam * HW + pix] = 1.0f - T;
  if (t_final) t_final[cam * HW + pix] = T;
  if (n_contrib) n_contrib[cam * HW + pix] = last;
}

__global__ __launch_bounds__(kWave) void k_composite_bwd(
    int64_t n, int W, int H, int TX, int64_t tiles_per_cam, int64_t total_tiles,
    const float4* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, DevOptions opt,
    const float* __restrict__ t_final,
    const int32_t* __restrict__ n_contrib, const float* __restrict__ g_rgb,
    const float* __restrict__ g_nrm, const float* __restrict__ g_depth,
    const float* __restrict__ g_alpha, float* __restrict__ sgrad) {
  __shared__ float4 s_f0[kWave], s_f1[kWave], s_f2[kWave], s_f3[kWave];   // blend forms
  __shared__ uint32_t s_g[kWave];
  int64_t opos;
  int quad;
  if (!quadrant_of_block(blockIdx.x, total_tiles, opos, quad)) return;
  const int64_t tile = order[opos];         // longest lists first
  const int64_t cam = tile / tiles_per_cam;
  const int64_t t = tile - cam * tiles_per_cam;
  const int tx = (int)(t % TX), ty = (int)(t / TX);
  const int lane = threadIdx.x;
  const TilePixel P = tile_pixel(tx, ty, quad * kWave + lane);
  const bool inside = P.x < W && P.y < H;
  const float pxf = (float)P.x + 0.5f, pyf = (float)P.y + 0.5f;
  const uint32_t start = ranges[tile];
  const float k_cut2 = kNegHalfLog2e * (opt.sigma_cut * opt.sigma_cut);
  const float amax = fmaxf(opt.alpha_max, opt.alpha_max);
  const float l2amin = opt.alpha_max < opt.alpha_min ? __builtin_inff() : __log2f(opt.alpha_min);
  // the conic's gradients from k-scaled entries: d/du of q = -2 (A dx + B dy) = (-2 / k) (k A dx + k B dy)
  constexpr float kM2OverK = -2.0f / kNegHalfLog2e;
  const float4* rec_cam = rec + cam * n * kRecFloat4;
  const int64_t HW = (int64_t)W * H;
  const int64_t pix = (int64_t)P.y * W + P.x;
  const uint64_t lt = lanemask_lt();
  float T = 1.0f;
  int32_t nc = 0;
  float g[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float g_cover = 0.f;                      // upstream gradient of the alpha output 1 - T_final
  if (inside) {
    T = t_final[cam * HW + pix];
    nc = n_contrib[cam * HW + pix];
    const int64_t c3 = cam * 3 * HW;
    if (g_rgb) { g[0] = g_rgb[c3 + pix]; g[1] = g_rgb[c3 + HW + pix]; g[2] = g_rgb[c3 + 2 * HW + pix]; }
    if (g_nrm) { g[3] = g_nrm[c3 + pix]; g[4] = g_nrm[c3 + HW + pix]; g[5] = g_nrm[c3 + 2 * HW + pix]; }
    if (g_depth) g[6] = g_depth[cam * HW + pix];
    if (g_alpha) g_cover = g_alpha[cam * HW + pix];
  }
  // g . (what lies behind the current splat), with behind = sum_{j>k} T_j a_j f_j + T_final * bg:
  // g is fixed along the walk, so the seven-channel sum enters only through this dot product. The
  // alpha output 1 - T_final adds -g_alpha T_final to it: like the background term, it scales with
  // T_final, whose derivative in alpha_k is -T_final / (1 - alpha_k).
  float gb = T * (fmaf(g[0], opt.bg[0], fmaf(g[1], opt.bg[1], g[2] * opt.bg[2])) - g_cover);
  // the quadrant's furthest last contributor bounds the walk
  int32_t max_nc = nc;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) max_nc = max(max_nc, __shfl_xor(max_nc, o, kWave));
  const int64_t base_idx = cam * n;
  // batches of 64 list positions, back to front; the batch below is fetched into registers while
  // the current one is walked
  // unconditional loads (positions past the batch re-read its last entry; the position test drops
  // them), which keeps the prefetched values in registers
  float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0, p2 = p0, p3 = p0;
  uint32_t pg_idx = 0;
  auto fetch = [&](int32_t bstart, int32_t bend) {
    const int32_t pos = min(bstart + lane, bend - 1);
    pg_idx = min(vals[start + pos], (uint32_t)(n - 1));
    const float4* r = rec_cam + (int64_t)pg_idx * kRecFloat4;
    p0 = r[0]; p1 = r[1]; p2 = r[2]; p3 = r[3];
  };
  if (max_nc > 0) fetch(max(0, max_nc - kWave), max_nc);
  for (int32_t bend = max_nc; bend > 0; bend -= kWave) {
    const int32_t bstart = max(0, bend - kWave);
    // pixels whose last contributor lies past the batch start are the only ones it can touch;
    // keep the records whose padded box reaches their rectangle
    const uint64_t live = __ballot(nc > bstart);
    const ActiveRect ar = active_rect(live, P.qx0, P.qy0);
    const bool rel = bstart + lane < bend && touches_rect(p0.x, p0.y, p1.w, p2.w, ar);
    const uint64_t relmask = __ballot(rel);
    if (rel) {
      const int slot = __popcll(relmask & lt);
      float4 f0, f1, f2, f3;
      blend_form(p0, p1, p2, p3, bstart + lane, k_cut2, l2amin, f0, f1, f2, f3);   // position from 0
      s_f0[slot] = f0; s_f1[slot] = f1; s_f2[slot] = f2; s_f3[slot] = f3;
      s_g[slot] = pg_idx;
    }
    if (bstart > 0) fetch(max(0, bstart - kWave), bstart);
    __syncthreads();                                  // one wavefront: orders the LDS writes
    // groups of kGroup kept records, back to front: first every record's blend decision, alpha and
    // 1 / (1 - alpha) (they do not depend on T), then the in-order steps, which select instead of
    // branching (a record that did not blend at this pixel leaves T, gb and its partials at zero)
    const int nrel = __popcll(relmask);
    for (int k0 = nrel - 1; k0 >= 0; k0 -= kGroup) {
      bool pass[kGroup];
      float sqv[kGroup], dxv[kGroup], dyv[kGroup], av[kGroup], arawv[kGroup], invv[kGroup];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const int k = max(k0 - j, 0);                 // slots below 0 re-read slot 0, never pass
        const float4 f0 = s_f0[k];
        const float4 f1 = s_f1[k];
        const float4 f2 = s_f2[k];
        float dx, dy;
        const float sq = blend_kq(f0, f1, pxf, pyf, dx, dy);
        // the forward pass's blend decision, for list positions (from 0) before the pixel's stop
        pass[j] = k0 - j >= 0 && __float_as_int(f2.w) < nc && sq >= f1.z;
        const float araw = __builtin_amdgcn_exp2f(sq + f1.y);
        const float a = fminf(amax, araw);
        sqv[j] = sq; dxv[j] = dx; dyv[j] = dy; av[j] = a; arawv[j] = araw;
        invv[j] = __builtin_amdgcn_rcpf(1.0f - a);
      }
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const bool contrib = pass[j];
        if (__ballot(contrib) == 0ull) continue;      // wave-uniform
        const int k = k0 - j;                         // >= 0 here: some lane passed
        const float4 f1 = s_f1[k];
        const float4 f2 = s_f2[k];
        const float4 f3 = s_f3[k];
        const float4 f0 = s_f0[k];
        const float a = av[j], inv = invv[j], dx = dxv[j], dy = dyv[j];
        T = contrib ? T * inv : T;                    // transmittance in front of this splat
        const float w = contrib ? a * T : 0.0f;
        const float gf = fmaf(g[0], f2.x, fmaf(g[1], f2.y, fmaf(g[2], f2.z, fmaf(g[3], f3.x,
                         fmaf(g[4], f3.y, fmaf(g[5], f3.z, g[6] * f1.w))))));
        const float dLda = contrib ? fmaf(T, gf, -gb * inv) : 0.0f;
        gb = contrib ? fmaf(w, gf, gb) : gb;
        float pg[kScreenGrads];
        pg[7] = g[0] * w;
        pg[8] = g[1] * w;
        pg[9] = g[2] * w;
        pg[10] = g[3] * w;
        pg[11] = g[4] * w;
        pg[12] = g[5] * w;
        pg[6] = g[6] * w;
        // alpha clamped at alpha_max: no gradient to opacity or the quadratic form
        const bool free_a = contrib && !(arawv[j] > opt.alpha_max);
        const float dLda_u = free_a ? dLda : 0.0f;
        pg[5] = free_a ? dLda * __builtin_amdgcn_exp2f(sqv[j]) : 0.0f;   // d alpha / d o = e^(-q/2)
        const float dLdq = dLda_u * (-0.5f * a);
        pg[2] = dLdq * dx * dx;
        pg[3] = dLdq * 2.0f * dx * dy;
        pg[4] = dLdq * dy * dy;
        const float dLdq2 = dLdq * kM2OverK;
        pg[0] = dLdq2 * fmaf(f0.z, dx, (0.5f * f0.w) * dy);
        pg[1] = dLdq2 * fmaf(0.5f * f0.w, dx, f1.x * dy);
        const int64_t dst = base_idx + s_g[k];
        float v16[16], sv[4];
#pragma unroll
        for (int i = 0; i < 16; ++i) v16[i] = i < kScreenGrads ? pg[i] : 0.0f;
        wave_sum16_rows(v16, sv);
        // sum i sits in lane 16 (i / 4) + 15, slot i % 4: bring it to lane i, then one atomic
        // instruction adds all thirteen into the splat's 64-byte line
        const int src = 16 * ((lane & 15) >> 2) + 15;
        const float t0 = __shfl(sv[0], src, kWave), t1 = __shfl(sv[1], src, kWave);
        const float t2 = __shfl(sv[2], src, kWave), t3 = __shfl(sv[3], src, kWave);
        const int jj = lane & 3;
        const float val = jj == 0 ? t0 : (jj == 1 ? t1 : (jj == 2 ? t2 : t3));
        if (lane < kScreenGrads && val != 0.0f) unsafeAtomicAdd(&sgrad[dst * kScreenStride + lane], val);
      }
    }
    __syncthreads();                                  // reads done before the next batch lands
  }
}

// Chain the per-(camera, Gaussian) screen-space gradients through the projection to the
// Gaussian parameters (one thread per Gaussian, cameras summed in registers).
__global__ __launch_bounds__(256) void k_project_bwd(
    int64_t n, int n_cams, const DevCamera* __restrict__ cams, DevOptions opt,
    const float* __restrict__ mean, const float* __restrict__ quat, const float* __restrict__ scale,
    const float* __restrict__ sgrad, float* __restrict__ d_mean,
    float* __restrict__ d_cov, float* __restrict__ d_quat, float* __restrict__ d_scale,
    float* __restrict__ d_opac, float* __restrict__ d_rgb, float* __restrict__ d_nrm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float px = mean[i], py = mean[n + i], pz = mean[2 * n + i];
  const float qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
  const float s0 = scale[i], s1 = scale[n + i], s2 = scale[2 * n + i];
  float gm[3] = {0.f, 0.f, 0.f}, gS[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float go = 0.f, gc[3] = {0.f, 0.f, 0.f}, gn[3] = {0.f, 0.f, 0.f};
  ProjGeo G;
  bool any = false;
  for (int c = 0; c < n_cams; ++c) {
    float sg[16];
    const float4* line = reinterpret_cast<const float4*>(sgrad + ((int64_t)c * n + i) * kScreenStride);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = line[q];
      sg[4 * q] = v.x; sg[4 * q + 1] = v.y; sg[4 * q + 2] = v.z; sg[4 * q + 3] = v.w;
    }
    bool nz = false;
#pragma unroll
    for (int k = 0; k < kScreenGrads; ++k) nz = nz || sg[k] != 0.0f;
    if (!nz) continue;
    any = true;
    const DevCamera& cam = cams[c];
    proj_geometry(px, py, pz, qw, qx, qy, qz, s0, s1, s2, cam, opt.lowpass, G);
    // conic (A,B,C) = (c, -b, a) / det  ->  Sigma_s = [[a, b], [b, c]]
    const float a = G.a, b = G.b, cc = G.c, det = G.det;
    const float id = 1.0f / det, id2 = id * id;
    const float gA = sg[2], gB = sg[3], gC = sg[4];
    const float ga = gA * (-cc * cc * id2) + gB * (b * cc * id2) + gC * (id - a * cc * id2);
    const float gb = gA * (2.0f * b * cc * id2) + gB * (-id - 2.0f * b * b * id2) + gC * (2.0f * a * b * id2);
    const float gcv = gA * (id - a * cc * id2) + gB * (a * b * id2) + gC * (-a * a * id2);
    const float Gs[4] = {ga, 0.5f * gb, 0.5f * gb, gcv};
    const float* M = G.M;
    // dL/dSigma = M^T Gs M
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        gS[3 * j + k] += M[j] * (Gs[0] * M[k] + Gs[1] * M[3 + k]) +
                         M[3 + j] * (Gs[2] * M[k] + Gs[3] * M[3 + k]);
    // dL/dM = 2 Gs M Sigma ; dL/dJ = dL/dM T^T
    float GM[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j)
          acc += (Gs[2 * r] * M[j] + Gs[2 * r + 1] * M[3 + j]) * G.S[3 * j + k];
        GM[3 * r + k] = 2.0f * acc;
      }
    const float* T = cam.T;
    float GJ[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int m = 0; m < 3; ++m)
        GJ[3 * r + m] = GM[3 * r] * T[3 * m] + GM[3 * r + 1] * T[3 * m + 1] + GM[3 * r + 2] * T[3 * m + 2];
    const float z = G.zc, iz = 1.0f / z, iz2 = iz * iz, iz3 = iz2 * iz;
    const float fx = cam.fx, fy = cam.fy;
    float gx = GJ[2] * (-fx * iz2);
    float gy = GJ[5] * (-fy * iz2);
    float gz = GJ[0] * (-fx * iz2) + GJ[4] * (-fy * iz2) + GJ[2] * (2.0f * fx * G.xc * iz3) +
               GJ[5] * (2.0f * fy * G.yc * iz3);
    gx += sg[0] * fx * iz;
    gz += sg[0] * (-fx * G.xc * iz2);
    gy += sg[1] * fy * iz;
    gz += sg[1] * (-fy * G.yc * iz2);
    gz += sg[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) gm[k] += T[k] * gx + T[3 + k] * gy + T[6 + k] * gz;
    go += sg[5];
    gc[0] += sg[7]; gc[1] += sg[8]; gc[2] += sg[9];
    gn[0] += sg[10]; gn[1] += sg[11]; gn[2] += sg[12];
  }
  if (!any) return;
  if (d_mean) { d_mean[i] += gm[0]; d_mean[n + i] += gm[1]; d_mean[2 * n + i] += gm[2]; }
  if (d_cov) {
    d_cov[i] += gS[0];
    d_cov[n + i] += gS[1] + gS[3];
    d_cov[2 * n + i] += gS[2] + gS[6];
    d_cov[3 * n + i] += gS[4];
    d_cov[4 * n + i] += gS[5] + gS[7];
    d_cov[5 * n + i] += gS[8];
  }
  if (d_scale || d_quat) {
    // Sigma = R diag(s^2) R^T: dL/ds_m = 2 s_m (R^T G R)_mm, dL/dR = 2 G R diag(s^2)
    const float* R = G.R;
    const float sc[3] = {s0, s1, s2};
    if (d_scale) {
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int k = 0; k < 3; ++k) acc += R[3 * j + m] * gS[3 * j + k] * R[3 * k + m];
        d_scale[m * n + i] += 2.0f * sc[m] * acc;
      }
    }
    if (d_quat && G.qlen > 0.0f) {
      float GR[9];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          float acc = 0.f;
#pragma unroll
          for (int k = 0; k < 3; ++k) acc += gS[3 * j + k] * R[3 * k + m];
          GR[3 * j + m] = 2.0f * acc * G.v[m];
        }
      const float w = G.qw, x = G.qx, y = G.qy, z = G.qz;
      float gq[4];
      gq[0] = 2.0f * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
      gq[1] = 2.0f * (y * GR[1] + z * GR[2] + y * GR[3] - 2.0f * x * GR[4] - w * GR[5] + z * GR[6] +
                      w * GR[7] - 2.0f * x * GR[8]);
      gq[2] = 2.0f * (-2.0f * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] +
                      z * GR[7] - 2.0f * y * GR[8]);
      gq[3] = 2.0f * (-2.0f * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2.0f * z * GR[4] +
                      y * GR[5] + x * GR[6] + y * GR[7]);
      const float dot = w * gq[0] + x * gq[1] + y * gq[2] + z * gq[3];
      const float il = 1.0f / G.qlen;
      d_quat[i] += (gq[0] - w * dot) * il;
      d_quat[n + i] += (gq[1] - x * dot) * il;
      d_quat[2 * n + i] += (gq[2] - y * dot) * il;
      d_quat[3 * n + i] += (gq[3] - z * dot) * il;
    }
  }
  if (d_opac) d_opac[i] += go;
  if (d_rgb) { d_rgb[i] += gc[0]; d_rgb[n + i] += gc[1]; d_rgb[2 * n + i] += gc[2]; }
  if (d_nrm) { d_nrm[i] += gn[0]; d_nrm[n + i] += gn[1]; d_nrm[2 * n + i] += gn[2]; }
}

}  // namespace

hipError_t launch_composite(int64_t n, int n_cams, int W, int H, const float4* rec,
                            const uint32_t* vals, const uint32_t* ranges, const uint32_t* order,
                            const DevOptions& opt, const pcs_images& out, float* t_final,
                            int32_t* n_contrib, hipStream_t s, hipEvent_t ev_start,
                            hipEvent_t ev_stop) {
  const int TX = (W + kTile - 1) / kTile, TY = (H + kTile - 1) / kTile;
  const int64_t tiles_per_cam = (int64_t)TX * TY;
  const int64_t total = tiles_per_cam * n_cams;
  if (total == 0) return hipSuccess;
  // four single-wavefront blocks per tile, in groups of 8 tiles (see quadrant_of_block)
  const int64_t blocks = (total + 7) / 8 * 32;
  if (ev_start || ev_stop)
    // the dispatch itself stamps the events: no marker packets in the stream around the kernel
    hipExtLaunchKernelGGL(k_composite, dim3((unsigned)blocks), dim3(kWave), 0, s, ev_start, ev_stop, 0,
                          n, W, H, TX, tiles_per_cam, total, rec, vals, ranges, order, opt, out.rgb,
                          out.normal, out.depth, out.alpha, t_final, n_contrib);
  else
    hipLaunchKernelGGL(k_composite, dim3((unsigned)blocks), dim3(kWave), 0, s, n, W, H, TX,
                       tiles_per_cam, total, rec, vals, ranges, order, opt, out.rgb, out.normal, out.depth,
                       out.alpha, t_final, n_contrib);
  return hipGetLastError();
}

hipError_t launch_composite_backward(int64_t n, int n_cams, int W, int H, const float4* rec,
                                     const uint32_t* vals, const uint32_t* ranges,
                                     const uint32_t* order, const DevOptions& opt, const float* t_final,
                                     const int32_t* n_contrib, const pcs_images& grad_out,
                                     float* sgrad, hipStream_t s) {
  const int TX = (W + kTile - 1) / kTile, TY = (H + kTile - 1) / kTile;
  const int64_t tiles_per_cam = (int64_t)TX * TY;
  const int64_t total = tiles_per_cam * n_cams;
  if (total == 0) return hipSuccess;
  const int64_t blocks = (total + 7) / 8 * 32;      // four single-wavefront blocks per tile
  hipLaunchKernelGGL(k_composite_bwd, dim3((unsigned)blocks), dim3(kWave), 0, s, n, W, H, TX,
                     tiles_per_cam, total, rec, vals, ranges, order, opt, t_final, n_contrib,
                     grad_out.rgb, grad_out.normal, grad_out.depth, grad_out.alpha, sgrad);
  return hipGetLastError();
}

hipError_t launch_project_backward(int64_t n, int n_cams, const DevCamera* cams,
                                   const DevOptions& opt, const pcs_gaussians& g,
                                   const float* sgrad, const pcs_grads& grads, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, n_cams,
                     cams, opt, g.mean, g.quat, g.scale, sgrad, grads.mean, grads.cov6,
                     grads.quat, grads.scale, grads.opacity, grads.rgb, grads.normal);
  return hipGetLastError();
}

}  // namespace pcs
