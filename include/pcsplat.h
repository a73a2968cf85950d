/*
 * pcsplat -- 3D elliptical-Gaussian splatting rasterizer for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libpcsplat.so. Every entry point takes plain pointers and sizes; no C++ type and no
 * exception crosses it. Unless stated otherwise:
 *   - array arguments are DEVICE pointers on the context's device, FP32, planar
 *     ("component-major": component k of item i lives at ptr[k * n + i]);
 *   - the caller owns every input and output buffer; the library owns the context, the render
 *     state and the workspace they hold (device memory from hipMalloc or from the allocator
 *     installed with pcs_context_set_allocator, grown on demand and released by the matching
 *     destroy call);
 *   - work is enqueued on `stream` (a hipStream_t; NULL = the null stream) in stream order; the
 *     host synchronises only where a size must be known: pcs_render_forward reads back the
 *     instance count and depth range (not in capacity mode, PCS_FLAG_CAPACITY_MODE), pcs_knn_pca
 *     the cloud's bounding box, pcs_voxelize the voxel count;
 *   - a context or state may be used by one host thread at a time;
 *   - the return value is a status code; pcs_last_error() gives a thread-local message.
 *
 * The method is Section 3.1 of "Low Latency Point Cloud Rendering with Learned Splatting"
 * (arXiv:2409.16504): every point is a 3D Gaussian <G(p, Sigma), o, c, n>; Sigma = R diag(s^2) R^T
 * with R from a unit quaternion; the Gaussian is projected with the EWA approximation of Eq. 4
 * (Sigma_s = J T Sigma T^T J^T, view W = [T t; 0 1] of Eq. 3), bounded at three standard
 * deviations, depth-sorted per pixel, and alpha-blended front to back (Eq. 1) with
 * alpha = o * exp(-1/2 d^T Sigma_s^-1 d) (Eq. 2); normals are blended like colours.
 */
#ifndef PCSPLAT_H
#define PCSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
#define PCS_OK 0
#define PCS_ERR_INVALID_ARG 1  /* null pointer, bad size, non-finite camera, ... */
#define PCS_ERR_HIP 2          /* a HIP runtime call failed (message names it) */
#define PCS_ERR_OOM 3          /* device allocation failed; nothing was leaked */
#define PCS_ERR_CAPACITY 4     /* a fixed-capacity buffer was too small */
#define PCS_ERR_UNSUPPORTED 5  /* size beyond a documented limit */

/* ---- render flags ---------------------------------------------------------------------- */
#define PCS_FLAG_SAVE_STATE 1u /* keep projection, sorted lists and tile ranges for backward */
/* Capacity mode: the render enqueues everything without waiting on the device. The tile-instance
 * buffers of the state keep a fixed capacity: 1.25 x the instance total of an earlier frame of the
 * same state (the previous one, once its count has reached the host; the state's first
 * capacity-mode frame waits for its own count, like a plain render, to size it). A frame with more
 * instances than the capacity is not composited (every tile is left empty: background only) and
 * pcs_state_status reports PCS_ERR_CAPACITY with the count it needs; the next capacity-mode render
 * of the state is sized for it. With the same inputs and a capacity that holds, the launch sequence
 * is the same on every call and allocates nothing, so it can be captured in a HIP graph and
 * replayed (the graph replays the captured frame's sizes; check pcs_state_status after a replay).
 * A captured graph keeps the device addresses of the context's and the state's buffers: while it
 * is in use, render nothing else into that state, and nothing on that context that needs more
 * workspace (more Gaussians, cameras or pixels, or a capacity that has to grow). */
#define PCS_FLAG_CAPACITY_MODE 2u

/* Pinhole camera (Section 3.1, Eq. 3-4). x_c = T p + t with T row-major; camera axes x right,
 * y down, z forward; pixel (i, j) has its centre at (i + 0.5, j + 0.5); u = fx x/z + cx,
 * v = fy y/z + cy. Host memory. */
typedef struct pcs_camera {
  float T[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} pcs_camera;

/* Gaussians (Section 3.1): n items; device pointers, planar FP32.
 *   mean[3][n], quat[4][n] (w,x,y,z, need not be unit; zero means identity), scale[3][n] (the
 *   standard deviations sigma_x,y,z along the rotated axes), opacity[n], rgb[3][n], normal[3][n].
 * Gaussians with any non-finite field are culled. */
typedef struct pcs_gaussians {
  int64_t n;
  const float* mean;
  const float* quat;
  const float* scale;
  const float* opacity;
  const float* rgb;
  const float* normal;
} pcs_gaussians;

/* Options (defaults from pcs_options_default):
 *   z_near 0.2     cull when camera-space z <= z_near (must be > 0: depths order as positive floats)
 *   lowpass 0.3    added to both diagonal entries of Sigma_s (pixels^2)
 *   sigma_cut 3    splat boundary at sigma_cut standard deviations (Section 3.1)
 *   alpha_min 1/255, alpha_max 0.99, t_eps 1e-4: a splat is skipped where alpha < alpha_min,
 *                  alpha is clamped to alpha_max, blending of a pixel stops after the splat that
 *                  takes its transmittance below t_eps (0 <= t_eps <= 1)
 *   bg[3] 0        background colour added with the final transmittance (RGB only) */
typedef struct pcs_options {
  float z_near, lowpass, sigma_cut, alpha_min, alpha_max, t_eps;
  float bg[3];
  uint32_t flags;
} pcs_options;

/* Output images, device FP32, planar per camera: rgb[C][3][H][W], normal[C][3][H][W],
 * depth[C][H][W] (sum of T_k alpha_k z_k, not normalised), alpha[C][H][W] (= 1 - final
 * transmittance). Any pointer may be NULL except rgb. For pcs_render_backward the same struct
 * carries the upstream gradients of rgb, normal, depth and alpha (NULL = zero). */
typedef struct pcs_images {
  float* rgb;
  float* normal;
  float* depth;
  float* alpha;
} pcs_images;

/* Gradients, device FP32, planar, ACCUMULATED (+=) into the caller's buffers (the caller zeroes
 * them). mean[3][n], cov6[6][n] (dL/dSigma for the six unique entries xx,xy,xz,yy,yz,zz, an
 * off-diagonal entry moving both symmetric elements), quat[4][n], scale[3][n], opacity[n],
 * rgb[3][n], normal[3][n]. Any pointer may be NULL. */
typedef struct pcs_grads {
  float* mean;
  float* cov6;
  float* quat;
  float* scale;
  float* opacity;
  float* rgb;
  float* normal;
} pcs_grads;

typedef struct pcs_context pcs_context; /* device, stream-independent workspace, timers */
typedef struct pcs_state pcs_state;     /* per-render saved data for backward and export */

/* Message of the last failing call on this host thread ("" if none). */
const char* pcs_last_error(void);

/* Create a context on HIP device `device` (makes it current on this thread). */
int pcs_context_create(int device, pcs_context** out);
void pcs_context_destroy(pcs_context* ctx);

/* Device memory of the workspace. By default the library takes its workspace (the context's,
 * states' and voxel objects' buffers, grown on demand and kept until they must grow or their owner
 * is destroyed) with hipMalloc and returns it with hipFree. With an allocator installed, every
 * buffer allocated from then on comes from alloc(bytes, user) (NULL: PCS_ERR_OOM, nothing leaked)
 * and goes back through release(ptr, user), e.g. a framework's caching allocator. Buffers keep the
 * allocator that made them, so the allocator may be changed at any time; both callbacks NULL
 * restores hipMalloc. The callbacks run on the calling host thread, inside the library call that
 * needs the memory (a render, a voxelisation, ...) or inside pcs_*_destroy; a buffer is released
 * only after the work that used it has been enqueued on the call's stream (destroy synchronises
 * the device first). Memory tied to one stream by the allocator must only be used on that stream. */
typedef void* (*pcs_alloc_fn)(size_t bytes, void* user);
typedef void (*pcs_free_fn)(void* ptr, void* user);
int pcs_context_set_allocator(pcs_context* ctx, pcs_alloc_fn alloc, pcs_free_fn release, void* user);

/* Per-stage timing with HIP events recorded on the caller's stream around every kernel stage.
 * pcs_context_timing(ctx, 1) resets the accumulators and enables timing; pcs_context_timings
 * copies up to `cap` accumulated millisecond totals (stage order: project, scan, binning, sort,
 * ranges, composite, backward_composite, backward_project, knn_pca, voxelize, conv, conv_backward,
 * head, head_backward, shade) plus per-stage launch counts
 * and synchronises the stream. */
int pcs_context_timing(pcs_context* ctx, int enable);
/* As pcs_context_timing(ctx, 1), but events are recorded only around the stages whose bit
 * (1 << stage index, order above) is set in stage_mask; 0 disables timing. */
int pcs_context_timing_stages(pcs_context* ctx, uint32_t stage_mask);
int pcs_context_timings(pcs_context* ctx, double* ms, int64_t* launches, int cap, void* stream);

int pcs_state_create(pcs_context* ctx, pcs_state** out);
void pcs_state_destroy(pcs_state* st);

void pcs_options_default(pcs_options* out);

/* Forward render (Section 3.1, Eq. 1-4) of `n_cams` cameras (host array) that share one width and
 * height. Limits (PCS_ERR_UNSUPPORTED beyond them): n < 2^31, n * n_cams < 2^30, instance count
 * M < 2^30, n_cams * tiles < 2^31. If `state` is non-NULL
 * it receives what pcs_render_backward and pcs_state_bins need (the flag SAVE_STATE is implied);
 * the state stays valid until it is passed to another render or destroyed. */
int pcs_render_forward(pcs_context* ctx, const pcs_gaussians* g, const pcs_camera* cams,
                       int32_t n_cams, const pcs_options* opt, const pcs_images* out,
                       pcs_state* state, void* stream);

/* Backward render: the adjoint of pcs_render_forward for the Gaussians, cameras and options saved
 * in `state`, given upstream gradients `grad_out` (same layout as the images). The compositing
 * is recomputed back to front from the saved per-pixel transmittance and last-contributor
 * index; per-splat screen-space gradients are reduced across each 64-lane wavefront and added
 * atomically, then chained through the EWA projection to the Gaussian parameters.
 * The saved options must leave the final transmittance recoverable: t_eps * (1 - alpha_max) >= 2^-100
 * (PCS_ERR_UNSUPPORTED otherwise, e.g. for t_eps = 0). */
int pcs_render_backward(pcs_context* ctx, const pcs_state* state, const pcs_images* grad_out,
                        const pcs_grads* grads, void* stream);

/* Allocation-free variant of pcs_render_backward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving or training loops, hosts that forbid hipMalloc).
 * Same arguments, kernels and results as pcs_render_backward (up to the order of the float atomic
 * additions); it calls no hipMalloc, hipFree or other allocating routine. The per-splat
 * screen-space gradient lines live instead in a fixed device array of the library, 16 MiB per GPU
 * (held from library load until the process ends), so the state may hold at most
 * n * n_cams <= 2^18 = 262,144 (camera, Gaussian) splats: PCS_ERR_CAPACITY beyond that, with
 * nothing launched. The array is cleared by a kernel at the start of every call and keeps the last
 * call's contents afterwards. All calls on one GPU share that one array: calls that overlap in
 * time on one GPU (different streams, host threads or contexts without ordering between them)
 * race and give wrong gradients; order them on one stream or with events. Other errors as for
 * pcs_render_backward. */
int pcs_render_backward_noalloc(pcs_context* ctx, const pcs_state* state, const pcs_images* grad_out,
                                const pcs_grads* grads, void* stream);

/* Status of the frame last rendered into `state`: synchronises `stream` and returns PCS_OK, or
 * PCS_ERR_CAPACITY (capacity mode: the frame had more tile instances than the state's capacity;
 * *required, if given, receives its count), or PCS_ERR_HIP (a wait of the instance ordering ran out
 * its bound, which only a broken launch does; the frame was not composited). A failed frame's
 * images hold the background only, and its backward adds nothing. */
int pcs_state_status(pcs_state* state, int64_t* required, void* stream);

/* Instance capacity the state's capacity-mode renders use (0 before the first one). */
int pcs_state_capacity(const pcs_state* state, int64_t* capacity);

/* Bound, in polling rounds, of the waits in the instance ordering's chained scans (0: the default,
 * 2^22 rounds). The waits end as soon as the earlier partitions of the launch have published, which
 * always happens in a correct launch; the bound only keeps a broken launch from hanging. A tiny
 * bound makes waits run out on purpose (diagnostics and tests of the error path): the frame then
 * reports PCS_ERR_HIP through pcs_state_status and pcs_state_bins, and every kernel still ends. */
int pcs_context_set_wait_limit(pcs_context* ctx, uint32_t rounds);

/* Measured LDS read bandwidth of the whole device in GB/s (a kernel of conflict-free 16-byte LDS
 * reads on every CU, timed with HIP events; synchronises the stream): the peak that the benchmark
 * holds the compositing kernel's LDS traffic against. */
int pcs_measure_lds_bandwidth(pcs_context* ctx, double* gbs, void* stream);

/* Parity export of a saved state (device pointers owned by the state). A splat is listed in every
 * 16x16 tile that meets the axis-aligned box of its sigma_cut ellipse (Section 3.1): half extents
 * (sigma_cut sqrt(a)) 1.001 + 0.01 and (sigma_cut sqrt(c)) 1.001 + 0.01 pixels for the screen
 * covariance [[a, b], [b, c]], evaluated in FP32.
 *   keys[m]:  ((cam * tiles_per_cam + ty * TX + tx) << 32) | bits(fp32 camera-space depth)
 *   vals[m]:  Gaussian index, sorted lexicographically by (key, value)
 *   ranges[2][n_tiles]: start and end of every tile's run (empty tiles: 0, 0)
 *   n_contrib[C][H][W] (int32): 1 + list position of the last blended splat of each pixel
 *   t_final[C][H][W]: final transmittance. Valid after the stream has reached the render. */
int pcs_state_bins(const pcs_state* st, const uint64_t** keys, const uint32_t** vals, int64_t* m,
                   const uint32_t** ranges, int64_t* n_tiles, const int32_t** n_contrib,
                   const float** t_final);

/* kNN-PCA surfel ellipsoids (the plain-path estimate of every point's Gaussian): for each of the
 * n points xyz[3][n] the k nearest points (itself included, ties by index, k <= 32) give a
 * covariance about their mean; its eigenvectors are the axes, sigma_i = kappa sqrt(lambda_i) with
 * sigma_3 >= floor * sigma_2, the normal is the least-variance axis oriented away from the cloud
 * centroid. Outputs quat[4][n] (w >= 0), scale[3][n], normal[3][n], and, if nn_dist is not
 * NULL, nn_dist[n]: the distance to the nearest other point (the second of the k, self included;
 * 0 for a duplicated point), from which the average point spacing of Section 4.1's global-sigma
 * baseline is taken. nn_dist needs k >= 2. */
int pcs_knn_pca(pcs_context* ctx, const float* xyz, int64_t n, int32_t k, float kappa,
                float floor_ratio, float* quat, float* scale, float* normal, float* nn_dist,
                void* stream);

/* ---- late shading (Section 3.1: the rendered normal map shaded by a pixel shader) -----------
 * The paper fixes no shading model; this is Blinn-Phong with one directional light. Per pixel of
 * camera c: fg = rgb - (1 - alpha) bg (the premultiplied albedo), n = normal / |normal| (world
 * frame; a zero normal keeps only the ambient term), v = the unit direction from the pixel back to
 * the camera (the pixel ray (x + 0.5 - cx) / fx, (y + 0.5 - cy) / fy, 1 rotated to world by T^T,
 * negated), l = light.dir normalised, h = (l + v) / |l + v|:
 *   out = (fg (ambient + diffuse max(0, n.l)) + alpha specular max(0, n.h)^shininess) color
 *         + (1 - alpha) bg.
 * in->rgb, in->normal ([C][3][H][W]) and in->alpha ([C][H][W]) are required; out_rgb [C][3][H][W]
 * may be in->rgb (each pixel is read before it is written). All cameras share width and height.
 * Errors: NULL buffers, non-positive shininess, a zero light direction -> PCS_ERR_INVALID_ARG. */
typedef struct {
  float dir[3];      /* towards the light, world frame (normalised by the library) */
  float color[3];
  float ambient, diffuse, specular, shininess;
} pcs_light;

int pcs_shade(pcs_context* ctx, const pcs_images* in, const pcs_camera* cams, int32_t n_cams,
              const pcs_light* light, const float bg[3], float* out_rgb, void* stream);

/* ---- sparse point-to-ellipsoid estimator (Section 3.2) -------------------------------------
 * Voxels of a point cloud on a grid of G^3 voxels over [-1,1]^3 (G a power of two <= 1024; G = 1024
 * is the 10-bit quantisation of Section 3.3; a coarser G is the density-adaptive voxel size of
 * Section 3.2): coordinate c = clamp(floor((p + 1) * G/2), 0, G-1), voxels numbered in ascending
 * linear key (x << 20 | y << 10 | z). Features are BF16 (bit patterns in uint16_t), row-major
 * [V][channels]; 32 input channels: mean colour (3), mean residual (p + 1) * G/2 - (c + 0.5) (3)
 * (Section 3.2's colour and coordinate residual), zeros. Owned by the voxels object. */
typedef struct pcs_voxels pcs_voxels;
int pcs_voxels_create(pcs_context* ctx, pcs_voxels** out);
void pcs_voxels_destroy(pcs_voxels* vox);

/* Voxelise n points xyz[3][n], rgb[3][n] (device, FP32) and build the kernel map (for every voxel
 * and offset k = 9 (dx+1) + 3 (dy+1) + (dz+1), the neighbour's index or -1). Synchronises the
 * stream once to size the voxel arrays; *n_voxels receives V. n < 2^30. */
int pcs_voxelize(pcs_context* ctx, const float* xyz, const float* rgb, int64_t n, int32_t grid,
                 pcs_voxels* vox, int64_t* n_voxels, void* stream);

/* Device pointers owned by vox: coords[3][V] (int32), nbr[27][V] (int32), point_voxel[n] (int32),
 * features[V][32] (BF16; a pooled level computes none, its features pointer holds unspecified
 * values: the parents' features come from pcs_pool_features). */
int pcs_voxels_get(const pcs_voxels* vox, const int32_t** coords, const int32_t** nbr,
                   const int32_t** point_voxel, const uint16_t** features, int64_t* n_voxels);

/* Submanifold 3x3x3 convolution (Section 3.2's sparse convolutions at the active voxels only):
 * y[v][o] = relu?(bias[o] + sum_k sum_c w[k][o][c] x[nbr_k(v)][c]), absent neighbours contribute
 * nothing. x[V][cin], y[V][cout], w[27][cout][cin] BF16; bias[cout] FP32 or NULL. Products on
 * BF16 matrix cores (MFMA) with FP32 accumulation; the output is rounded to BF16.
 * cin and cout in {32, 64, 128}, not both 128 (UNSUPPORTED otherwise). */
int pcs_subm_conv_forward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* x, int32_t cin,
                          const uint16_t* w, const float* bias, int32_t cout, int32_t relu, uint16_t* y,
                          void* stream);

/* pcs_subm_conv_forward of the channel concatenation [x1 | x2] (the UNet's skip connections,
 * Section 3.2), read where the two parts lie: x1[V][c1], x2[V][c2] BF16, w[27][cout][c1 + c2].
 * Equal halves c1 = c2, a multiple of 32, with c1 + c2 and cout as for pcs_subm_conv_forward
 * (UNSUPPORTED otherwise). Same arithmetic, bit for bit, as pcs_subm_conv_forward on the
 * concatenated rows. */
int pcs_subm_conv_forward_cat(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* x1, int32_t c1,
                              const uint16_t* x2, int32_t c2, const uint16_t* w, const float* bias,
                              int32_t cout, int32_t relu, uint16_t* y, void* stream);

/* Adjoint of pcs_subm_conv_forward. If y (the forward output) is given, dy is first multiplied by
 * the ReLU derivative (y > 0). dx[V][cin] (BF16, overwritten) or NULL; dw[27][cout][cin] and
 * dbias[cout] FP32, ACCUMULATED (+=), or NULL. */
int pcs_subm_conv_backward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* x, int32_t cin,
                           const uint16_t* w, int32_t cout, const uint16_t* y, const uint16_t* dy,
                           uint16_t* dx, float* dw, float* dbias, void* stream);

/* ---- the paper's UNet-like estimator (Section 3.2, its network figure) ----------------------
 * Encoder: 2x2x2 average pooling of the sparse grid, averaging only the occupied children;
 * decoder: stride-2 transposed 2x2x2 convolution whose outputs are pruned to the encoder's
 * occupancy at that level (so it has exactly the encoder's voxels there, for the skip connection);
 * head: a shared MLP per point predicting offset, scale, rotation, opacity and normal.
 *
 * pcs_pool: the parent voxels of `child` on the grid of half the resolution (coordinates c >> 1,
 * numbered in ascending linear key like a voxelisation; the child grid must be >= 2). `parent`
 * then also holds the child -> parent map and the upsampling tables of pcs_up_conv_*. It must be
 * another object than `child`; the child must stay unchanged while the parent is used.
 * Synchronises the stream once (the parent count), like pcs_voxelize; *n_parents receives it. */
int pcs_pool(pcs_context* ctx, const pcs_voxels* child, pcs_voxels* parent, int64_t* n_parents,
             void* stream);

/* Average pooling of features: parent_feat[p] = mean of child_feat over the occupied children of
 * p (BF16 [V][channels], channels 32, 64 or 128; FP32 sums). The backward writes
 * d_child[j] = d_parent[parent(j)] / (number of children of that parent) (overwritten). */
int pcs_pool_features(pcs_context* ctx, const pcs_voxels* parent, const uint16_t* child_feat, int32_t channels,
                      uint16_t* parent_feat, void* stream);
int pcs_pool_features_backward(pcs_context* ctx, const pcs_voxels* parent, const uint16_t* d_parent,
                               int32_t channels, uint16_t* d_child, void* stream);

/* Transposed stride-2 convolution pruned to the encoder's occupancy: for every child voxel j of
 * the pooled level `parent`, y[j] = relu?(bias + W[k(j)] x[parent(j)]), k(j) = 4 (cx & 1) +
 * 2 (cy & 1) + (cz & 1) the child's position in its parent's 2x2x2 block. x[Vp][cin],
 * y[Vc][cout], w[8][cout][cin] BF16 (cin, cout in {32, 64, 128}, not both 128), bias FP32 or NULL;
 * BF16 MFMA with FP32 accumulation. The backward: dy masked by y > 0 if y is given; dx[Vp][cin]
 * (BF16, overwritten) or NULL, dw[8][cout][cin] and dbias FP32 accumulated, or NULL. */
int pcs_up_conv_forward(pcs_context* ctx, const pcs_voxels* parent, const uint16_t* x, int32_t cin,
                        const uint16_t* w, const float* bias, int32_t cout, int32_t relu, uint16_t* y,
                        void* stream);
int pcs_up_conv_backward(pcs_context* ctx, const pcs_voxels* parent, const uint16_t* x, int32_t cin,
                         const uint16_t* w, int32_t cout, const uint16_t* y, const uint16_t* dy,
                         uint16_t* dx, float* dw, float* dbias, void* stream);

/* The paper's head (Section 3.2): a shared MLP per point. Point i in voxel v (edge e = 2 / grid,
 * integer coordinates c_v) has the input x_i = [feat[v][0:32], (xyz_i + 1) grid / 2 - (c_v + 0.5)]
 * (its voxel's decoder features, BF16, and its own residual inside the voxel in edges, FP32);
 * raw_i = W2 relu(W1 x_i + b1) + b2 with w1[32][35], b1[32], w2[14][32], b2[14] (FP32, row-major
 * [out][in]). Outputs: mean = xyz + e tanh(raw[0:3]) (the offset stays within one voxel edge),
 * scale = e exp(raw[3:6]), quat = normalise(raw[6:10] + (1,0,0,0)), opacity = sigmoid(raw[10]),
 * normal = normalise(raw[11:14]), rgb = the point's colour (Section 3.1 keeps the original colour);
 * all planar [3|4][n] or [n] FP32. xyz must be the points the voxels were built from (a pooled level
 * is refused with PCS_ERR_INVALID_ARG). The backward
 * takes per-point gradients of mean, quat, scale, opacity and normal (any may be NULL = zero) and
 * gives d_feat[V][32] (BF16, overwritten) and the weight gradients (FP32, accumulated: zero them
 * first). No gradient flows to xyz. */
int pcs_unet_head_forward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* feat, const float* w1,
                          const float* b1, const float* w2, const float* b2, const float* xyz,
                          const float* rgb, float* mean, float* quat, float* scale, float* opacity,
                          float* out_rgb, float* normal, void* stream);
int pcs_unet_head_backward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* feat, const float* w1,
                           const float* b1, const float* w2, const float* b2, const float* xyz,
                           const float* d_mean, const float* d_quat, const float* d_scale, const float* d_opacity,
                           const float* d_normal, uint16_t* d_feat, float* d_w1, float* d_b1, float* d_w2,
                           float* d_b2, void* stream);

/* Estimator head (Section 3.2's shared per-point head, with the outputs of configuration 4): per
 * voxel raw = wh f + bh (wh[11][32], bh[11] FP32; f = features[V][32] BF16); per point of the voxel:
 * scale = (2/G) exp(raw[0:3]) (the voxel edge times exp), quat = normalise(raw[3:7] + (1,0,0,0)), opacity =
 * sigmoid(raw[7]), rgb = point colour + raw[8:11], normal = rotated axis of the smallest scale
 * oriented away from the cloud centroid. xyz, rgb are the voxelised points; outputs planar. */
int pcs_estimator_head_forward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* feat,
                               const float* wh, const float* bh, const float* xyz, const float* rgb,
                               float* quat, float* scale, float* opacity, float* out_rgb,
                               float* normal, void* stream);

/* Adjoint of the head for per-point gradients of quat, scale, opacity and rgb (the normal is not
 * differentiated): d_feat[V][32] BF16 (overwritten), d_wh[11][32] and d_bh[11] FP32 accumulated. */
int pcs_estimator_head_backward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* feat,
                                const float* wh, const float* bh, const float* d_quat,
                                const float* d_scale, const float* d_opacity, const float* d_rgb,
                                uint16_t* d_feat, float* d_wh, float* d_bh, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PCSPLAT_H */
