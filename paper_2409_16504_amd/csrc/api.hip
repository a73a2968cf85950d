// C ABI of libpcsplat.so: argument checking, workspace management, stage timing and the launch
// sequence of the renderer (projection -> scan -> binning -> radix sort -> tile ranges ->
// compositing) and of its adjoint.

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pcs_internal.hpp"

using namespace pcs;

// Screen-space gradient lines of pcs_render_backward_noalloc: one 64-byte line per
// (camera, Gaussian) splat, at most kNoAllocSplats splats (16 MiB). Host code never uses the
// array's name as an address: its device address is taken once per device with
// hipGetSymbolAddress (noalloc_scratch) and only that pointer reaches kernels and copies.
constexpr int64_t kNoAllocSplats = int64_t(1) << 18;
static __device__ __align__(256) float scratch[kNoAllocSplats * kScreenStride];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define PCS_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(PCS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define PCS_TRY(expr)           \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != PCS_OK) return rc_; \
  } while (0)

// Where device buffers come from: the context's allocator callbacks, or hipMalloc / hipFree.
struct Allocator {
  pcs_alloc_fn alloc = nullptr;
  pcs_free_fn release = nullptr;
  void* user = nullptr;
};

// A device buffer remembers the allocator that made it and returns its memory there.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  Allocator from;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (from.release) from.release(p, from.user);
      else (void)hipFree(p);
    }
    p = nullptr;
    cap = 0;
    from = Allocator{};
  }
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

void swap_buf(DevBuf& a, DevBuf& b) {
  std::swap(a.p, b.p);
  std::swap(a.cap, b.cap);
  std::swap(a.from, b.from);
}

// Grow-only device buffer; 25% headroom so slowly growing sizes do not reallocate every call.
int ensure_with(const Allocator& al, DevBuf& b, size_t bytes, const char* what) {
  if (bytes <= b.cap && b.p) return PCS_OK;
  b.release();
  const size_t want = std::max<size_t>(256, bytes + bytes / 4);
  if (al.alloc) {
    b.p = al.alloc(want, al.user);
    if (!b.p)
      return fail(PCS_ERR_OOM, std::string("the allocator callback returned no memory for ") +
                                   std::to_string(want) + " bytes of " + what);
    b.from = al;
    b.cap = want;
    return PCS_OK;
  }
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(PCS_ERR_OOM, std::string("hipMalloc of ") + std::to_string(want) + " bytes for " +
                                 what + " failed: " + hipGetErrorString(e));
  }
  b.cap = want;
  return PCS_OK;
}

enum Stage {
  ST_PROJECT = 0, ST_SCAN, ST_BINNING, ST_SORT, ST_RANGES, ST_COMPOSITE, ST_BWD_COMPOSITE,
  ST_BWD_PROJECT, ST_KNN, ST_VOXELIZE, ST_CONV, ST_CONV_BWD, ST_HEAD, ST_HEAD_BWD, ST_SHADE, ST_COUNT
};

int bit_length(uint64_t v) {
  int b = 0;
  while (v) { ++b; v >>= 1; }
  return b;
}

// Smallest final transmittance the adjoint accepts (2^-100): far above the smallest normal float,
// so that the per-splat transmittances recovered from it by division keep full precision.
constexpr double kMinFinalTransmittance = 7.888609052210118e-31;

std::mutex g_scratch_mutex;
std::vector<float*> g_scratch_ptr;   // per device; null until taken

// Device address of `scratch` on `device` (which must be current), taken on first use per device.
int noalloc_scratch(int device, float** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PCS_ERR_HIP, std::string("hipGetSymbolAddress of the backward scratch: ") +
                                   hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[device];
  return PCS_OK;
}

bool finite_camera(const pcs_camera& c) {
  for (float v : c.T) if (!std::isfinite(v)) return false;
  for (float v : c.t) if (!std::isfinite(v)) return false;
  return std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) && std::isfinite(c.cy) &&
         c.fx != 0.0f && c.fy != 0.0f;
}

}  // namespace

struct pcs_state;

struct pcs_context {
  int device = 0;
  DevBuf zbits, rect, keys_alt, vals_alt, scan_scratch, sort_scratch, sgrad, small;
  DevBuf dkeys, dkeys_alt, dvals, dvals_alt, dsort_scratch;   // depth sort of the splats
  DevBuf knn_scratch, conv_tmp, wt_tmp, shade_cams, tile_hist, probe;
  uint32_t* host_small = nullptr;   // pinned 4 KiB: readback of the small device words
  uint32_t seq = 0;                 // frame sequence number (never 0 once used)
  void* small_reset_for = nullptr;  // the small-word buffer whose projection slots are reset
  uint32_t wait_limit = 0;          // look-back wait bound of the ordering kernels (0: default)
  float* noalloc_sgrad = nullptr;   // device address of `scratch` on this context's device
  Allocator alloc;                  // where new workspace comes from (default: hipMalloc)
  pcs_state* internal = nullptr;    // state used when the caller passes none
  bool timing = false;
  uint32_t stage_mask = ~0u;        // stages whose launches are timed
  struct Ev {
    hipEvent_t a, b;
    int stage;
  };
  std::vector<Ev> pool;
  size_t used = 0;
  double acc_ms[ST_COUNT] = {};
  int64_t launches[ST_COUNT] = {};
};

struct pcs_state {
  pcs_context* ctx = nullptr;
  DevBuf rec, keys, vals, ranges, order, t_final, n_contrib, canon, dcams;   // keys: u32 tile ids
  DevBuf words;                     // the frame's error word (device)
  // pinned, coherent host words the kernels set to seq << 32 | value: [0] instance total (from the
  // projection's counts), [1] depth bits, [2] the frame's error word (set once ordering is done)
  unsigned long long* host = nullptr;
  unsigned long long* host_dev = nullptr;   // their device address
  uint32_t seq = 0;                 // sequence number of the last frame rendered into the state
  pcs_gaussians g{};
  std::vector<pcs_camera> cams;
  pcs_options opt{};
  int W = 0, H = 0, C = 0;
  int64_t n = 0, m = 0, n_tiles = 0;
  bool m_known = false;             // m holds the frame's instance total (else read from host[0])
  int64_t capacity = 0;             // instance capacity of capacity-mode frames (0: not sized yet)
  bool capacity_frame = false;      // the last frame ran in capacity mode
  bool valid = false;
  ~pcs_state() {
    if (host) (void)hipHostFree(host);
  }
};

struct pcs_voxels {
  pcs_context* ctx = nullptr;
  int64_t n = 0, V = 0;
  int log2cap = 0;
  int grid = 1024;
  DevBuf keys, order, flag, excl, start, coords, feat, point_voxel, hkeys, hvals, nbr, centroid;
  // a pooled (parent) voxel set: its "points" are the child voxels (point_voxel maps child ->
  // parent), up_fwd[8][n] and up_bwd[8][V] are the transposed convolution's tables
  DevBuf up_fwd, up_bwd, centres, head_gh;
  bool pooled = false;
  bool valid = false;
};

namespace {

// Workspace of a context (or of a state or voxels object on it) from the context's allocator.
int ensure(pcs_context* ctx, DevBuf& b, size_t bytes, const char* what) {
  return ensure_with(ctx->alloc, b, bytes, what);
}

// Records HIP events around a stage when timing is on. A stage of one kernel can instead hand the
// pair to its launch (around = false), which stamps the kernel's own start and end into them.
struct StageTimer {
  pcs_context* ctx;
  int stage;
  hipStream_t s;
  bool around;
  size_t slot = (size_t)-1;
  StageTimer(pcs_context* c, int st, hipStream_t stream, bool around_stage = true, bool enabled = true)
      : ctx(c), stage(st), s(stream), around(around_stage) {
    if (!enabled || !ctx->timing || !((ctx->stage_mask >> stage) & 1u)) return;
    if (ctx->used == ctx->pool.size()) {
      pcs_context::Ev ev{};
      // timing only (read after a stream synchronisation): no system-scope fence, whose cache
      // writeback would otherwise stall the stream at every record
      if (hipEventCreateWithFlags(&ev.a, hipEventDisableSystemFence) != hipSuccess ||
          hipEventCreateWithFlags(&ev.b, hipEventDisableSystemFence) != hipSuccess)
        return;
      ctx->pool.push_back(ev);
    }
    slot = ctx->used++;
    ctx->pool[slot].stage = stage;
    if (around) (void)hipEventRecord(ctx->pool[slot].a, s);
  }
  hipEvent_t start() const { return !around && slot != (size_t)-1 ? ctx->pool[slot].a : nullptr; }
  hipEvent_t stop() const { return !around && slot != (size_t)-1 ? ctx->pool[slot].b : nullptr; }
  ~StageTimer() {
    if (around && slot != (size_t)-1) (void)hipEventRecord(ctx->pool[slot].b, s);
  }
};

DevCamera to_dev(const pcs_camera& c) {
  DevCamera d{};
  std::memcpy(d.T, c.T, sizeof d.T);
  std::memcpy(d.t, c.t, sizeof d.t);
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  d.W = c.width; d.H = c.height;
  return d;
}

DevOptions to_dev(const pcs_options& o) {
  DevOptions d{};
  d.z_near = o.z_near; d.lowpass = o.lowpass; d.sigma_cut = o.sigma_cut;
  d.alpha_min = o.alpha_min; d.alpha_max = o.alpha_max; d.t_eps = o.t_eps;
  d.bg[0] = o.bg[0]; d.bg[1] = o.bg[1]; d.bg[2] = o.bg[2];
  return d;
}

int check_options(const pcs_options& o) {
  const float v[] = {o.z_near, o.lowpass, o.sigma_cut, o.alpha_min, o.alpha_max, o.t_eps,
                     o.bg[0], o.bg[1], o.bg[2]};
  for (float x : v)
    if (!std::isfinite(x)) return fail(PCS_ERR_INVALID_ARG, "options must be finite");
  if (o.z_near <= 0.0f || o.sigma_cut <= 0.0f || o.lowpass < 0.0f || o.alpha_max <= 0.0f ||
      o.alpha_max >= 1.0f || o.alpha_min < 0.0f || o.t_eps < 0.0f || o.t_eps > 1.0f)
    return fail(PCS_ERR_INVALID_ARG,
                "options out of range (need z_near > 0, sigma_cut > 0, lowpass >= 0, "
                "0 < alpha_max < 1, alpha_min >= 0, 0 <= t_eps <= 1)");
  return PCS_OK;
}

// Polls the two pinned words until both carry this frame's sequence number (word 0: instance
// total, word 1: depth bits). After the first millisecond the stream is queried every 100
// microseconds (a query is not free: it is kept off the common path), so a failed launch or a
// stream that drained without the stores is an error instead of a hang.
int wait_frame_words(pcs_state* st, hipStream_t s, uint64_t* total, int* depth_bits) {
  volatile unsigned long long* w = st->host;
  using clock = std::chrono::steady_clock;
  auto next_query = clock::now() + std::chrono::milliseconds(1);
  auto ready = [&](unsigned long long a, unsigned long long b) {
    return (uint32_t)(a >> 32) == st->seq && (uint32_t)(b >> 32) == st->seq;
  };
  for (uint64_t it = 1;; ++it) {
    unsigned long long a = w[0], b = w[1];
    bool ok = ready(a, b);
    if (!ok && (it & 255) == 0 && clock::now() >= next_query) {
      next_query = clock::now() + std::chrono::microseconds(100);
      const hipError_t q = hipStreamQuery(s);
      if (q != hipSuccess && q != hipErrorNotReady)
        return fail(PCS_ERR_HIP, std::string("stream error: ") + hipGetErrorString(q));
      if (q == hipSuccess) {
        a = w[0];
        b = w[1];
        if (!ready(a, b)) return fail(PCS_ERR_HIP, "instance total not delivered");
        ok = true;
      }
    }
    if (ok) {
      *total = a & 0xFFFFFFFFull;
      *depth_bits = (int)(b & 0xFFFFFFFFull);
      return PCS_OK;
    }
  }
}

int check_gaussians(const pcs_gaussians* g) {
  if (!g) return fail(PCS_ERR_INVALID_ARG, "gaussians is NULL");
  if (g->n < 0) return fail(PCS_ERR_INVALID_ARG, "gaussian count is negative");
  if (g->n >= (int64_t(1) << 31)) return fail(PCS_ERR_UNSUPPORTED, "n must be below 2^31");
  if (g->n > 0 && (!g->mean || !g->quat || !g->scale || !g->opacity || !g->rgb || !g->normal))
    return fail(PCS_ERR_INVALID_ARG, "a gaussian attribute pointer is NULL");
  return PCS_OK;
}


// A state's pinned host words (allocated once, on the state's first render).
int state_host_words(pcs_state* st) {
  if (st->host) return PCS_OK;
  void* hw = nullptr;
  void* hw_dev = nullptr;
  if (hipHostMalloc(&hw, 64, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
    (void)hipGetLastError();
    return fail(PCS_ERR_OOM, "pinned host allocation of the state's words failed");
  }
  if (hipHostGetDevicePointer(&hw_dev, hw, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(hw);
    return fail(PCS_ERR_HIP, "no device address for the state's pinned words");
  }
  st->host = reinterpret_cast<unsigned long long*>(hw);
  st->host_dev = reinterpret_cast<unsigned long long*>(hw_dev);
  for (int i = 0; i < 8; ++i) st->host[i] = 0ull;
  return PCS_OK;
}

// Status of the frame last rendered into the state, once the stream has reached its end: the
// error word the ordering reported (host[2]) and, for a capacity-mode frame, its instance total.
int frame_status(pcs_state* st, int64_t* required) {
  if (required) *required = 0;
  if (!st->host) return PCS_OK;
  volatile unsigned long long* w = st->host;
  const unsigned long long e = w[2], t = w[0];
  if ((uint32_t)(e >> 32) != st->seq || (uint32_t)(t >> 32) != st->seq)
    return fail(PCS_ERR_HIP, "the frame's status words were not delivered (stream not finished?)");
  const uint32_t err = (uint32_t)e;
  const int64_t total = (int64_t)(uint32_t)t;
  if (!st->m_known && !(err & kErrSpin) && total <= st->capacity) {
    st->m = total;
    st->m_known = true;
  }
  if (err & kErrSpin)
    return fail(PCS_ERR_HIP, "a look-back wait of the instance ordering ran out (broken launch); "
                             "the frame was not composited");
  if (err & kErrCapacity) {
    if (required) *required = total;
    return fail(PCS_ERR_CAPACITY, "the frame has " + std::to_string(total) +
                                      " tile instances, more than the state's capacity of " +
                                      std::to_string(st->capacity) + "; the next capacity-mode "
                                      "render of this state is sized for it");
  }
  return PCS_OK;
}

int check_backward(pcs_context* ctx, const pcs_state* st, const pcs_images* grad_out,
                   const pcs_grads* grads) {
  if (!ctx || !st || !grad_out || !grads) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  if (st->ctx != ctx) return fail(PCS_ERR_INVALID_ARG, "state belongs to another context");
  if (!st->valid) return fail(PCS_ERR_INVALID_ARG, "state holds no completed forward render");
  // the adjoint recovers each splat's transmittance from the final one by division; the final
  // transmittance is at least t_eps (1 - alpha_max), which must stay a normal float with room to
  // spare, or the recovered values (and every gradient through them) collapse to zero
  if (!((double)st->opt.t_eps * (1.0 - (double)st->opt.alpha_max) >= kMinFinalTransmittance))
    return fail(PCS_ERR_UNSUPPORTED,
                "the backward needs t_eps * (1 - alpha_max) >= 2^-100 (the final transmittance "
                "must stay recoverable); render with a larger t_eps");
  return PCS_OK;
}

// The adjoint's launches with the screen-space gradient lines in `sgrad` (cn lines, cleared here
// by a fill kernel). `timed`: record stage events when timing is on.
int backward_launch(pcs_context* ctx, const pcs_state* st, const pcs_images* grad_out,
                    const pcs_grads* grads, float* sgrad, bool timed, hipStream_t s) {
  const int64_t cn = st->n * st->C;
  PCS_HIP(launch_fill_f32(sgrad, 0.0f, cn * kScreenStride, s));
  const DevOptions dopt = to_dev(st->opt);
  {
    StageTimer tm(ctx, ST_BWD_COMPOSITE, s, true, timed);
    PCS_HIP(launch_composite_backward(st->n, st->C, st->W, st->H, st->rec.as<float4>(),
                                      st->vals.as<uint32_t>(), st->ranges.as<uint32_t>(),
                                      st->order.as<uint32_t>(), dopt,
                                      st->t_final.as<float>(), st->n_contrib.as<int32_t>(),
                                      *grad_out, sgrad, s));
  }
  {
    StageTimer tm(ctx, ST_BWD_PROJECT, s, true, timed);
    PCS_HIP(launch_project_backward(st->n, st->C, st->dcams.as<DevCamera>(), dopt, st->g, sgrad,
                                    *grads, s));
  }
  return PCS_OK;
}

}  // namespace

extern "C" {

const char* pcs_last_error(void) { return g_err.c_str(); }

void pcs_options_default(pcs_options* o) {
  if (!o) return;
  o->z_near = 0.2f;
  o->lowpass = 0.3f;
  o->sigma_cut = 3.0f;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_eps = 1e-4f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
  o->flags = 0;
}

int pcs_context_create(int device, pcs_context** out) {
  if (!out) return fail(PCS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  PCS_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(PCS_ERR_INVALID_ARG, "no such HIP device");
  PCS_HIP(hipSetDevice(device));
  pcs_context* ctx = new pcs_context();
  ctx->device = device;
  void* hp = nullptr;
  if (hipHostMalloc(&hp, 4096, hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return fail(PCS_ERR_OOM, "pinned host allocation failed");
  }
  ctx->host_small = reinterpret_cast<uint32_t*>(hp);
  // device address of the allocation-free backward's scratch on this device (taken once)
  if (noalloc_scratch(device, &ctx->noalloc_sgrad) != PCS_OK) {
    const std::string msg = g_err;
    pcs_context_destroy(ctx);
    return fail(PCS_ERR_HIP, msg);
  }
  *out = ctx;
  return PCS_OK;
}

void pcs_state_destroy(pcs_state* st) { delete st; }

void pcs_context_destroy(pcs_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& ev : ctx->pool) {
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  delete ctx->internal;
  if (ctx->host_small) (void)hipHostFree(ctx->host_small);
  delete ctx;
}

int pcs_context_set_allocator(pcs_context* ctx, pcs_alloc_fn alloc, pcs_free_fn release, void* user) {
  if (!ctx) return fail(PCS_ERR_INVALID_ARG, "context is NULL");
  if ((alloc == nullptr) != (release == nullptr))
    return fail(PCS_ERR_INVALID_ARG, "give both allocator callbacks or neither");
  ctx->alloc = Allocator{alloc, release, user};
  return PCS_OK;
}

int pcs_context_timing_stages(pcs_context* ctx, uint32_t stage_mask) {
  if (!ctx) return fail(PCS_ERR_INVALID_ARG, "context is NULL");
  PCS_TRY(pcs_context_timing(ctx, stage_mask != 0u));
  ctx->stage_mask = stage_mask;
  return PCS_OK;
}

int pcs_context_timing(pcs_context* ctx, int enable) {
  if (!ctx) return fail(PCS_ERR_INVALID_ARG, "context is NULL");
  ctx->timing = enable != 0;
  ctx->stage_mask = ~0u;
  ctx->used = 0;
  std::fill(std::begin(ctx->acc_ms), std::end(ctx->acc_ms), 0.0);
  std::fill(std::begin(ctx->launches), std::end(ctx->launches), int64_t(0));
  return PCS_OK;
}

int pcs_context_timings(pcs_context* ctx, double* ms, int64_t* launches, int cap, void* stream) {
  if (!ctx) return fail(PCS_ERR_INVALID_ARG, "context is NULL");
  PCS_HIP(hipSetDevice(ctx->device));
  PCS_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  for (size_t i = 0; i < ctx->used; ++i) {
    float t = 0.0f;
    PCS_HIP(hipEventElapsedTime(&t, ctx->pool[i].a, ctx->pool[i].b));
    ctx->acc_ms[ctx->pool[i].stage] += t;
    ctx->launches[ctx->pool[i].stage] += 1;
  }
  ctx->used = 0;
  for (int i = 0; i < cap && i < ST_COUNT; ++i) {
    if (ms) ms[i] = ctx->acc_ms[i];
    if (launches) launches[i] = ctx->launches[i];
  }
  return PCS_OK;
}

int pcs_state_create(pcs_context* ctx, pcs_state** out) {
  if (!ctx || !out) return fail(PCS_ERR_INVALID_ARG, "context or out is NULL");
  *out = new pcs_state();
  (*out)->ctx = ctx;
  return PCS_OK;
}

int pcs_render_forward(pcs_context* ctx, const pcs_gaussians* g, const pcs_camera* cams,
                       int32_t n_cams, const pcs_options* opt, const pcs_images* out,
                       pcs_state* state, void* stream) {
  if (!ctx) return fail(PCS_ERR_INVALID_ARG, "context is NULL");
  PCS_TRY(check_gaussians(g));
  if (!cams || n_cams <= 0) return fail(PCS_ERR_INVALID_ARG, "need at least one camera");
  if (!opt) return fail(PCS_ERR_INVALID_ARG, "options is NULL");
  PCS_TRY(check_options(*opt));
  if (!out || !out->rgb) return fail(PCS_ERR_INVALID_ARG, "output rgb image is NULL");
  const int W = cams[0].width, H = cams[0].height;
  if (W <= 0 || H <= 0) return fail(PCS_ERR_INVALID_ARG, "image width and height must be positive");
  if (W > 65535 * kTile || H > 65535 * kTile)
    return fail(PCS_ERR_UNSUPPORTED, "image side above 65535 tiles");
  for (int c = 0; c < n_cams; ++c) {
    if (cams[c].width != W || cams[c].height != H)
      return fail(PCS_ERR_INVALID_ARG, "all cameras of one call must share width and height");
    if (!finite_camera(cams[c])) return fail(PCS_ERR_INVALID_ARG, "camera has non-finite or zero focal values");
  }
  if (state && state->ctx != ctx) return fail(PCS_ERR_INVALID_ARG, "state belongs to another context");
  const int TX = (W + kTile - 1) / kTile, TY = (H + kTile - 1) / kTile;
  const int64_t tiles_per_cam = (int64_t)TX * TY;
  const bool narrow_rect = TX <= kNarrowRectTiles && TY <= kNarrowRectTiles;   // 4-byte rectangles
  const int64_t total_tiles = tiles_per_cam * n_cams;
  if (total_tiles >= (int64_t(1) << 31)) return fail(PCS_ERR_UNSUPPORTED, "cameras x tiles must be below 2^31");
  const int64_t n = g->n;
  const int64_t cn = n * n_cams;
  // the depth sort's chained scan carries counts in 30-bit status words
  if (cn >= (int64_t(1) << 30)) return fail(PCS_ERR_UNSUPPORTED, "n x cameras must be below 2^30");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  const bool capacity_mode = (opt->flags & PCS_FLAG_CAPACITY_MODE) != 0;
  pcs_state* st = state;
  if (!st) {
    if (!ctx->internal) {
      ctx->internal = new pcs_state();
      ctx->internal->ctx = ctx;
    }
    st = ctx->internal;
  }
  st->valid = false;
  PCS_TRY(state_host_words(st));
  // Capacity mode: the tile buffers keep a fixed capacity, sized from an earlier frame's instance
  // total (x 1.25), and the host does not wait for this frame's total. The previous frame's total,
  // if its word has arrived, grows the capacity before anything is enqueued; the state's first
  // capacity-mode frame is sized like a plain one (it waits once).
  int64_t capacity = 0;
  if (capacity_mode && st->capacity > 0) {
    volatile unsigned long long* w = st->host;
    const unsigned long long prev = w[0];
    int64_t need = st->capacity;
    if ((uint32_t)(prev >> 32) == st->seq && st->seq != 0) need = (int64_t)(uint32_t)prev;
    if (need > st->capacity) st->capacity = std::min<int64_t>(need + need / 4, (int64_t(1) << 30) - 1);
    capacity = st->capacity;
  }
  // cameras reach the device as kernel arguments of the frame's first launch (no copy to wait on)
  std::vector<DevCamera> dc(n_cams);
  for (int c = 0; c < n_cams; ++c) dc[c] = to_dev(cams[c]);
  PCS_TRY(ensure(ctx, st->dcams, sizeof(DevCamera) * n_cams, "cameras"));
  PCS_TRY(ensure(ctx, st->words, 64, "frame words"));
  uint32_t* d_err = st->words.as<uint32_t>();
  const DevOptions dopt = to_dev(*opt);

  const int64_t cn1 = std::max<int64_t>(cn, 1);
  PCS_TRY(ensure(ctx, st->rec, cn1 * kRecFloat4 * sizeof(float4), "splat records"));
  PCS_TRY(ensure(ctx, ctx->zbits, cn1 * sizeof(uint32_t), "depth bits"));
  PCS_TRY(ensure(ctx, ctx->rect, cn1 * sizeof(uint2), "tile rectangles"));
  PCS_TRY(ensure(ctx, ctx->scan_scratch, scan_scratch_bytes(cn), "scan scratch"));
  PCS_TRY(ensure(ctx, ctx->small, kSmallWords * 4, "small"));
  PCS_TRY(ensure(ctx, st->ranges, 2 * total_tiles * sizeof(uint32_t), "tile ranges"));
  PCS_TRY(ensure(ctx, st->order, total_tiles * sizeof(uint32_t), "tile order"));
  const int64_t HWC = (int64_t)W * H * n_cams;
  // the final transmittance and last contributor are kept only for a caller's state (backward,
  // parity export); a render without one does not write them
  if (state) {
    PCS_TRY(ensure(ctx, st->t_final, HWC * sizeof(float), "final transmittance"));
    PCS_TRY(ensure(ctx, st->n_contrib, HWC * sizeof(int32_t), "last contributor"));
  }

  uint64_t* d_total = ctx->small.as<uint64_t>();
  uint32_t* d_zrange = ctx->small.as<uint32_t>() + 2;
  auto* d_counts = reinterpret_cast<unsigned long long*>(ctx->small.as<uint32_t>() + kCountWord);
  uint32_t* d_depth = ctx->small.as<uint32_t>() + kDepthWord;   // passes, depth bits, min depth bits
  PCS_TRY(ensure(ctx, ctx->dkeys, cn1 * sizeof(uint32_t), "depth keys"));
  PCS_TRY(ensure(ctx, ctx->dkeys_alt, cn1 * sizeof(uint32_t), "depth keys (alternate)"));
  PCS_TRY(ensure(ctx, ctx->dvals, cn1 * sizeof(uint32_t), "depth order"));
  PCS_TRY(ensure(ctx, ctx->dvals_alt, cn1 * sizeof(uint32_t), "depth order (alternate)"));
  PCS_TRY(ensure(ctx, ctx->dsort_scratch, sort_scratch_bytes(cn), "depth sort scratch"));
  // digit histograms counted by the kernels that write the keys: the tile sort's, then the depth
  // sort's
  PCS_TRY(ensure(ctx, ctx->tile_hist, 2 * kTileHistWords * sizeof(uint32_t), "digit histograms"));
  if (capacity > 0) {
    PCS_TRY(ensure(ctx, st->keys, capacity * sizeof(uint32_t), "keys"));
    PCS_TRY(ensure(ctx, st->vals, capacity * sizeof(uint32_t), "values"));
    PCS_TRY(ensure(ctx, ctx->keys_alt, capacity * sizeof(uint32_t), "keys (alternate)"));
    PCS_TRY(ensure(ctx, ctx->vals_alt, capacity * sizeof(uint32_t), "values (alternate)"));
    PCS_TRY(ensure(ctx, ctx->sort_scratch, sort_scratch_bytes(capacity), "sort scratch"));
  }
  uint32_t* depth_hist = ctx->tile_hist.as<uint32_t>() + kTileHistWords;
  // Cameras reach the projection as kernel arguments and it resets the frame's error word and
  // instance total; the projection slots were reset by the previous frame's tile order. A set-up
  // kernel runs first only for more cameras than one launch carries, for a frame without Gaussians
  // (no projection runs) and where the slots are not known to be reset (a new buffer, or a frame
  // that ended on the host before its tile order was queued: the mark stays cleared until then).
  // A frame captured into a HIP graph always starts with the set-up kernel, so that every replay
  // resets the slots itself, and leaves the mark alone (captured launches do not run).
  hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
  PCS_HIP(hipStreamIsCapturing(s, &capture));
  const bool capturing = capture != hipStreamCaptureStatusNone;
  const bool arg_cams = n_cams <= kArgCams && cn > 0;
  const bool slots_reset = !capturing && ctx->small_reset_for == ctx->small.p;
  if (!capturing) ctx->small_reset_for = nullptr;
  if (!arg_cams || !slots_reset)
    PCS_HIP(launch_init_small(ctx->small.as<uint32_t>(), dc.data(), n_cams, st->dcams.as<DevCamera>(), s, d_err));
  if (cn == 0 && !capturing) ctx->small_reset_for = ctx->small.p;   // no projection: the slots stay reset
  CamBatch batch{};
  for (int c = 0; arg_cams && c < n_cams; ++c) batch.c[c] = dc[c];
  {
    // the projection also clears what the depth sort and the scan need zeroed
    ClearSpans clear;
    clear.p[0] = ctx->dsort_scratch.as<uint32_t>();
    clear.count[0] = sort_clear_words(cn);
    clear.p[1] = ctx->scan_scratch.as<uint32_t>();
    clear.count[1] = scan_clear_words(cn);
    clear.p[2] = ctx->tile_hist.as<uint32_t>();            // both sorts' digit histograms
    clear.count[2] = 2 * kTileHistWords;
    StageTimer tm(ctx, ST_PROJECT, s);
    PCS_HIP(launch_project(n, n_cams, st->dcams.as<DevCamera>(), dopt, *g, st->rec.as<float4>(),
                           ctx->zbits.as<uint32_t>(), ctx->rect.as<uint2>(), narrow_rect, d_zrange, d_counts,
                           clear, s, arg_cams ? &batch : nullptr, d_err, d_total));
  }
  // The instance total reaches the host from the first depth-sort kernel (a store into a pinned
  // word, which the host polls); the (camera, depth) order needs nothing from the host (the depth
  // range is read from the projection's slots on the device, and sort passes beyond the bits that
  // range needs return at once), so it is all queued at once and the host sizes the tile buffers
  // while the GPU sorts by depth. A capacity-mode frame queues every depth pass and never waits.
  ctx->seq = ctx->seq + 1 == 0 ? 1 : ctx->seq + 1;
  st->seq = ctx->seq;
  if (cn > 0) {
    StageTimer tm(ctx, ST_SORT, s);
    bool unused = false;
    PCS_HIP(launch_depth_keys_hist(cn, ctx->zbits.as<uint32_t>(), d_counts, st->host_dev, st->seq,
                                   d_zrange, d_depth, ctx->dkeys.as<uint32_t>(), ctx->dvals.as<uint32_t>(),
                                   depth_hist, s));
    // the first pass now (it returns at once if the depths need none), the others once the host
    // knows how many the depth range needs (all of them in capacity mode)
    PCS_HIP(launch_sort(ctx->dkeys.as<uint32_t>(), ctx->dvals.as<uint32_t>(), ctx->dkeys_alt.as<uint32_t>(),
                        ctx->dvals_alt.as<uint32_t>(), cn, 32, ctx->dsort_scratch.p, s, &unused, d_depth,
                        true, true, depth_hist, 0, capacity > 0 ? -1 : 1, nullptr, 0, d_err,
                        ctx->wait_limit, nullptr, true));
  }
  uint64_t m64 = 0;
  if (cn > 0 && capacity == 0) {
    int depth_bits = 0;
    PCS_TRY(wait_frame_words(st, s, &m64, &depth_bits));
    const int depth_passes = (depth_bits + 7) / 8;
    if (depth_passes > 1) {
      StageTimer tm(ctx, ST_SORT, s);
      bool unused = false;
      PCS_HIP(launch_sort(ctx->dkeys.as<uint32_t>(), ctx->dvals.as<uint32_t>(), ctx->dkeys_alt.as<uint32_t>(),
                          ctx->dvals_alt.as<uint32_t>(), cn, 32, ctx->dsort_scratch.p, s, &unused, d_depth,
                          true, true, depth_hist, 1, depth_passes, nullptr, 0, d_err, ctx->wait_limit,
                          nullptr, true));
    }
    if (m64 >= (uint64_t(1) << 30))
      return fail(PCS_ERR_UNSUPPORTED, "instance count " + std::to_string(m64) + " is not below 2^30");
    if (capacity_mode) {       // the state's first capacity-mode frame sizes the capacity
      st->capacity = std::max<int64_t>(1024, std::min<int64_t>((int64_t)m64 + (int64_t)m64 / 4,
                                                               (int64_t(1) << 30) - 1));
      capacity = st->capacity;
    }
  }
  // the tile buffers: the instance total, or the fixed capacity (then the count stays on the device)
  const int64_t m = cn == 0 ? 0 : (capacity > 0 ? capacity : (int64_t)m64);
  const uint64_t* m_dev = capacity > 0 ? d_total : nullptr;
  const int tile_bits = bit_length((uint64_t)(total_tiles - 1));

  PCS_TRY(ensure(ctx, st->keys, std::max<int64_t>(m, 1) * sizeof(uint32_t), "keys"));
  PCS_TRY(ensure(ctx, st->vals, std::max<int64_t>(m, 1) * sizeof(uint32_t), "values"));
  PCS_TRY(ensure(ctx, ctx->keys_alt, std::max<int64_t>(m, 1) * sizeof(uint32_t), "keys (alternate)"));
  PCS_TRY(ensure(ctx, ctx->vals_alt, std::max<int64_t>(m, 1) * sizeof(uint32_t), "values (alternate)"));
  PCS_TRY(ensure(ctx, ctx->sort_scratch, sort_scratch_bytes(m), "sort scratch"));
  if (m > 0) {
    {
      StageTimer tm(ctx, ST_BINNING, s);
      // binning (with the prefix sum that places its keys) also clears what the tile sort and
      // the tile ranges need zeroed
      ClearSpans clear;
      clear.p[0] = ctx->sort_scratch.as<uint32_t>();
      clear.count[0] = sort_clear_words(m);
      clear.p[1] = st->ranges.as<uint32_t>();
      clear.count[1] = 2 * total_tiles;
      PCS_HIP(launch_scan_binning(n, n_cams, TX, tiles_per_cam, ctx->dvals.as<uint32_t>(),
                                  ctx->dvals_alt.as<uint32_t>(), d_depth, ctx->rect.as<uint2>(), narrow_rect,
                                  ctx->scan_scratch.p, d_total, st->keys.as<uint32_t>(),
                                  st->vals.as<uint32_t>(), tile_bits, ctx->tile_hist.as<uint32_t>(),
                                  clear, s, d_err, ctx->wait_limit,
                                  capacity > 0 ? (uint64_t)capacity : ~uint64_t(0)));
    }
    bool in_alt = false;
    {
      StageTimer tm(ctx, ST_SORT, s);
      // its last pass also finds the tiles' runs
      PCS_HIP(launch_sort(st->keys.as<uint32_t>(), st->vals.as<uint32_t>(), ctx->keys_alt.as<uint32_t>(),
                          ctx->vals_alt.as<uint32_t>(), m, tile_bits, ctx->sort_scratch.p, s, &in_alt,
                          nullptr, true, false, ctx->tile_hist.as<uint32_t>(), 0, -1,
                          st->ranges.as<uint32_t>(), total_tiles, d_err, ctx->wait_limit, m_dev));
    }
    if (in_alt) {
      swap_buf(st->keys, ctx->keys_alt);
      swap_buf(st->vals, ctx->vals_alt);
    }
  }
  if (m == 0) PCS_HIP(launch_fill_u32(st->ranges.as<uint32_t>(), 0u, 2 * total_tiles, s));
  {
    StageTimer tm(ctx, ST_RANGES, s);
    // runs found by the tile sort unless it had no pass to run (one instance or one tile)
    if ((capacity == 0 && m <= 1) || tile_bits == 0)
      PCS_HIP(launch_ranges(st->keys.as<uint32_t>(), m, total_tiles, st->ranges.as<uint32_t>(), s, m_dev, d_err));
    // the ordering is done: the frame's error word goes to the host
    // and the projection slots are reset for the next frame
    PCS_HIP(launch_tile_order(st->ranges.as<uint32_t>(), total_tiles, st->order.as<uint32_t>(), s, d_err,
                              st->host_dev + 2, st->seq, ctx->small.as<uint32_t>() + 2));
    if (total_tiles > 0 && !capturing) ctx->small_reset_for = ctx->small.p;
  }
  {
    StageTimer tm(ctx, ST_COMPOSITE, s, false);   // the kernel's own start and end
    PCS_HIP(launch_composite(n, n_cams, W, H, st->rec.as<float4>(), st->vals.as<uint32_t>(),
                             st->ranges.as<uint32_t>(), st->order.as<uint32_t>(), dopt, *out,
                             state ? st->t_final.as<float>() : nullptr,
                             state ? st->n_contrib.as<int32_t>() : nullptr, s, tm.start(), tm.stop()));
  }
  st->g = *g;
  st->cams.assign(cams, cams + n_cams);
  st->opt = *opt;
  st->W = W;
  st->H = H;
  st->C = n_cams;
  st->n = n;
  st->m = capacity > 0 ? 0 : m;
  st->m_known = capacity == 0;
  st->capacity_frame = capacity > 0;
  st->n_tiles = total_tiles;
  st->valid = true;
  return PCS_OK;
}

int pcs_render_backward(pcs_context* ctx, const pcs_state* st, const pcs_images* grad_out,
                        const pcs_grads* grads, void* stream) {
  PCS_TRY(check_backward(ctx, st, grad_out, grads));
  PCS_HIP(hipSetDevice(ctx->device));
  const int64_t cn = st->n * st->C;
  if (cn == 0) return PCS_OK;
  PCS_TRY(ensure(ctx, ctx->sgrad, (size_t)cn * kScreenStride * sizeof(float), "screen-space gradients"));
  return backward_launch(ctx, st, grad_out, grads, ctx->sgrad.as<float>(), true,
                         reinterpret_cast<hipStream_t>(stream));
}

int pcs_render_backward_noalloc(pcs_context* ctx, const pcs_state* st, const pcs_images* grad_out,
                                const pcs_grads* grads, void* stream) {
  PCS_TRY(check_backward(ctx, st, grad_out, grads));
  const int64_t cn = st->n * st->C;
  if (cn > kNoAllocSplats)
    return fail(PCS_ERR_CAPACITY, "the allocation-free backward takes at most " +
                                      std::to_string(kNoAllocSplats) + " (camera, Gaussian) splats, got " +
                                      std::to_string(cn));
  PCS_HIP(hipSetDevice(ctx->device));
  if (cn == 0) return PCS_OK;
  return backward_launch(ctx, st, grad_out, grads, ctx->noalloc_sgrad, false,
                         reinterpret_cast<hipStream_t>(stream));
}

int pcs_state_bins(const pcs_state* st_c, const uint64_t** keys, const uint32_t** vals, int64_t* m,
                   const uint32_t** ranges, int64_t* n_tiles, const int32_t** n_contrib,
                   const float** t_final) {
  if (!st_c) return fail(PCS_ERR_INVALID_ARG, "state is NULL");
  if (!st_c->valid) return fail(PCS_ERR_INVALID_ARG, "state holds no completed forward render");
  pcs_state* st = const_cast<pcs_state*>(st_c);
  PCS_HIP(hipSetDevice(st->ctx->device));
  PCS_HIP(hipDeviceSynchronize());
  if (st->n * st->C > 0) PCS_TRY(frame_status(st, nullptr));   // a failed frame has no lists
  PCS_TRY(ensure(st->ctx, st->canon, std::max<int64_t>(st->m, 1) * sizeof(uint64_t), "canonical keys"));
  PCS_HIP(launch_canonical_keys(st->keys.as<uint32_t>(), st->vals.as<uint32_t>(), st->m, st->n,
                                st->n_tiles / std::max(st->C, 1), st->rec.as<float4>(),
                                st->canon.as<uint64_t>(), nullptr));
  PCS_HIP(hipDeviceSynchronize());
  if (keys) *keys = st->canon.as<uint64_t>();
  if (vals) *vals = st->vals.as<uint32_t>();
  if (m) *m = st->m;
  if (ranges) *ranges = st->ranges.as<uint32_t>();
  if (n_tiles) *n_tiles = st->n_tiles;
  if (n_contrib) *n_contrib = st->n_contrib.as<int32_t>();
  if (t_final) *t_final = st->t_final.as<float>();
  return PCS_OK;
}

int pcs_state_status(pcs_state* st, int64_t* required, void* stream) {
  if (required) *required = 0;
  if (!st) return fail(PCS_ERR_INVALID_ARG, "state is NULL");
  if (!st->valid) return fail(PCS_ERR_INVALID_ARG, "state holds no completed forward render");
  PCS_HIP(hipSetDevice(st->ctx->device));
  PCS_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  if (st->n * st->C == 0) return PCS_OK;
  return frame_status(st, required);
}

int pcs_state_capacity(const pcs_state* st, int64_t* capacity) {
  if (!st || !capacity) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  *capacity = st->capacity;
  return PCS_OK;
}

int pcs_context_set_wait_limit(pcs_context* ctx, uint32_t rounds) {
  if (!ctx) return fail(PCS_ERR_INVALID_ARG, "context is NULL");
  ctx->wait_limit = rounds;
  return PCS_OK;
}

int pcs_measure_lds_bandwidth(pcs_context* ctx, double* gbs, void* stream) {
  if (!ctx || !gbs) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int cus = 0;
  PCS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  const int blocks = 8 * std::max(cus, 1), iters = 2000;
  PCS_TRY(ensure(ctx, ctx->probe, (size_t)blocks * 256 * sizeof(float), "probe sink"));
  hipEvent_t a = nullptr, b = nullptr;
  PCS_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(PCS_ERR_HIP, "hipEventCreate failed");
  }
  hipError_t e = launch_lds_probe(blocks, iters / 10, ctx->probe.as<float>(), s);   // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch_lds_probe(blocks, iters, ctx->probe.as<float>(), s);
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(PCS_ERR_HIP, std::string("LDS probe: ") + hipGetErrorString(e));
  *gbs = (double)lds_probe_bytes(blocks, iters) / (ms * 1e-3) / 1e9;
  return PCS_OK;
}

int pcs_knn_pca(pcs_context* ctx, const float* xyz, int64_t n, int32_t k, float kappa,
                float floor_ratio, float* quat, float* scale, float* normal, float* nn_dist,
                void* stream) {
  if (!ctx) return fail(PCS_ERR_INVALID_ARG, "context is NULL");
  if (n < 0 || (n > 0 && (!xyz || !quat || !scale || !normal)))
    return fail(PCS_ERR_INVALID_ARG, "bad point buffers");
  if (k < 1 || k > 32) return fail(PCS_ERR_INVALID_ARG, "k must be in [1, 32]");
  if (n > 0 && k > n) return fail(PCS_ERR_INVALID_ARG, "k exceeds the number of points");
  if (nn_dist && k < 2) return fail(PCS_ERR_INVALID_ARG, "the nearest-neighbour distance needs k >= 2");
  if (!std::isfinite(kappa) || !std::isfinite(floor_ratio) || kappa <= 0.0f || floor_ratio < 0.0f)
    return fail(PCS_ERR_INVALID_ARG, "kappa must be positive and floor_ratio non-negative");
  if (n >= (int64_t(1) << 31)) return fail(PCS_ERR_UNSUPPORTED, "n must be below 2^31");
  if (n == 0) return PCS_OK;
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  PCS_TRY(ensure(ctx, ctx->knn_scratch, knn_scratch_bytes(n), "kNN scratch"));
  StageTimer tm(ctx, ST_KNN, s);
  PCS_HIP(launch_knn_pca(xyz, n, k, kappa, floor_ratio, quat, scale, normal, nn_dist, ctx->knn_scratch.p,
                         ctx->knn_scratch.cap, ctx->host_small + 192, s));
  return PCS_OK;
}

int pcs_shade(pcs_context* ctx, const pcs_images* in, const pcs_camera* cams, int32_t n_cams,
              const pcs_light* light, const float bg[3], float* out_rgb, void* stream) {
  if (!ctx || !in || !cams || !light || !out_rgb) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  if (!in->rgb || !in->normal || !in->alpha) return fail(PCS_ERR_INVALID_ARG, "shading needs rgb, normal and alpha");
  if (n_cams <= 0) return fail(PCS_ERR_INVALID_ARG, "need at least one camera");
  const int W = cams[0].width, H = cams[0].height;
  if (W <= 0 || H <= 0) return fail(PCS_ERR_INVALID_ARG, "image width and height must be positive");
  for (int c = 0; c < n_cams; ++c) {
    if (cams[c].width != W || cams[c].height != H)
      return fail(PCS_ERR_INVALID_ARG, "all cameras of one call must share width and height");
    if (!finite_camera(cams[c])) return fail(PCS_ERR_INVALID_ARG, "camera has non-finite or zero focal values");
  }
  const float dl = std::sqrt(light->dir[0] * light->dir[0] + light->dir[1] * light->dir[1] +
                             light->dir[2] * light->dir[2]);
  if (!(dl > 0.0f) || !std::isfinite(dl)) return fail(PCS_ERR_INVALID_ARG, "light direction must be non-zero");
  if (!(light->shininess > 0.0f)) return fail(PCS_ERR_INVALID_ARG, "shininess must be positive");
  DevLight L{};
  for (int k = 0; k < 3; ++k) {
    L.dir[k] = light->dir[k] / dl;
    L.color[k] = light->color[k];
    L.bg[k] = bg ? bg[k] : 0.0f;
  }
  L.ambient = light->ambient; L.diffuse = light->diffuse; L.specular = light->specular;
  L.shininess = light->shininess;
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<DevCamera> dc(n_cams);
  for (int c = 0; c < n_cams; ++c) dc[c] = to_dev(cams[c]);
  PCS_TRY(ensure(ctx, ctx->shade_cams, sizeof(DevCamera) * n_cams, "cameras"));
  PCS_HIP(hipMemcpyAsync(ctx->shade_cams.p, dc.data(), sizeof(DevCamera) * n_cams, hipMemcpyHostToDevice, s));
  StageTimer tm(ctx, ST_SHADE, s);
  PCS_HIP(launch_shade(W, H, n_cams, ctx->shade_cams.as<DevCamera>(), in->rgb, in->normal, in->alpha, L,
                       out_rgb, s));
  return PCS_OK;
}

int pcs_voxels_create(pcs_context* ctx, pcs_voxels** out) {
  if (!ctx || !out) return fail(PCS_ERR_INVALID_ARG, "context or out is NULL");
  *out = new pcs_voxels();
  (*out)->ctx = ctx;
  return PCS_OK;
}

void pcs_voxels_destroy(pcs_voxels* v) { delete v; }

namespace {
// with_features false (a pooled level): coordinates, point -> voxel map, starts and kernel map only;
// no features and no centroid
int voxelize_impl(pcs_context* ctx, const float* xyz, const float* rgb, int64_t n, int32_t grid,
                  pcs_voxels* vox, int64_t* n_voxels, void* stream, bool with_features) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!ctx || !vox || !n_voxels) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  if (grid < 2 || grid > 1024 || (grid & (grid - 1)) != 0)
    return fail(PCS_ERR_INVALID_ARG, "grid must be a power of two in [2, 1024]");
  if (vox->ctx != ctx) return fail(PCS_ERR_INVALID_ARG, "voxels belong to another context");
  if (n <= 0 || !xyz || !rgb) return fail(PCS_ERR_INVALID_ARG, "need at least one point");
  if (n >= (int64_t(1) << 30)) return fail(PCS_ERR_UNSUPPORTED, "n must be below 2^30");
  PCS_HIP(hipSetDevice(ctx->device));
  vox->valid = false;
  vox->pooled = false;
  PCS_TRY(ensure(ctx, vox->keys, n * sizeof(uint32_t), "voxel keys"));
  PCS_TRY(ensure(ctx, vox->order, n * sizeof(uint32_t), "voxel point order"));
  PCS_TRY(ensure(ctx, ctx->keys_alt, n * sizeof(uint32_t), "keys (alternate)"));
  PCS_TRY(ensure(ctx, ctx->vals_alt, n * sizeof(uint32_t), "values (alternate)"));
  PCS_TRY(ensure(ctx, ctx->sort_scratch, sort_scratch_bytes(n), "sort scratch"));
  PCS_TRY(ensure(ctx, vox->flag, n * sizeof(uint32_t), "voxel flags"));
  PCS_TRY(ensure(ctx, vox->excl, n * sizeof(uint32_t) + 64, "voxel numbering"));
  PCS_TRY(ensure(ctx, ctx->scan_scratch, scan_scratch_bytes(n), "scan scratch"));
  PCS_TRY(ensure(ctx, ctx->small, kSmallWords * 4, "small"));
  PCS_TRY(ensure(ctx, vox->point_voxel, n * sizeof(int32_t), "point to voxel map"));
  PCS_TRY(ensure(ctx, vox->centroid, 64, "centroid"));
  StageTimer tm(ctx, ST_VOXELIZE, s);
  uint32_t* d_err = ctx->small.as<uint32_t>() + kVoxErrWord;
  PCS_HIP(launch_fill_u32(d_err, 0u, 1, s));
  PCS_HIP(launch_vox_keys(xyz, n, grid, vox->keys.as<uint32_t>(), vox->order.as<uint32_t>(), s));
  bool in_alt = false;
  PCS_HIP(launch_sort(vox->keys.as<uint32_t>(), vox->order.as<uint32_t>(), ctx->keys_alt.as<uint32_t>(),
                      ctx->vals_alt.as<uint32_t>(), n, 3 * grid_bits(grid), ctx->sort_scratch.p, s, &in_alt, nullptr, false,
                      false, nullptr, 0, -1, nullptr, 0, d_err, ctx->wait_limit));
  if (in_alt) {
    swap_buf(vox->keys, ctx->keys_alt);
    swap_buf(vox->order, ctx->vals_alt);
  }
  PCS_HIP(launch_vox_flags(vox->keys.as<uint32_t>(), n, vox->flag.as<uint32_t>(), s));
  uint64_t* d_total = ctx->small.as<uint64_t>();
  PCS_HIP(launch_scan(vox->flag.as<uint32_t>(), nullptr, nullptr, nullptr, vox->excl.as<uint32_t>(), n, d_total,
                      ctx->scan_scratch.p, s, false, d_err, ctx->wait_limit));
  PCS_HIP(hipMemcpyAsync(ctx->host_small, d_total, 8, hipMemcpyDeviceToHost, s));
  PCS_HIP(hipMemcpyAsync(ctx->host_small + 2, d_err, 4, hipMemcpyDeviceToHost, s));
  PCS_HIP(hipStreamSynchronize(s));
  if (ctx->host_small[2] != 0u)
    return fail(PCS_ERR_HIP, "a look-back wait of the voxel sort or numbering ran out (broken launch)");
  uint64_t V;
  std::memcpy(&V, ctx->host_small, 8);
  int log2cap = 6;
  while ((int64_t(1) << log2cap) < (int64_t)(2 * V)) ++log2cap;
  PCS_TRY(ensure(ctx, vox->start, V * sizeof(uint32_t) + 64, "voxel starts"));
  PCS_TRY(ensure(ctx, vox->coords, 3 * V * sizeof(int32_t), "voxel coordinates"));
  PCS_TRY(ensure(ctx, vox->feat, V * 32 * sizeof(uint16_t), "voxel features"));
  PCS_TRY(ensure(ctx, vox->hkeys, (size_t(1) << log2cap) * sizeof(uint32_t), "voxel hash keys"));
  PCS_TRY(ensure(ctx, vox->hvals, (size_t(1) << log2cap) * sizeof(int32_t), "voxel hash values"));
  PCS_TRY(ensure(ctx, vox->nbr, 27 * V * sizeof(int32_t), "kernel map"));
  PCS_HIP(launch_vox_build(vox->keys.as<uint32_t>(), vox->order.as<uint32_t>(), vox->flag.as<uint32_t>(),
                           vox->excl.as<uint32_t>(), n, (int64_t)V, xyz, rgb, grid, vox->start.as<uint32_t>(),
                           vox->coords.as<int32_t>(), with_features ? vox->feat.as<uint16_t>() : nullptr,
                           vox->point_voxel.as<int32_t>(), vox->hkeys.as<uint32_t>(),
                           vox->hvals.as<int32_t>(), log2cap, vox->nbr.as<int32_t>(), s));
  if (with_features) PCS_HIP(launch_centroid(xyz, n, vox->centroid.as<double>(), vox->centroid.as<float>() + 8, s));
  vox->n = n;
  vox->V = (int64_t)V;
  vox->log2cap = log2cap;
  vox->grid = grid;
  vox->valid = true;
  *n_voxels = (int64_t)V;
  return PCS_OK;
}
}  // namespace

int pcs_voxelize(pcs_context* ctx, const float* xyz, const float* rgb, int64_t n, int32_t grid,
                 pcs_voxels* vox, int64_t* n_voxels, void* stream) {
  return voxelize_impl(ctx, xyz, rgb, n, grid, vox, n_voxels, stream, true);
}

int pcs_voxels_get(const pcs_voxels* vox, const int32_t** coords, const int32_t** nbr,
                   const int32_t** point_voxel, const uint16_t** features, int64_t* n_voxels) {
  if (!vox || !vox->valid) return fail(PCS_ERR_INVALID_ARG, "voxels hold no completed voxelisation");
  if (coords) *coords = vox->coords.as<int32_t>();
  if (nbr) *nbr = vox->nbr.as<int32_t>();
  if (point_voxel) *point_voxel = vox->point_voxel.as<int32_t>();
  if (features) *features = vox->feat.as<uint16_t>();
  if (n_voxels) *n_voxels = vox->V;
  return PCS_OK;
}

int pcs_subm_conv_forward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* x, int32_t cin,
                          const uint16_t* w, const float* bias, int32_t cout, int32_t relu, uint16_t* y,
                          void* stream) {
  if (!ctx || !vox || !vox->valid || !x || !w || !y) return fail(PCS_ERR_INVALID_ARG, "NULL argument or empty voxels");
  if (!conv_shape_supported(cin, cout)) return fail(PCS_ERR_UNSUPPORTED, "channels must be 32 or 64");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_CONV, s);
  PCS_HIP(launch_subm_conv(x, cin, w, bias, cout, vox->nbr.as<int32_t>(), vox->V, relu ? 1 : 0, y, s));
  return PCS_OK;
}

int pcs_subm_conv_forward_cat(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* x1, int32_t c1,
                              const uint16_t* x2, int32_t c2, const uint16_t* w, const float* bias,
                              int32_t cout, int32_t relu, uint16_t* y, void* stream) {
  if (!ctx || !vox || !vox->valid || !x1 || !x2 || !w || !y) return fail(PCS_ERR_INVALID_ARG, "NULL argument or empty voxels");
  if (c1 != c2 || c1 % 32 != 0 || c1 <= 0 || !conv_shape_supported(c1 + c2, cout))
    return fail(PCS_ERR_UNSUPPORTED, "the halves must be equal multiples of 32, with c1 + c2 and cout supported");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_CONV, s);
  PCS_HIP(launch_subm_conv(x1, c1 + c2, w, bias, cout, vox->nbr.as<int32_t>(), vox->V, relu ? 1 : 0, y, s,
                           27, x2, c1));
  return PCS_OK;
}

int pcs_subm_conv_backward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* x, int32_t cin,
                           const uint16_t* w, int32_t cout, const uint16_t* y, const uint16_t* dy,
                           uint16_t* dx, float* dw, float* dbias, void* stream) {
  if (!ctx || !vox || !vox->valid || !x || !w || !dy) return fail(PCS_ERR_INVALID_ARG, "NULL argument or empty voxels");
  if (!conv_shape_supported(cin, cout)) return fail(PCS_ERR_UNSUPPORTED, "channels must be 32 or 64");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_CONV_BWD, s);
  const uint16_t* g = dy;
  if (y) {
    PCS_TRY(ensure(ctx, ctx->conv_tmp, (size_t)vox->V * cout * sizeof(uint16_t), "masked output gradient"));
    PCS_HIP(launch_relu_mask(y, dy, vox->V * cout, ctx->conv_tmp.as<uint16_t>(), s));
    g = ctx->conv_tmp.as<uint16_t>();
  }
  if (dbias) PCS_HIP(launch_bias_grad(g, vox->V, cout, dbias, s));
  if (dw) PCS_HIP(launch_subm_conv_dw(x, cin, g, cout, vox->nbr.as<int32_t>(), vox->V, dw, s));
  if (dx) {
    PCS_TRY(ensure(ctx, ctx->wt_tmp, (size_t)27 * cin * cout * sizeof(uint16_t), "transposed weights"));
    PCS_HIP(launch_weight_t(w, 27, cin, cout, true, ctx->wt_tmp.as<uint16_t>(), s));
    PCS_HIP(launch_subm_conv(g, cout, ctx->wt_tmp.as<uint16_t>(), nullptr, cin, vox->nbr.as<int32_t>(),
                             vox->V, 0, dx, s));
  }
  return PCS_OK;
}

int pcs_pool(pcs_context* ctx, const pcs_voxels* child, pcs_voxels* parent, int64_t* n_parents,
             void* stream) {
  if (!ctx || !child || !parent || !n_parents) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  if (!child->valid || child->ctx != ctx || parent->ctx != ctx)
    return fail(PCS_ERR_INVALID_ARG, "child voxels empty or of another context");
  if (child == parent) return fail(PCS_ERR_INVALID_ARG, "parent and child must be different objects");
  if (child->grid < 2) return fail(PCS_ERR_INVALID_ARG, "a grid of one voxel has no coarser level");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t Vc = child->V;
  // the child voxels' centres, voxelised on the grid of half the resolution, give the parents
  PCS_TRY(ensure(ctx, parent->centres, 3 * Vc * sizeof(float), "child voxel centres"));
  PCS_HIP(launch_voxel_centres(child->coords.as<int32_t>(), Vc, child->grid, parent->centres.as<float>(), s));
  PCS_TRY(voxelize_impl(ctx, parent->centres.as<float>(), parent->centres.as<float>(), Vc, child->grid / 2,
                        parent, n_parents, stream, false));
  PCS_TRY(ensure(ctx, parent->up_fwd, 8 * Vc * sizeof(int32_t), "upsampling table"));
  PCS_TRY(ensure(ctx, parent->up_bwd, 8 * parent->V * sizeof(int32_t), "upsampling adjoint table"));
  PCS_HIP(launch_up_tables(child->coords.as<int32_t>(), parent->point_voxel.as<int32_t>(), Vc, parent->V,
                           parent->up_fwd.as<int32_t>(), parent->up_bwd.as<int32_t>(), s));
  parent->pooled = true;
  return PCS_OK;
}

int pcs_pool_features(pcs_context* ctx, const pcs_voxels* parent, const uint16_t* child_feat, int32_t channels,
                      uint16_t* parent_feat, void* stream) {
  if (!ctx || !parent || !child_feat || !parent_feat) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  if (!parent->valid || !parent->pooled) return fail(PCS_ERR_INVALID_ARG, "voxels are not a pooled level");
  if (channels != 32 && channels != 64 && channels != 128) return fail(PCS_ERR_UNSUPPORTED, "channels must be 32, 64 or 128");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_CONV, s);
  PCS_HIP(launch_pool_features(parent->order.as<uint32_t>(), parent->start.as<uint32_t>(), parent->V, parent->n,
                               child_feat, channels, parent_feat, s));
  return PCS_OK;
}

int pcs_pool_features_backward(pcs_context* ctx, const pcs_voxels* parent, const uint16_t* d_parent,
                               int32_t channels, uint16_t* d_child, void* stream) {
  if (!ctx || !parent || !d_parent || !d_child) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  if (!parent->valid || !parent->pooled) return fail(PCS_ERR_INVALID_ARG, "voxels are not a pooled level");
  if (channels != 32 && channels != 64 && channels != 128) return fail(PCS_ERR_UNSUPPORTED, "channels must be 32, 64 or 128");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_CONV_BWD, s);
  PCS_HIP(launch_pool_features_bwd(parent->point_voxel.as<int32_t>(), parent->start.as<uint32_t>(), parent->V,
                                   parent->n, d_parent, channels, d_child, s));
  return PCS_OK;
}

int pcs_up_conv_forward(pcs_context* ctx, const pcs_voxels* parent, const uint16_t* x, int32_t cin,
                        const uint16_t* w, const float* bias, int32_t cout, int32_t relu, uint16_t* y,
                        void* stream) {
  if (!ctx || !parent || !x || !w || !y) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  if (!parent->valid || !parent->pooled) return fail(PCS_ERR_INVALID_ARG, "voxels are not a pooled level");
  if (!conv_shape_supported(cin, cout)) return fail(PCS_ERR_UNSUPPORTED, "unsupported channel counts");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_CONV, s);
  // child j: y_j = W_{k(j)} x_{parent(j)}, the gather-GEMM over the 8-offset upsampling table
  PCS_HIP(launch_subm_conv(x, cin, w, bias, cout, parent->up_fwd.as<int32_t>(), parent->n, relu ? 1 : 0, y, s, 8));
  return PCS_OK;
}

int pcs_up_conv_backward(pcs_context* ctx, const pcs_voxels* parent, const uint16_t* x, int32_t cin,
                         const uint16_t* w, int32_t cout, const uint16_t* y, const uint16_t* dy,
                         uint16_t* dx, float* dw, float* dbias, void* stream) {
  if (!ctx || !parent || !x || !w || !dy) return fail(PCS_ERR_INVALID_ARG, "NULL argument");
  if (!parent->valid || !parent->pooled) return fail(PCS_ERR_INVALID_ARG, "voxels are not a pooled level");
  if (!conv_shape_supported(cin, cout) || !conv_shape_supported(cout, cin))
    return fail(PCS_ERR_UNSUPPORTED, "unsupported channel counts");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_CONV_BWD, s);
  const int64_t Vc = parent->n;
  const uint16_t* g = dy;
  if (y) {
    PCS_TRY(ensure(ctx, ctx->conv_tmp, (size_t)Vc * cout * sizeof(uint16_t), "masked output gradient"));
    PCS_HIP(launch_relu_mask(y, dy, Vc * cout, ctx->conv_tmp.as<uint16_t>(), s));
    g = ctx->conv_tmp.as<uint16_t>();
  }
  if (dbias) PCS_HIP(launch_bias_grad(g, Vc, cout, dbias, s));
  if (dw) PCS_HIP(launch_subm_conv_dw(x, cin, g, cout, parent->up_fwd.as<int32_t>(), Vc, dw, s, 8));
  if (dx) {
    // parent p: dx_p = sum_k W_k^T dy_{child_k(p)} over the adjoint table
    PCS_TRY(ensure(ctx, ctx->wt_tmp, (size_t)8 * cin * cout * sizeof(uint16_t), "transposed weights"));
    PCS_HIP(launch_weight_t(w, 8, cin, cout, false, ctx->wt_tmp.as<uint16_t>(), s));
    PCS_HIP(launch_subm_conv(g, cout, ctx->wt_tmp.as<uint16_t>(), nullptr, cin, parent->up_bwd.as<int32_t>(),
                             parent->V, 0, dx, s, 8));
  }
  return PCS_OK;
}

int pcs_unet_head_forward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* feat, const float* w1,
                          const float* b1, const float* w2, const float* b2, const float* xyz,
                          const float* rgb, float* mean, float* quat, float* scale, float* opacity,
                          float* out_rgb, float* normal, void* stream) {
  if (!ctx || !vox || !vox->valid || !feat || !w1 || !b1 || !w2 || !b2 || !xyz || !rgb || !mean || !quat ||
      !scale || !opacity || !out_rgb || !normal)
    return fail(PCS_ERR_INVALID_ARG, "NULL argument or empty voxels");
  if (vox->pooled) return fail(PCS_ERR_INVALID_ARG, "the head takes the voxels of the points, not a pooled level");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_HEAD, s);
  PCS_HIP(launch_mlp_points(feat, vox->coords.as<int32_t>(), vox->V, vox->point_voxel.as<int32_t>(), w1, b1, w2,
                            b2, xyz, rgb, vox->n, vox->grid, mean, quat, scale, opacity, out_rgb, normal, s));
  return PCS_OK;
}

int pcs_unet_head_backward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* feat, const float* w1,
                           const float* b1, const float* w2, const float* b2, const float* xyz,
                           const float* d_mean, const float* d_quat, const float* d_scale, const float* d_opacity,
                           const float* d_normal, uint16_t* d_feat, float* d_w1, float* d_b1, float* d_w2,
                           float* d_b2, void* stream) {
  if (!ctx || !vox || !vox->valid || !feat || !w1 || !b1 || !w2 || !b2 || !xyz || !d_feat || !d_w1 || !d_b1 ||
      !d_w2 || !d_b2)
    return fail(PCS_ERR_INVALID_ARG, "NULL argument or empty voxels");
  if (vox->pooled) return fail(PCS_ERR_INVALID_ARG, "the head takes the voxels of the points, not a pooled level");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_HEAD_BWD, s);
  pcs_voxels* v = const_cast<pcs_voxels*>(vox);
  PCS_TRY(ensure(ctx, v->head_gh, (size_t)std::max<int64_t>(vox->n, 1) * 32 * sizeof(float),
                 "head hidden-layer gradients"));
  PCS_HIP(launch_mlp_backward(feat, vox->coords.as<int32_t>(), vox->V, vox->point_voxel.as<int32_t>(),
                              vox->order.as<uint32_t>(), vox->start.as<uint32_t>(), w1, b1, w2, b2, xyz, vox->n,
                              vox->grid, d_mean, d_quat, d_scale, d_opacity, d_normal, v->head_gh.as<float>(),
                              d_feat, d_w1, d_b1, d_w2, d_b2, s));
  return PCS_OK;
}

int pcs_estimator_head_forward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* feat,
                               const float* wh, const float* bh, const float* xyz, const float* rgb,
                               float* quat, float* scale, float* opacity, float* out_rgb,
                               float* normal, void* stream) {
  if (!ctx || !vox || !vox->valid || !feat || !wh || !bh || !xyz || !rgb || !quat || !scale ||
      !opacity || !out_rgb || !normal)
    return fail(PCS_ERR_INVALID_ARG, "NULL argument or empty voxels");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_HEAD, s);
  PCS_HIP(launch_head_forward(feat, wh, bh, vox->point_voxel.as<int32_t>(), xyz, rgb,
                              vox->centroid.as<float>() + 8, vox->n, 2.0f / (float)vox->grid, quat,
                              scale, opacity, out_rgb, normal, s));
  return PCS_OK;
}

int pcs_estimator_head_backward(pcs_context* ctx, const pcs_voxels* vox, const uint16_t* feat,
                                const float* wh, const float* bh, const float* d_quat,
                                const float* d_scale, const float* d_opacity, const float* d_rgb,
                                uint16_t* d_feat, float* d_wh, float* d_bh, void* stream) {
  if (!ctx || !vox || !vox->valid || !feat || !wh || !bh || !d_quat || !d_scale || !d_opacity ||
      !d_rgb || !d_feat || !d_wh || !d_bh)
    return fail(PCS_ERR_INVALID_ARG, "NULL argument or empty voxels");
  PCS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageTimer tm(ctx, ST_HEAD_BWD, s);
  PCS_HIP(launch_head_backward(feat, wh, bh, vox->order.as<uint32_t>(), vox->start.as<uint32_t>(),
                               vox->V, vox->n, 2.0f / (float)vox->grid, d_quat, d_scale, d_opacity, d_rgb,
                               d_feat, d_wh, d_bh, s));
  return PCS_OK;
}

}  // extern "C"
