// Instance ordering: depth sort of the projected splats, prefix sum of their tile counts in that
// order, tile-key emission, stable tile sort and tile ranges.
//
//  * scan:     single-pass exclusive prefix sum with decoupled look-back (Merrill & Garland,
//              "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016), optionally
//              reading its input through a permutation. Block b scans partition b: blocks are
//              dispatched in index order on each XCD, so every partition a block waits on
//              belongs to a block that is already running or done. The look-back reads 64
//              predecessors per step, one per lane of a wavefront; its spin is bounded.
//  * depth keys / binning: the (camera, depth) order of the splats is found by sorting one key per
//              (camera, Gaussian); each visible splat then writes its tile keys, in rectangle order,
//              at its offset in that order. A stable sort by tile afterwards leaves every tile's
//              run in (depth, Gaussian index) order: the (tile, depth, index) order of Section 3.1
//              with the deep key sort done over splats rather than over their tile instances.
//  * sort:     Onesweep-style LSD radix sort (Adinets & Merrill, "Onesweep: A Faster Least
//              Significant Digit Radix Sort for GPUs", 2022) on 32- or 64-bit keys: one histogram
//              pass over all digits, then one chained-scan scatter per 8-bit digit. Ranks inside a
//              wavefront come from eight ballots (lanes holding the same digit), so the sort is
//              stable; each block reorders its 4096 keys through LDS so global writes leave in
//              digit runs. The chained scan looks back in two levels: the last partition of each
//              group of 32 publishes the group's digit totals as soon as it has read the group, so
//              a look-back crosses earlier groups one status row per group.
//  * ranges:   tile start/end from tile-id changes in the sorted keys.
//
// Depth keys are fp32 depth bits - minimum depth bits over all cameras: positive floats order
// like their bit patterns, so only the significant bits are sorted.

#include "pcs_internal.hpp"

namespace pcs {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kPart = kThreads * kItems;   // 4096 elements per partition
constexpr int kWaves = kThreads / kWave;

// ---- scan -----------------------------------------------------------------------------------
constexpr uint64_t kScanAgg = 1ull << 62;
constexpr uint64_t kScanPrefix = 2ull << 62;
constexpr uint64_t kScanValue = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kBins = 256;

__device__ __forceinline__ uint64_t atomic_load_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_load_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The frame's error word (null: none kept): a kernel whose input a failed stage produced returns
// at once.
__device__ __forceinline__ bool frame_failed(const uint32_t* err) {
  return err && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

__device__ __forceinline__ void flag_error(uint32_t* err, uint32_t bits) {
  if (err) atomicOr(err, bits);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__global__ __launch_bounds__(kThreads) void k_scan(const uint32_t* __restrict__ in,
                                                   const uint32_t* __restrict__ gather0,
                                                   const uint32_t* __restrict__ gather1,
                                                   const uint32_t* __restrict__ sel,
                                                   uint32_t* __restrict__ out, int64_t n,
                                                   int64_t n_parts, uint64_t* __restrict__ status,
                                                   uint64_t* __restrict__ total,
                                                   uint32_t* __restrict__ err, uint32_t spin_limit) {
  __shared__ uint64_t s_wave[kWaves];
  __shared__ uint64_t s_excl;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int64_t part = blockIdx.x;    // in-order dispatch: predecessors are running or done
  const int64_t base = part * kPart + (int64_t)tid * kItems;
  const uint32_t* gather = (sel && (*sel & 1u)) ? gather1 : gather0;
  uint32_t x[kItems];
  if (gather) {
#pragma unroll
    for (int k = 0; k < kItems; ++k) x[k] = (base + k < n) ? in[gather[base + k]] : 0u;
  } else if (base + kItems <= n) {
    const uint4* src = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
    for (int q = 0; q < kItems / 4; ++q) {
      uint4 w = src[q];
      x[4 * q + 0] = w.x; x[4 * q + 1] = w.y; x[4 * q + 2] = w.z; x[4 * q + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kItems; ++k) x[k] = (base + k < n) ? in[base + k] : 0u;
  }
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) sum += x[k];
  const uint64_t incl = wave_inclusive_scan64(sum);
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint64_t wave_prefix = 0, block_total = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wave) wave_prefix += s_wave[w];
    block_total += s_wave[w];
  }
  if (wave == 0) {
    uint64_t excl = 0;
    if (part == 0) {
      if (lane == 0) atomic_store_u64(&status[0], kScanPrefix | block_total);
    } else {
      if (lane == 0) atomic_store_u64(&status[part], kScanAgg | block_total);
      int64_t p = part - 1;
      uint32_t spins = 0;
      while (true) {
        const int64_t idx = p - lane;
        const uint64_t v = idx >= 0 ? atomic_load_u64(&status[idx]) : kScanPrefix;
        const uint64_t flag = v & ~kScanValue;
        const uint64_t pre = __ballot(flag == kScanPrefix);
        const uint64_t zero = __ballot(flag == 0);
        const int first = pre ? __ffsll((unsigned long long)pre) - 1 : kWave;
        const uint64_t need = first < kWave ? (first == 63 ? ~0ull : ((2ull << first) - 1)) : ~0ull;
        // a predecessor has not published yet; a wait that runs out (a broken launch) marks the
        // result as failed and goes on with what it has, so the kernel still ends
        if (zero & need) {
          if (++spins < spin_limit) continue;
          if (lane == 0) flag_error(err, kErrSpin);
        }
        excl += wave_sum_u64(lane <= first ? (v & kScanValue) : 0ull);
        if (first < kWave) break;
        p -= kWave;
      }
      if (lane == 0) atomic_store_u64(&status[part], kScanPrefix | (excl + block_total));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  uint64_t running = s_excl + wave_prefix + incl - sum;
  if (base + kItems <= n) {
    uint32_t y[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) { y[k] = (uint32_t)running; running += x[k]; }
    uint4* dst = reinterpret_cast<uint4*>(out + base);
#pragma unroll
    for (int q = 0; q < kItems / 4; ++q)
      dst[q] = make_uint4(y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < kItems; ++k)
      if (base + k < n) { out[base + k] = (uint32_t)running; running += x[k]; }
  }
  if (part == n_parts - 1 && tid == 0) *total = s_excl + block_total;
}

// ---- depth keys and binning ----------------------------------------------------------------
// One key per (camera, Gaussian); culled splats get all bits set (they have no tile instances,
// so where they land in the order does not matter).
// Tile count of a rectangle (x0 | x_end << 16, y0 | y_end << 16); zero for a culled splat.
__device__ __forceinline__ uint32_t rect_count(uint2 r) {
  return ((r.x >> 16) - (r.x & 0xFFFFu)) * ((r.y >> 16) - (r.y & 0xFFFFu));
}

// Binning fused with the prefix sum that places it. Block b takes positions
// [kBinPart b, kBinPart (b + 1)) of the depth order (kBinItems per thread): their tile counts, the
// block's scan and a decoupled look-back (as in k_scan) give each position its offset. The block
// then writes its keys in output order, kBinSlots slots per thread per step, consecutive threads
// on consecutive slots (coalesced, and balanced whatever the splat sizes): a binary search over
// the block's offsets finds the position whose rectangle holds slot p, and the slot's rank inside
// that rectangle gives the tile (row-major). The keys' digits are counted in LDS and added to one
// of kTileHistCopies copies.
constexpr int kBinItems = 4;
constexpr int kBinPart = kThreads * kBinItems;   // 1024 positions per block
constexpr int kBinSlots = 4;                      // output slots searched together per thread

__global__ __launch_bounds__(kThreads) void k_scan_bin(
    int64_t total, uint32_t n, int TX, uint32_t tiles_per_cam, const uint32_t* __restrict__ order0,
    const uint32_t* __restrict__ order1, const uint32_t* __restrict__ passes,
    const uint2* __restrict__ rect, bool narrow_rect, int64_t n_parts, uint64_t* __restrict__ status,
    uint64_t* __restrict__ instances, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
    int n_digits, uint32_t* __restrict__ hist, ClearSpans clear, uint32_t* __restrict__ err,
    uint32_t spin_limit, uint64_t capacity) {
  __shared__ uint32_t s_off[kBinPart];          // block-relative offset of each position
  __shared__ uint32_t s_idx[kBinPart];          // its (camera, Gaussian) entry
  __shared__ uint2 s_rect[kBinPart];
  __shared__ uint32_t sh[kTileHistPasses][kBins];
  __shared__ uint64_t s_wave[kWaves];
  __shared__ uint64_t s_excl;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  clear_spans(clear, (int64_t)blockIdx.x * kThreads + tid, (int64_t)gridDim.x * kThreads);
  if (frame_failed(err)) return;          // the depth order is not valid: nothing to place
  for (int d = 0; d < kTileHistPasses; ++d) sh[d][tid] = 0u;
  const int64_t part = blockIdx.x;    // in-order dispatch: predecessors are running or done
  const int64_t base = part * kBinPart + (int64_t)tid * kBinItems;
  const uint32_t* order = (*passes & 1u) ? order1 : order0;   // where the depth sort ended
  uint32_t idx[kBinItems], cnt[kBinItems];
  uint2 r[kBinItems];
#pragma unroll
  for (int k = 0; k < kBinItems; ++k) idx[k] = base + k < total ? order[base + k] : 0u;
#pragma unroll
  for (int k = 0; k < kBinItems; ++k) {
    r[k] = base + k < total ? load_rect(rect, idx[k], narrow_rect) : make_uint2(0u, 0u);
    cnt[k] = rect_count(r[k]);
  }
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kBinItems; ++k) sum += cnt[k];
  const uint64_t incl = wave_inclusive_scan64(sum);
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint64_t wave_prefix = 0, block_total = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wave) wave_prefix += s_wave[w];
    block_total += s_wave[w];
  }
  {
    uint32_t running = (uint32_t)(wave_prefix + incl - sum);
#pragma unroll
    for (int k = 0; k < kBinItems; ++k) {
      const int j = tid * kBinItems + k;
      s_off[j] = running;
      s_idx[j] = idx[k];
      s_rect[j] = r[k];
      running += cnt[k];
    }
  }
  if (wave == 0) {
    uint64_t excl = 0;
    if (part == 0) {
      if (lane == 0) atomic_store_u64(&status[0], kScanPrefix | block_total);
    } else {
      if (lane == 0) atomic_store_u64(&status[part], kScanAgg | block_total);
      int64_t p = part - 1;
      uint32_t spins = 0;
      while (true) {
        const int64_t q = p - lane;
        const uint64_t v = q >= 0 ? atomic_load_u64(&status[q]) : kScanPrefix;
        const uint64_t flag = v & ~kScanValue;
        const uint64_t pre = __ballot(flag == kScanPrefix);
        const uint64_t zero = __ballot(flag == 0);
        const int first = pre ? __ffsll((unsigned long long)pre) - 1 : kWave;
        const uint64_t need = first < kWave ? (first == 63 ? ~0ull : ((2ull << first) - 1)) : ~0ull;
        // a predecessor has not published yet; a wait that runs out (a broken launch) marks the
        // frame as failed and goes on with what it has, so the kernel still ends
        if (zero & need) {
          if (++spins < spin_limit) continue;
          if (lane == 0) flag_error(err, kErrSpin);
        }
        excl += wave_sum_u64(lane <= first ? (v & kScanValue) : 0ull);
        if (first < kWave) break;
        p -= kWave;
      }
      if (lane == 0) atomic_store_u64(&status[part], kScanPrefix | (excl + block_total));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  const uint64_t out0 = s_excl;
  const uint32_t bt = (uint32_t)block_total;
  for (uint32_t p0 = tid; p0 < bt; p0 += kThreads * kBinSlots) {
    // per slot: the last position whose offset is <= p (offsets never decrease, and that
    // position's count is > 0); the kBinSlots searches run interleaved
    int j[kBinSlots];
#pragma unroll
    for (int t = 0; t < kBinSlots; ++t) j[t] = 0;
#pragma unroll
    for (int step = kBinPart / 2; step >= 1; step >>= 1)
#pragma unroll
      for (int t = 0; t < kBinSlots; ++t)
        if (s_off[j[t] + step] <= p0 + t * kThreads) j[t] += step;
#pragma unroll
    for (int t = 0; t < kBinSlots; ++t) {
      const uint32_t p = p0 + t * kThreads;
      if (p >= bt) break;
      const uint32_t local = p - s_off[j[t]];
      const uint2 rr = s_rect[j[t]];
      const uint32_t x0 = rr.x & 0xFFFFu, w = (rr.x >> 16) - x0, y0 = rr.y & 0xFFFFu;
      const uint32_t dy = local / w, dx = local - dy * w;
      const uint32_t i = s_idx[j[t]];
      const uint32_t cam = i / n;
      const uint32_t key = cam * tiles_per_cam + (y0 + dy) * (uint32_t)TX + x0 + dx;
      if (out0 + p >= capacity) break;           // beyond a fixed capacity: counted, not written
      keys[out0 + p] = key;
      vals[out0 + p] = i - cam * n;
      for (int d = 0; d < n_digits; ++d) atomicAdd(&sh[d][(key >> (8 * d)) & 0xFF], 1u);
    }
  }
  __syncthreads();
  uint32_t* h = hist + (blockIdx.x % kTileHistCopies) * (kTileHistPasses * kBins);
  for (int d = 0; d < n_digits; ++d) {
    const uint32_t v = sh[d][tid];
    if (v) atomicAdd(&h[d * kBins + tid], v);
  }
  if (part == n_parts - 1 && tid == 0) {
    *instances = out0 + block_total;
    if (out0 + block_total > capacity) flag_error(err, kErrCapacity);
  }
}

// ---- radix sort -----------------------------------------------------------------------------
constexpr int kMaxPasses = 8;
constexpr uint32_t kSortAgg = 1u << 30;
constexpr uint32_t kSortPrefix = 2u << 30;
constexpr uint32_t kSortValue = (1u << 30) - 1;
constexpr int kLookWindow = 32;
// Partitions per look-back group: the group's last partition publishes the group's digit total
// (or its inclusive prefix) in a second status row, so a look-back walks over groups, not
// partitions, once it has left its own group.
constexpr int kGroupParts = kLookWindow;
constexpr int kHistBlocks = 256;

// Digit histograms of every pass in one read of the keys. Each block takes partitions of 4096 keys
// (16 per thread, all loads issued before any is used). Lanes of a wavefront holding the same digit
// are matched with eight ballots and their count is added once, so the long runs of equal digits
// cost one LDS atomic per run.
template <typename K>
__global__ __launch_bounds__(256) void k_radix_hist(const K* __restrict__ keys, int64_t m,
                                                    int n_passes, uint32_t* __restrict__ hist) {
  __shared__ uint32_t sh[kMaxPasses][kBins];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (int p = 0; p < kMaxPasses; ++p) sh[p][tid] = 0;
  __syncthreads();
  const uint64_t lt_mask = lanemask_lt();
  for (int64_t part = blockIdx.x; part * kPart < m; part += gridDim.x) {
    const int64_t wbase = part * kPart + (int64_t)wave * (kWave * kItems);
    K k[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const int64_t pos = wbase + (int64_t)it * kWave + lane;
      k[it] = pos < m ? keys[pos] : (K)0;
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const bool valid = wbase + (int64_t)it * kWave + lane < m;
      const uint64_t vmask = __ballot(valid);
      if (vmask == 0) break;
      for (int p = 0; p < n_passes; ++p) {
        const uint32_t d = (uint32_t)(k[it] >> (8 * p)) & 0xFF;
        if (p < n_passes - 1) {                       // lower digits: spread, one atomic per key
          if (valid) atomicAdd(&sh[p][d], 1u);
          continue;
        }
        // top digit: few distinct values in a wavefront (sorted runs), so equal digits are
        // matched with eight ballots and counted once
        uint64_t peers = vmask;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const bool bit = (d >> b) & 1u;
          const uint64_t bal = __ballot(bit);
          peers &= bit ? bal : ~bal;
        }
        if (valid && (peers & lt_mask) == 0) atomicAdd(&sh[p][d], (uint32_t)__popcll(peers));
      }
    }
  }
  __syncthreads();
  for (int p = 0; p < n_passes; ++p) {
    const uint32_t v = sh[p][tid];
    if (v) atomicAdd(&hist[p * kBins + tid], v);
  }
}

// Depth keys and their digit histograms in one pass (the key of entry j, over all cameras, is the
// bits of its depth above the frame's minimum, or all ones for a culled splat; its value is j).
// The depth-bit range comes from the projection's slots; block 0 also records the pass count.
// The histograms of the four 8-bit digits go to hist[4][256] (zeroed beforehand).
__global__ __launch_bounds__(256) void k_depth_keys_hist(int64_t m, const uint32_t* __restrict__ zbits,
                                                         const unsigned long long* __restrict__ count_slots,
                                                         unsigned long long* __restrict__ host_word,
                                                         uint32_t seq,
                                                         const uint32_t* __restrict__ zrange,
                                                         uint32_t* __restrict__ info,
                                                         uint32_t* __restrict__ keys,
                                                         uint32_t* __restrict__ vals,
                                                         uint32_t* __restrict__ hist) {
  constexpr int kDigits = 4;
  constexpr int kDkItems = 4;
  constexpr int kDkPart = kThreads * kDkItems;
  __shared__ uint32_t sh[kDigits][kBins];
  __shared__ uint32_t s_z[2];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  // the first partition's depth bits are requested before the depth range is reduced, so the two
  // round trips overlap
  uint32_t zb[kDkItems];
  auto load_bits = [&](int64_t part) {
    const int64_t wbase = part * kDkPart + (int64_t)wave * (kWave * kDkItems);
#pragma unroll
    for (int it = 0; it < kDkItems; ++it) {
      const int64_t pos = wbase + (int64_t)it * kWave + lane;
      zb[it] = pos < m ? zbits[pos] : 0u;
    }
  };
  load_bits(blockIdx.x);
  for (int p = 0; p < kDigits; ++p) sh[p][tid] = 0;
  if (tid < kWave) {
    uint32_t lo = zrange[tid], hi = zrange[kZSlots + tid];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, kWave));
      hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, kWave));
    }
    if (tid == 0) { s_z[0] = lo; s_z[1] = hi; }
  }
  __syncthreads();
  const uint32_t zmin = s_z[0], zmax = s_z[1];
  // block 0 also sends the instance total (the projection's count slots) to the host's pinned
  // word with the frame's sequence number: one system-scope store, which the host polls
  if (blockIdx.x == 0 && wave == 0) {
    unsigned long long c = count_slots[lane];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, kWave);
    if (lane == 0)
      __hip_atomic_store(host_word, ((unsigned long long)seq << 32) | (c < 0xFFFFFFFFull ? c : 0xFFFFFFFFull),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (blockIdx.x == 0 && tid == 0) {
    const int depth_bits = zmax > zmin ? 32 - __clz(zmax - zmin) : 0;
    info[0] = (uint32_t)((depth_bits + 7) / 8);          // passes the depth sort needs
    info[1] = (uint32_t)depth_bits;
    info[2] = zmin;
    // the host launches only the passes after the first that the depth range needs
    __hip_atomic_store(host_word + 1, ((unsigned long long)seq << 32) | (unsigned)depth_bits,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  const uint64_t lt_mask = lanemask_lt();
  for (int64_t part = blockIdx.x; part * kDkPart < m; part += gridDim.x) {
    const int64_t wbase = part * kDkPart + (int64_t)wave * (kWave * kDkItems);
    if (part != (int64_t)blockIdx.x) load_bits(part);
#pragma unroll
    for (int it = 0; it < kDkItems; ++it) {
      const int64_t pos = wbase + (int64_t)it * kWave + lane;
      const bool valid = pos < m;
      const uint64_t vmask = __ballot(valid);
      if (vmask == 0) break;
      const uint32_t k = zb[it] ? zb[it] - zmin : ~0u;        // zero bits: culled
      if (valid) { keys[pos] = k; vals[pos] = (uint32_t)pos; }
#pragma unroll
      for (int p = 0; p < kDigits - 1; ++p)            // lower digits: one atomic per key
        if (valid) atomicAdd(&sh[p][(k >> (8 * p)) & 0xFF], 1u);
      // top digit: few distinct values (0, or all ones for culled splats): count runs once
      const uint32_t d = k >> 24;
      uint64_t peers = vmask;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
      }
      if (valid && (peers & lt_mask) == 0) atomicAdd(&sh[kDigits - 1][d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  // blocks spread their sums over kTileHistCopies copies (blocks of a copy share an XCD)
  uint32_t* h = hist + (blockIdx.x % kTileHistCopies) * (kTileHistPasses * kBins);
  for (int p = 0; p < kDigits; ++p) {
    const uint32_t v = sh[p][tid];
    if (v) atomicAdd(&h[p * kBins + tid], v);
  }
}

// One scatter pass over digit `shift`. THREADS threads take a partition of THREADS * ITEMS keys
// (4096: 512 threads x 8 keys for 32-bit keys, so each wavefront ranks half as many keys in
// sequence; 256 x 16 for 64-bit keys).
template <typename K, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_onesweep(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
    uint32_t* __restrict__ vout, uint32_t m_arg, int shift, int digit_bits,
    const uint32_t* __restrict__ hist_row,
    int copies, int64_t copy_stride, uint32_t* __restrict__ status,
    uint32_t* __restrict__ status_next, uint32_t* __restrict__ gstatus,
    uint32_t* __restrict__ gstatus_next, const uint32_t* __restrict__ live_passes, int pass,
    uint32_t* __restrict__ ranges, uint32_t n_tiles, uint32_t* __restrict__ err, uint32_t spin_limit,
    const uint64_t* __restrict__ m_dev) {
  constexpr int W = THREADS / kWave;
  constexpr int PART = THREADS * ITEMS;
  constexpr int kItems = ITEMS;
  if (live_passes && pass >= (int)*live_passes) return;    // digit beyond the data's bits
  if (frame_failed(err)) return;
  // with the count on the device (a fixed-capacity launch), partitions past it have nothing to do
  const uint32_t m = m_dev ? (uint32_t)min(*m_dev, (uint64_t)m_arg) : m_arg;
  if (blockIdx.x * (uint32_t)PART >= m) return;
  __shared__ uint32_t s_hist[W][kBins];        // per-wave counts, then per-wave offsets
  __shared__ uint32_t s_local[kBins];          // block-local start of each digit run
  __shared__ uint32_t s_global[kBins];         // global start of the run minus its local start
  __shared__ uint32_t s_wsum[kBins / kWave];
  __shared__ uint32_t s_tsum[kBins / kWave];
  __shared__ K s_buf[PART];                    // keys in block-local digit order
  __shared__ uint32_t s_val[PART];             // values in the same order
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (int i = tid; i < W * kBins; i += THREADS) (&s_hist[0][0])[i] = 0u;
  __syncthreads();
  const uint32_t part = blockIdx.x;   // in-order dispatch: predecessors are running or done
  const uint32_t wbase = part * PART + (uint32_t)wave * (kWave * kItems);   // 32-bit: m < 2^32
  K key[kItems];
  uint32_t val[kItems];
  uint32_t rank[kItems];
  const uint64_t lt_mask = lanemask_lt();
  // partition 0: the pass's digit totals, loaded first so that they arrive during the ranking
  uint32_t tot = 0;
  if (part == 0 && tid < kBins) {
#pragma unroll 8
    for (int c = 0; c < copies; ++c) tot += hist_row[c * copy_stride + tid];
  }
  // every load issued before the first is used
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const uint32_t pos = wbase + (uint32_t)(it * kWave + lane);
    key[it] = pos < m ? kin[pos] : (K)0;
  }
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const uint32_t pos = wbase + (uint32_t)(it * kWave + lane);
    val[it] = pos < m ? vin[pos] : 0u;
  }
  // rank within the wave: lanes holding the same digit are matched with eight ballots; the lowest
  // of them adds the run to the wave's digit counter (an LDS atomic returning the old count, so
  // the items' updates pipeline instead of waiting on each other) and its peers read the old count
  // from it
  int leader[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const bool valid = wbase + (uint32_t)(it * kWave + lane) < m;
    const uint32_t d = (uint32_t)(key[it] >> shift) & 0xFF;
    uint64_t peers = __ballot(valid);
    // digit bits above digit_bits are zero in every key: they need no ballot
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b >= digit_bits) break;
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t below = __popcll(peers & lt_mask);
    uint32_t old = 0;
    if (valid && below == 0) old = atomicAdd(&s_hist[wave][d], (uint32_t)__popcll(peers));
    leader[it] = valid ? (int)__builtin_ctzll(peers) : lane;
    rank[it] = old + below;                     // the leader's old count arrives below
  }
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const uint32_t lead_old = __shfl(rank[it], leader[it], kWave);   // the leader holds its old count
    rank[it] = lane == leader[it] ? lead_old : lead_old + rank[it];
  }
  __syncthreads();
  // per digit (threads 0..255, one digit each): offsets of each wave's run and the block total
  const bool digit_thread = tid < kBins;
  uint32_t count = 0, incl = 0;
  uint32_t cw[W];
  if (digit_thread) {
#pragma unroll
    for (int w = 0; w < W; ++w) { cw[w] = s_hist[w][tid]; count += cw[w]; }
    // publish this partition's digit count as early as possible
    if (part > 0) atomic_store_u32(&status[part * kBins + tid], kSortAgg | count);
    // block-local exclusive scan of the digit counts
    incl = wave_inclusive_scan(count);
    if (lane == kWave - 1) s_wsum[wave] = incl;
  }
  // Partition 0 turns the pass's digit totals (the sum of `copies` partial histograms) into the
  // digit bases and publishes base + count as its inclusive prefix, so every later partition's
  // look-back already includes the base.
  uint32_t excl = 0;
  if (part == 0) {
    const uint32_t tincl = digit_thread ? wave_inclusive_scan(tot) : 0u;
    if (digit_thread && lane == kWave - 1) s_tsum[wave] = tincl;
    __syncthreads();
    if (digit_thread) {
      uint32_t pre = 0;
      for (int w = 0; w < wave; ++w) pre += s_tsum[w];
      excl = pre + tincl - tot;
      atomic_store_u32(&status[tid], kSortPrefix | (excl + count));
    }
  }
  __syncthreads();
  uint32_t local_start = 0;
  if (digit_thread) {
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += s_wsum[w];
    local_start = pre + incl - count;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) { s_hist[w][tid] = run; run += cw[w]; }
    s_local[tid] = local_start;
  }
  __syncthreads();
  // keys and values to LDS in block-local digit order before the look-back, so that they no
  // longer hold registers while the digit threads wait on their predecessors
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const uint32_t pos = wbase + (uint32_t)(it * kWave + lane);
    const uint32_t d = (uint32_t)(key[it] >> shift) & 0xFF;
    const uint32_t lp = s_local[d] + s_hist[wave][d] + rank[it];
    if (pos < m && lp < (uint32_t)PART) {
      s_buf[lp] = key[it];
      s_val[lp] = val[it];
    }
  }
  // the staged keys and values leave registers before the look-back's loads are issued
  __builtin_amdgcn_sched_barrier(0);
  if (digit_thread) {
    // look back for this digit: first over the earlier partitions of this partition's group, then,
    // if none of them holds an inclusive prefix, over the group rows of the earlier groups
    if (part > 0) {
      const uint32_t grp = part / kGroupParts, g_first = grp * kGroupParts;
      const bool group_last = part - g_first == kGroupParts - 1;
      const int n_in_group = (int)(part - g_first);   // earlier partitions of the group
      uint32_t spins = 0, acc = 0;
      int state = 0;                         // 0: all aggregates, 1: reached a prefix, 2: not ready
      const uint32_t* win = status + ((int64_t)part - 1) * kBins + tid;
      while (true) {
        // one window of predecessors (loads at fixed offsets from one address, which is re-derived
        // each round so that 32 addresses do not stay live across the wait); those before the
        // group are read but count as empty aggregates
        asm volatile("" : "+v"(win));
        uint32_t v[kGroupParts];
#pragma unroll
        for (int w = 0; w < kGroupParts; ++w)
          v[w] = ((int64_t)part - 1 - w >= 0) ? atomic_load_u32(win - (int64_t)w * kBins) : kSortAgg;
        acc = 0;
        state = 0;
#pragma unroll
        for (int w = 0; w < kGroupParts; ++w) {
          if (state != 0 || w >= n_in_group) continue;
          const uint32_t flag = v[w] & ~kSortValue;
          if (flag == 0) { state = 2; continue; }
          acc += v[w] & kSortValue;
          if (flag == kSortPrefix) state = 1;
        }
        if (state == 2) {
          if (++spins < spin_limit) continue;
          flag_error(err, kErrSpin);           // a broken launch: the frame is marked failed
        }
        break;
      }
      excl += acc;
      // the group's total is known as soon as its last partition has read the group (group 0 always
      // meets partition 0's prefix, so only later groups publish a total)
      if (group_last && state == 0) atomic_store_u32(&gstatus[grp * kBins + tid], kSortAgg | (acc + count));
      if (state == 0) {
        int64_t q = (int64_t)grp - 1;       // grp >= 1 here
        spins = 0;
        while (true) {
          uint32_t v[kLookWindow];
#pragma unroll
          for (int w = 0; w < kLookWindow; ++w)
            v[w] = (q - w >= 0) ? atomic_load_u32(&gstatus[(q - w) * kBins + tid]) : kSortPrefix;
          acc = 0;
          state = 0;
#pragma unroll
          for (int w = 0; w < kLookWindow; ++w) {
            if (state != 0) continue;
            const uint32_t flag = v[w] & ~kSortValue;
            if (flag == 0) { state = 2; continue; }
            acc += v[w] & kSortValue;
            if (flag == kSortPrefix) state = 1;
          }
          if (state == 2) {
            if (++spins < spin_limit) continue;
            flag_error(err, kErrSpin);
            break;
          }
          excl += acc;
          if (state == 1) break;
          q -= kLookWindow;
        }
      }
      atomic_store_u32(&status[part * kBins + tid], kSortPrefix | (excl + count));
      if (group_last) atomic_store_u32(&gstatus[grp * kBins + tid], kSortPrefix | (excl + count));
    }
    // clear this partition's slices of the other status buffers for the next pass
    status_next[part * kBins + tid] = 0u;
    if (part % kGroupParts == kGroupParts - 1) gstatus_next[(part / kGroupParts) * kBins + tid] = 0u;
    s_global[tid] = excl - local_start;
  }
  __syncthreads();
  // keys and values leave in digit runs
  const uint32_t pbase = part * PART;
  const int n_here = (int)min((uint32_t)PART, m - pbase);
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int j = tid + r * THREADS;
    if (j < n_here) {
      const K k = s_buf[j];
      const uint32_t g = s_global[(uint32_t)(k >> shift) & 0xFF] + (uint32_t)j;
      if (g < m) {
        kout[g] = k;
        vout[g] = s_val[j];
        // last pass of a tile sort: every run boundary in the block proposes its tile's start and
        // end; the earliest start and the latest end win (starts stored complemented, so that one
        // atomic maximum serves both and zero still means "no run")
        if (ranges && (uint64_t)k < n_tiles) {
          if (j == 0 || s_buf[j - 1] != k) atomicMax(&ranges[(uint32_t)k], ~g);
          if (j == n_here - 1 || s_buf[j + 1] != k) atomicMax(&ranges[n_tiles + (uint32_t)k], g + 1);
        }
      }
    }
  }
}

__global__ void k_ranges(const uint32_t* __restrict__ keys, int64_t m_arg, int64_t n_tiles,
                         uint32_t* __restrict__ ranges, const uint64_t* __restrict__ m_dev,
                         const uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (frame_failed(err)) return;
  const int64_t m = m_dev ? (int64_t)min(*m_dev, (uint64_t)m_arg) : m_arg;
  if (i >= m) return;
  const uint32_t t = keys[i];
  if (t >= (uint64_t)n_tiles) return;
  if (i == 0 || keys[i - 1] != t) ranges[t] = ~(uint32_t)i;        // complemented, as the sort writes it
  if (i == m - 1 || keys[i + 1] != t) ranges[n_tiles + t] = (uint32_t)(i + 1);
}

// Compositing order of the tiles, longest list first (a list-scheduling heuristic for blocks of
// very unequal work): lengths are bucketed by 64 entries, buckets taken in descending order, empty
// tiles last; the order inside a bucket is arbitrary. One block; it writes a permutation of all
// tiles.
constexpr int kOrderThreads = 1024;
// Length of a run whose start is stored complemented (0: empty tile).
__device__ __forceinline__ uint32_t run_length(uint32_t start_complemented, uint32_t end) {
  return start_complemented ? end - ~start_complemented : 0u;
}
constexpr int kOrderBuckets = 257;              // 256 length buckets + empty tiles
__device__ __forceinline__ int order_bucket(uint32_t len) {
  return len == 0 ? kOrderBuckets - 1 : 255 - (int)min(len >> 6, 255u);
}

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(uint32_t* __restrict__ ranges,
                                                              int64_t n_tiles,
                                                              uint32_t* __restrict__ order,
                                                              const uint32_t* __restrict__ err,
                                                              unsigned long long* __restrict__ report,
                                                              uint32_t seq, uint32_t* __restrict__ slots) {
  __shared__ uint32_t s_cnt[kOrderBuckets + 1];
  const int tid = threadIdx.x, lane = lane_id();
  // the projection slots have been read (by the depth-key pass): reset for the next frame
  if (slots && tid < kSlotWords) slots[tid] = tid < kZSlots ? 0xFFFFFFFFu : 0u;
  // the frame's ordering is complete here: its error word goes to the host (one system-scope
  // store), and a failed frame has no valid runs to order
  if (tid == 0 && report)
    __hip_atomic_store(report, ((unsigned long long)seq << 32) | (err ? *err : 0u), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  if (frame_failed(err)) {
    for (int64_t t = tid; t < n_tiles; t += kOrderThreads) {
      ranges[t] = 0u;
      ranges[n_tiles + t] = 0u;
      order[t] = (uint32_t)t;
    }
    return;
  }
  const uint64_t lt = lanemask_lt();
  constexpr int kPer = 8;                          // tiles per thread per step, loads issued first
  constexpr int64_t kStep = (int64_t)kOrderThreads * kPer;
  for (int b = tid; b <= kOrderBuckets; b += kOrderThreads) s_cnt[b] = 0;
  __syncthreads();
  // with every tile in one step (a 1080p frame: 8,160 tiles) the second sweep reuses the lengths
  // and starts held in registers instead of reading the ranges again
  const bool one_step = n_tiles <= kStep;
  uint32_t kept_len[kPer], kept_raw[kPer];
  for (int64_t t0 = 0; t0 < n_tiles; t0 += kStep) {
    uint32_t len[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t t = t0 + (int64_t)j * kOrderThreads + tid;
      kept_raw[j] = t < n_tiles ? ranges[t] : 0u;
      len[j] = t < n_tiles ? run_length(kept_raw[j], ranges[n_tiles + t]) : 0u;
      kept_len[j] = len[j];
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t t = t0 + (int64_t)j * kOrderThreads + tid;
      const bool valid = t < n_tiles;
      // empty tiles, most of a frame, are counted once per wavefront
      const uint64_t em = __ballot(valid && len[j] == 0);
      if (em && lane == (int)__builtin_ctzll(em)) atomicAdd(&s_cnt[kOrderBuckets - 1], (uint32_t)__popcll(em));
      if (valid && len[j] != 0) atomicAdd(&s_cnt[order_bucket(len[j])], 1u);
    }
  }
  __syncthreads();
  if (tid < kWave) {                                // exclusive scan of the bucket counts
    uint32_t carry = 0;
    for (int b0 = 0; b0 < kOrderBuckets; b0 += kWave) {
      const uint32_t v = b0 + tid < kOrderBuckets ? s_cnt[b0 + tid] : 0u;
      const uint32_t incl = wave_inclusive_scan(v);
      if (b0 + tid < kOrderBuckets) s_cnt[b0 + tid] = carry + incl - v;
      carry += __shfl(incl, kWave - 1, kWave);
    }
  }
  __syncthreads();
  for (int64_t t0 = 0; t0 < n_tiles; t0 += kStep) {
    uint32_t len[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t t = t0 + (int64_t)j * kOrderThreads + tid;
      len[j] = 0u;
      if (t < n_tiles) {
        const uint32_t raw = one_step ? kept_raw[j] : ranges[t];
        len[j] = one_step ? kept_len[j] : run_length(raw, ranges[n_tiles + t]);
        ranges[t] = raw ? ~raw : 0u;                  // plain starts for the tiles' readers
      }
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t t = t0 + (int64_t)j * kOrderThreads + tid;
      const bool valid = t < n_tiles;
      const uint64_t em = __ballot(valid && len[j] == 0);
      uint32_t base = 0;
      if (em && lane == (int)__builtin_ctzll(em)) base = atomicAdd(&s_cnt[kOrderBuckets - 1], (uint32_t)__popcll(em));
      if (em) base = __shfl(base, (int)__builtin_ctzll(em), kWave);
      uint32_t pos;
      if (len[j] == 0) pos = base + (uint32_t)__popcll(em & lt);
      else pos = valid ? atomicAdd(&s_cnt[order_bucket(len[j])], 1u) : 0u;
      if (valid && pos < (uint64_t)n_tiles) order[pos] = (uint32_t)t;
    }
  }
}

// Canonical key (tile << 32) | fp32 depth bits, the depth read back from the splat record.
__global__ void k_canonical(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                            int64_t m, int64_t n, int64_t tiles_per_cam,
                            const float4* __restrict__ rec, uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t t = keys[i];
  const int64_t cam = (int64_t)t / tiles_per_cam;
  const float z = rec[(cam * n + vals[i]) * kRecFloat4].w;
  out[i] = ((uint64_t)t << 32) | (uint64_t)__float_as_uint(z);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---- host launchers -------------------------------------------------------------------------
size_t scan_scratch_bytes(int64_t n) {
  const int64_t parts = (n + kBinPart - 1) / kBinPart;     // kBinPart <= kPart: covers both scans
  return (size_t)(parts + 1) * sizeof(uint64_t) + 256;
}

// (the fused binning scan uses partitions of kBinPart <= kPart positions: counted in those)
int64_t scan_clear_words(int64_t n) { return (n + kBinPart - 1) / kBinPart * 2; }

hipError_t launch_scan(const uint32_t* in, const uint32_t* gather0, const uint32_t* gather1,
                       const uint32_t* sel, uint32_t* out, int64_t n, uint64_t* total, void* scratch,
                       hipStream_t s, bool scratch_cleared, uint32_t* err, uint32_t spin_limit) {
  const int64_t parts = (n + kPart - 1) / kPart;
  uint64_t* status = reinterpret_cast<uint64_t*>(scratch);
  hipError_t e = scratch_cleared ? hipSuccess
                                 : launch_fill_u32(reinterpret_cast<uint32_t*>(scratch), 0u, parts * 2, s);
  if (e != hipSuccess) return e;
  if (n == 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(total), 0u, 2, s);
  hipLaunchKernelGGL(k_scan, dim3((unsigned)parts), dim3(kThreads), 0, s, in, gather0, gather1, sel, out,
                     n, parts, status, total, err, spin_limit ? spin_limit : kSpinLimit);
  return hipGetLastError();
}

hipError_t launch_depth_keys_hist(int64_t m, const uint32_t* zbits,
                                  const unsigned long long* count_slots,
                                  unsigned long long* host_word, uint32_t seq, const uint32_t* zrange,
                                  uint32_t* info, uint32_t* keys, uint32_t* vals, uint32_t* hist_copies,
                                  hipStream_t s) {
  if (m == 0) return hipSuccess;
  static_assert(kZSlots == kWave, "one count slot per lane");
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, (m + kThreads * 4 - 1) / (kThreads * 4));
  hipLaunchKernelGGL(k_depth_keys_hist, dim3(blocks), dim3(256), 0, s, m, zbits, count_slots, host_word,
                     seq, zrange, info, keys, vals, hist_copies);
  return hipGetLastError();
}

hipError_t launch_scan_binning(int64_t n, int n_cams, int TX, int64_t tiles_per_cam,
                               const uint32_t* order0, const uint32_t* order1,
                               const uint32_t* passes, const uint2* rect, bool narrow_rect,
                               void* scan_scratch, uint64_t* total, uint32_t* keys, uint32_t* vals, int tile_bits,
                               uint32_t* hist, const ClearSpans& clear, hipStream_t s, uint32_t* err,
                               uint32_t spin_limit, uint64_t capacity) {
  const int64_t cn = n * n_cams;
  if (cn == 0) return hipSuccess;
  if (tile_bits > 8 * kTileHistPasses) return hipErrorInvalidValue;
  const int64_t parts = (cn + kBinPart - 1) / kBinPart;
  hipLaunchKernelGGL(k_scan_bin, dim3((unsigned)parts), dim3(kThreads), 0, s, cn, (uint32_t)n, TX,
                     (uint32_t)tiles_per_cam, order0, order1, passes, rect, narrow_rect, parts,
                     reinterpret_cast<uint64_t*>(scan_scratch), total, keys, vals, (tile_bits + 7) / 8,
                     hist, clear, err, spin_limit ? spin_limit : kSpinLimit, capacity);
  return hipGetLastError();
}


// Scatter partitions of 4096 keys: 32-bit keys 512 threads x 8 (1024 x 4 when the caller asks for
// the wide shape), 64-bit keys 256 x 16. Scratch is sized (and cleared) for kSortPartMin-key
// partitions.
constexpr int kSortPartMin = 4096;
template <typename K> struct SweepShape {
  static constexpr int threads = sizeof(K) == 4 ? 512 : 256;
  static constexpr int items = sizeof(K) == 4 ? 8 : 16;
  static constexpr int part = threads * items;
};
static_assert(SweepShape<uint32_t>::part >= kSortPartMin && SweepShape<uint64_t>::part >= kSortPartMin,
              "scratch sizing assumes partitions of at least kSortPartMin keys");

size_t sort_scratch_bytes(int64_t m) {
  const int64_t parts = (m + kSortPartMin - 1) / kSortPartMin;
  const int64_t groups = (parts + kGroupParts - 1) / kGroupParts;
  return (size_t)(kMaxPasses * kBins + 2 * (parts + groups) * kBins) * sizeof(uint32_t) + 256;
}

int64_t sort_clear_words(int64_t m) {
  const int64_t parts = (m + kSortPartMin - 1) / kSortPartMin;
  return kMaxPasses * kBins + (parts + (parts + kGroupParts - 1) / kGroupParts) * kBins;
}

template <typename K>
hipError_t launch_sort(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t m, int bits, void* scratch,
                       hipStream_t s, bool* result_in_alt, const uint32_t* live_passes,
                       bool scratch_cleared, bool hist_ready, const uint32_t* ext_hist,
                       int pass_begin, int pass_end, uint32_t* ranges, int64_t n_tiles,
                       uint32_t* err, uint32_t spin_limit, const uint64_t* m_dev, bool wide) {
  *result_in_alt = false;
  if (m <= 1 || bits <= 0) return hipSuccess;
  // the chained scan's status words carry 30-bit counts
  if (m >= (int64_t(1) << 30)) return hipErrorInvalidValue;
  const int n_passes = (bits + 7) / 8;
  if (pass_end < 0 || pass_end > n_passes) pass_end = n_passes;
  const int64_t parts = (m + kPart - 1) / kPart;    // partitions of the histogram
  constexpr int kSweepThreads = SweepShape<K>::threads;
  constexpr int kSweepItems = SweepShape<K>::items;
  const int64_t sweep_parts = (m + SweepShape<K>::part - 1) / SweepShape<K>::part;
  // scratch: hist[8][256] | status0[parts][256] | gstatus0[groups][256] | status1[parts][256] |
  // gstatus1[groups][256]. One fill clears the histograms, status0 and gstatus0; pass p reads the
  // buffers of parity p & 1 and clears its slices of the other pair for pass p + 1.
  const int64_t sweep_groups = (sweep_parts + kGroupParts - 1) / kGroupParts;
  uint32_t* hist = reinterpret_cast<uint32_t*>(scratch);
  uint32_t* status0 = hist + kMaxPasses * kBins;
  uint32_t* gstatus0 = status0 + sweep_parts * kBins;
  uint32_t* status1 = gstatus0 + sweep_groups * kBins;
  uint32_t* gstatus1 = status1 + sweep_parts * kBins;
  hipError_t e = (scratch_cleared || pass_begin > 0)
                     ? hipSuccess
                     : launch_fill_u32(hist, 0u, kMaxPasses * kBins + (sweep_parts + sweep_groups) * kBins, s);
  if (e != hipSuccess) return e;
  const int hblocks = (int)std::min<int64_t>(kHistBlocks, parts);
  if (!hist_ready && !ext_hist && pass_begin == 0) {
    hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)hblocks), dim3(256), 0, s, k0, m, n_passes, hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const uint32_t* rows = ext_hist ? ext_hist : hist;
  const int copies = ext_hist ? kTileHistCopies : 1;
  const int64_t copy_stride = ext_hist ? (int64_t)kTileHistPasses * kBins : 0;
  K *ki = k0, *ko = k1;
  uint32_t *vi = v0, *vo = v1;
  if (pass_begin & 1) {
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  if (ranges && (sizeof(K) != 4 || n_tiles <= 0 || n_tiles > 0xFFFFFFFFll)) return hipErrorInvalidValue;
  // the same 4096-key partitions as 1024 threads x 4 keys: twice the wavefronts per CU to hide
  // each pass's load, look-back and scatter latency where the partitions are few (one per CU)
  auto sweep = k_onesweep<K, kSweepThreads, kSweepItems>;
  int sweep_threads = kSweepThreads;
  if constexpr (sizeof(K) == 4) {
    static_assert(1024 * 4 == SweepShape<uint32_t>::part, "the wide shape keeps the partition size");
    if (wide) {
      sweep = k_onesweep<K, 1024, 4>;
      sweep_threads = 1024;
    }
  }
  for (int p = pass_begin; p < pass_end; ++p) {
    uint32_t* st = (p & 1) ? status1 : status0;
    uint32_t* st_next = (p & 1) ? status0 : status1;
    uint32_t* gst = (p & 1) ? gstatus1 : gstatus0;
    uint32_t* gst_next = (p & 1) ? gstatus0 : gstatus1;
    uint32_t* rng = p == n_passes - 1 ? ranges : nullptr;
    hipLaunchKernelGGL(sweep, dim3((unsigned)sweep_parts), dim3(sweep_threads), 0, s, ki, vi, ko, vo, (uint32_t)m,
                       8 * p, std::min(8, bits - 8 * p), rows + p * kBins, copies, copy_stride, st, st_next, gst, gst_next, live_passes, p,
                       rng, (uint32_t)n_tiles, err, spin_limit ? spin_limit : kSpinLimit, m_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  *result_in_alt = (pass_end % 2) == 1;
  return hipSuccess;
}
template hipError_t launch_sort<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, int64_t, int,
                                          void*, hipStream_t, bool*, const uint32_t*, bool, bool,
                                          const uint32_t*, int, int, uint32_t*, int64_t, uint32_t*,
                                          uint32_t, const uint64_t*, bool);
template hipError_t launch_sort<uint64_t>(uint64_t*, uint32_t*, uint64_t*, uint32_t*, int64_t, int,
                                          void*, hipStream_t, bool*, const uint32_t*, bool, bool,
                                          const uint32_t*, int, int, uint32_t*, int64_t, uint32_t*,
                                          uint32_t, const uint64_t*, bool);

hipError_t launch_ranges(const uint32_t* keys, int64_t m, int64_t n_tiles, uint32_t* ranges,
                         hipStream_t s, const uint64_t* m_dev, const uint32_t* err) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ranges, dim3(blocks_for(m, 256)), dim3(256), 0, s, keys, m, n_tiles, ranges,
                     m_dev, err);
  return hipGetLastError();
}

hipError_t launch_tile_order(uint32_t* ranges, int64_t n_tiles, uint32_t* order, hipStream_t s,
                             const uint32_t* err, unsigned long long* report, uint32_t seq,
                             uint32_t* slots) {
  if (n_tiles == 0) return hipSuccess;
  static_assert(kSlotWords <= kOrderThreads, "one thread per slot word");
  hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, s, ranges, n_tiles, order, err,
                     report, seq, slots);
  return hipGetLastError();
}

hipError_t launch_canonical_keys(const uint32_t* keys, const uint32_t* vals, int64_t m, int64_t n,
                                 int64_t tiles_per_cam, const float4* rec, uint64_t* out,
                                 hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_canonical, dim3(blocks_for(m, 256)), dim3(256), 0, s, keys, vals, m, n,
                     tiles_per_cam, rec, out);
  return hipGetLastError();
}

}  // namespace pcs
