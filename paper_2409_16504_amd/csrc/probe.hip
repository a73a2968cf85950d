// Peak-rate probe used by the benchmark: LDS read bandwidth of the whole GPU, measured with a
// kernel that does nothing but conflict-free 16-byte LDS reads. The compositing kernel's LDS
// traffic is reported against this measured figure rather than a datasheet number.

#include "pcs_internal.hpp"

namespace pcs {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeWords = 8192;            // floats of the LDS array (32 KiB)

// Each thread reads float4 words at consecutive addresses of its wavefront (lane-contiguous, so
// the 64 lanes of one read cover 1 KiB without bank conflicts), `iters` times over a 32 KiB array.
__global__ __launch_bounds__(kProbeThreads) void k_lds_read(int iters, float* __restrict__ sink) {
  __shared__ float4 buf[kProbeWords / 4];
  const int tid = threadIdx.x;
  for (int i = tid; i < kProbeWords / 4; i += kProbeThreads)
    buf[i] = make_float4((float)i, 1.0f, 2.0f, 3.0f);
  __syncthreads();
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  int idx = tid;
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float4 v = buf[(idx + k * kProbeThreads) & (kProbeWords / 4 - 1)];
      acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    idx = (idx + 64) & (kProbeWords / 4 - 1);
  }
  // one store per thread keeps the reads alive; the value itself is never used
  if (acc.x == -1.0f) sink[blockIdx.x * kProbeThreads + tid] = acc.y + acc.z + acc.w;
}

}  // namespace

hipError_t launch_lds_probe(int blocks, int iters, float* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_lds_read, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s, iters, sink);
  return hipGetLastError();
}

int64_t lds_probe_bytes(int blocks, int iters) {
  return (int64_t)blocks * kProbeThreads * iters * 8 * 16;
}

}  // namespace pcs
