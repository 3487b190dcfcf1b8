// Read-bandwidth probe: the rate at which the device streams a buffer from
// memory, the practical ceiling for the two products' matrix streams.
#include <algorithm>

#include "imrt_internal.h"

using namespace imrt;

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 8;   // 16-byte loads in flight per thread

// Sum of every float of the buffer (n4 groups of four), eight loads in flight
// per thread; a block's sum is stored only if negative (never, for a buffer
// of nonnegative values), which keeps the loads without a write stream.
__global__ __launch_bounds__(kProbeThreads) void read_probe_kernel(const float4* __restrict__ src, int64_t n4,
                                                                    float* __restrict__ sink) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kProbeThreads;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
  float acc = 0.0f;
  for (; i + (kProbeUnroll - 1) * stride < n4; i += kProbeUnroll * stride) {
    float4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < n4; i += stride) {
    const float4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc < 0.0f) sink[blockIdx.x] = acc;
}

}  // namespace

int imrt_read_probe(imrt_ctx* ctx, const void* buf, int64_t bytes, int32_t reps, double* gbs_out) {
  if (!ctx || !buf || !gbs_out) return set_error(IMRT_EINVAL, "ctx, buf or gbs_out is NULL");
  if (bytes < 16 || reps < 1) return set_error(IMRT_EINVAL, "bytes must be >= 16 and reps >= 1");
  if (reinterpret_cast<uintptr_t>(buf) % 16 != 0) return set_error(IMRT_EINVAL, "buf must be 16-byte aligned");
  IMRT_HIP(hipSetDevice(ctx->device));
  const int64_t n4 = bytes / 16;
  const int grid = ctx->num_cu * 16;
  float* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&sink), sizeof(float) * grid);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best = 0.0;
  for (int r = 0; e == hipSuccess && r <= reps; ++r) {   // the first launch warms up, untimed
    e = hipEventRecord(e0, ctx->stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(read_probe_kernel, dim3(grid), dim3(kProbeThreads), 0, ctx->stream,
                         static_cast<const float4*>(buf), n4, sink);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0 && ms > 0.0f) best = std::max(best, 16.0 * n4 / (ms * 1e-3) / 1e9);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sink) (void)hipFree(sink);
  if (e != hipSuccess) return hip_error(e, "read probe");
  *gbs_out = best;
  return IMRT_OK;
}
