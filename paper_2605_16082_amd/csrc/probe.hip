// Streaming probes: the device's read-only, write-only and copy bandwidth
// with 16-byte accesses per lane, the ceiling the stage and solve kernels'
// algorithmic bandwidth is compared with (not part of the method).
//
// Grid-stride loops over 16-byte elements, four independent accesses in
// flight per lane per iteration; every workgroup covers a contiguous quarter
// of the grid's stride so that a wavefront's accesses stay 1 KiB contiguous.
#include "internal.h"
#include "slimdg.h"

namespace sdg {
namespace {

struct alignas(16) V16 {
  double x, y;
};

constexpr int kProbeThreads = 256;
constexpr int kUnroll = 4;

// sum of every element (read only); one partial per workgroup in out
__global__ __launch_bounds__(kProbeThreads) void probe_read(const V16* __restrict__ src, int64_t n,
                                                            double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads * kUnroll;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kProbeThreads * kUnroll + threadIdx.x; i < n; i += stride) {
    V16 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t j = i + (int64_t)u * kProbeThreads;
      v[u] = j < n ? src[j] : V16{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc += v[u].x + v[u].y;
  }
  __shared__ double red[kProbeThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kProbeThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kProbeThreads) void probe_write(V16* __restrict__ dst, int64_t n, double val) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads * kUnroll;
  for (int64_t i = (int64_t)blockIdx.x * kProbeThreads * kUnroll + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t j = i + (int64_t)u * kProbeThreads;
      if (j < n) dst[j] = V16{val, val};
    }
  }
}

__global__ __launch_bounds__(kProbeThreads) void probe_copy(const V16* __restrict__ src, V16* __restrict__ dst,
                                                            int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads * kUnroll;
  for (int64_t i = (int64_t)blockIdx.x * kProbeThreads * kUnroll + threadIdx.x; i < n; i += stride) {
    V16 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t j = i + (int64_t)u * kProbeThreads;
      v[u] = j < n ? src[j] : V16{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t j = i + (int64_t)u * kProbeThreads;
      if (j < n) dst[j] = v[u];
    }
  }
}

}  // namespace
}  // namespace sdg

extern "C" sdg_status sdg_stream_probe(int kind, const void* dev_src, void* dev_dst, size_t bytes, int workgroups,
                                       void* hip_stream) {
  using namespace sdg;
  if (bytes % 16 != 0 || bytes == 0 || workgroups < 1) return SDG_E_ARG;
  if ((kind == SDG_PROBE_READ || kind == SDG_PROBE_COPY) && !dev_src) return SDG_E_ARG;
  if (!dev_dst) return SDG_E_ARG;
  if ((reinterpret_cast<uintptr_t>(dev_src) | reinterpret_cast<uintptr_t>(dev_dst)) % 16 != 0) return SDG_E_ARG;
  const int64_t n = (int64_t)(bytes / 16);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const dim3 grid(workgroups), block(kProbeThreads);
  switch (kind) {
    case SDG_PROBE_READ:
      hipLaunchKernelGGL(probe_read, grid, block, 0, s, static_cast<const V16*>(dev_src), n,
                         static_cast<double*>(dev_dst));
      break;
    case SDG_PROBE_WRITE:
      hipLaunchKernelGGL(probe_write, grid, block, 0, s, static_cast<V16*>(dev_dst), n, 1.0);
      break;
    case SDG_PROBE_COPY:
      hipLaunchKernelGGL(probe_copy, grid, block, 0, s, static_cast<const V16*>(dev_src),
                         static_cast<V16*>(dev_dst), n);
      break;
    default:
      return SDG_E_ARG;
  }
  return hipGetLastError() == hipSuccess ? SDG_OK : SDG_E_HIP;
}
