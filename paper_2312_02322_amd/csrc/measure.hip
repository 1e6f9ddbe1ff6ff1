// Achievable streaming-read bandwidth of the device: the reference point for
// the bandwidth-bound kernels' roofline fractions beside the datasheet peak.
// Every wave reads 1 KiB contiguous per load (16 bytes per lane), eight loads
// in flight per lane, over a grid of four workgroups per compute unit that
// strides through the buffer.
#include "internal.h"

#include <algorithm>

namespace mqct {

constexpr int RB_THREADS = 256;
constexpr int RB_UNROLL = 8;

// never written in practice: the sums land here only if they hit an exact value;
// external linkage keeps the loads from being removed
__device__ float probe_sink[RB_THREADS];

namespace {

__global__ void __launch_bounds__(RB_THREADS)
read_probe(const float4* __restrict__ p, int64_t n16) {
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  const int64_t span = (int64_t)RB_THREADS * RB_UNROLL;
  const int64_t stride = (int64_t)gridDim.x * span;
  for (int64_t i = (int64_t)blockIdx.x * span + threadIdx.x; i < n16; i += stride) {
    float4 v[RB_UNROLL];
#pragma unroll
    for (int u = 0; u < RB_UNROLL; ++u) {
      const int64_t j = i + (int64_t)u * RB_THREADS;
      v[u] = j < n16 ? p[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < RB_UNROLL; ++u) {
      acc.x += v[u].x; acc.y += v[u].y; acc.z += v[u].z; acc.w += v[u].w;
    }
  }
  if (acc.x + acc.y + acc.z + acc.w == 1234.5f) probe_sink[threadIdx.x] = acc.x;
}

}  // namespace

hipError_t launch_read_probe(const void* buf, int64_t bytes, int n_cu, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  const int64_t span = (int64_t)RB_THREADS * RB_UNROLL;
  int64_t grid = 4 * (int64_t)n_cu;
  grid = std::min(grid, (n16 + span - 1) / span);
  if (grid < 1) grid = 1;
  read_probe<<<(unsigned)grid, RB_THREADS, 0, s>>>((const float4*)buf, n16);
  return hipGetLastError();
}

}  // namespace mqct
