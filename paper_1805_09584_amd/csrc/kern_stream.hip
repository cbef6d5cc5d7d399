// Streaming-bandwidth reference kernels: the ceiling that the bandwidth-bound
// kernels of the library are compared with on the same device.  Each moves
// 16 bytes per lane with non-temporal accesses over a grid-stride loop.
#include "ndtm_internal.h"

namespace ndtm {
namespace {

typedef unsigned v4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_copy_k(const v4u* __restrict__ a, v4u* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ __launch_bounds__(256) void stream_read_k(const v4u* __restrict__ a, size_t n, unsigned* sink) {
  unsigned s = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const v4u v = __builtin_nontemporal_load(a + i);
    s ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  // the xor of all words is data dependent: the store keeps the loads alive
  if (s == 0x9e3779b9u) sink[0] = s;
}

__global__ __launch_bounds__(256) void stream_write_k(v4u* __restrict__ b, size_t n) {
  const v4u z = {0u, 0u, 0u, 0u};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(z, b + i);
}

}  // namespace

void launch_stream(int kind, const void* a, void* b, size_t bytes, unsigned* sink, hipStream_t st) {
  const size_t n = bytes / 16;
  const dim3 grid(1024), block(256);
  if (kind == 0)
    hipLaunchKernelGGL(stream_copy_k, grid, block, 0, st, static_cast<const v4u*>(a), static_cast<v4u*>(b), n);
  else if (kind == 1)
    hipLaunchKernelGGL(stream_read_k, grid, block, 0, st, static_cast<const v4u*>(a), n, sink);
  else
    hipLaunchKernelGGL(stream_write_k, grid, block, 0, st, static_cast<v4u*>(b), n);
}

}  // namespace ndtm
