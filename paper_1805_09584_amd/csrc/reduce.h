// Per-thread part of a fixed-order sum over reduction partials.
//
// Thread t adds p[t], p[t + T], p[t + 2T], ... (T threads) in that order.  The
// loads are issued eight at a time before any is added, so a thread waits on one
// memory latency per eight partials instead of one per partial; the additions
// keep their order, so the result is the same bits as the plain loop.
#pragma once

#include <hip/hip_runtime.h>

namespace ndtm {

__device__ __forceinline__ double strided_sum(const double* p, int n) {
  constexpr int kBatch = 8;
  const int T = (int)blockDim.x;
  double v = 0;
  for (int i0 = (int)threadIdx.x; i0 < n; i0 += kBatch * T) {
    double t[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int i = i0 + j * T;
      t[j] = i < n ? p[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (i0 + j * T < n) v += t[j];
  }
  return v;
}

}  // namespace ndtm
