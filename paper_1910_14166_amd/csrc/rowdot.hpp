// Row products of the d x d step kernels (H, its inverse or a shifted copy
// against a d-vector), one wavefront per row, and the width from which the
// step applies an explicit inverse.
#pragma once

#include "kernels.hpp"

namespace ihs {

// Lane l takes the columns l, l + 64, ... in ascending order (one fma chain
// per lane, or a sum of absolute values), then the fixed-order wavefront sum.
// A lane issues up to kRowDotLoads of its loads before its first fma: one
// wavefront's product is bound by the latency of its reads, not by their
// bandwidth, so for d <= 64 * kRowDotLoads it waits for memory once.
constexpr int kRowDotLoads = 16;

// From this width on the unconstrained step (and the l2 ball's cold start)
// forms H^{-1} (blocked triangular inverse on matrix cores) and applies it
// with these row products: the two triangular solves of one workgroup take
// 2 d / 64 block steps one after the other (about 0.8 ms at d = 1024 against
// about 0.3 ms for the inverse).
constexpr int64_t kQpInverseMinD = 89;

template <bool ABS>
__device__ __forceinline__ double row_dot(const double* __restrict__ row,
                                          const double* __restrict__ v, int64_t d, int lane) {
  double s = 0.0;
  for (int64_t k0 = lane; k0 < d; k0 += 64 * kRowDotLoads) {
    double a[kRowDotLoads], b[kRowDotLoads];
#pragma unroll
    for (int u = 0; u < kRowDotLoads; ++u) {
      const int64_t k = k0 + 64 * u;
      a[u] = k < d ? row[k] : 0.0;
      b[u] = (!ABS && k < d) ? v[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kRowDotLoads; ++u)
      if (k0 + 64 * u < d) s = ABS ? s + fabs(a[u]) : fma(a[u], b[u], s);
  }
  return wave_sum(s);
}

}  // namespace ihs
