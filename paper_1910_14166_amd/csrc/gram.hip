// The sketched Hessian H = (SA)^T (SA) (Sec. 1, the T_QP term; App. A.1.1:
// forming it costs O(m d^2)) on gfx950 matrix cores.
//
// Two wavefronts share each 32 x 32 tile of the upper triangle of H (16 rows
// each), for a contiguous slice of the m rows of SA (split-K). Operands come straight from
// L2: for a 16 x 16 x 4 product a lane supplies SA[k0 + lane/16][col0 + lane%16],
// so every operand load is four 128-byte row segments. Partial tiles are
// summed over the slices in a fixed order and mirrored into both triangles,
// so H is exactly symmetric and bitwise reproducible.
#include <algorithm>

#include "kernels.hpp"

namespace ihs {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTile = 32;

struct GramPlan {
  int64_t m, d, ld;
  int32_t batch, ntile, ntri, splits;
  int64_t kchunk;
};

static GramPlan make_gram_plan(int64_t m, int64_t d, int64_t ld, int32_t batch) {
  GramPlan g;
  g.m = m;
  g.d = d;
  g.ld = ld;
  g.batch = batch;
  g.ntile = (int32_t)((d + kTile - 1) / kTile);
  g.ntri = g.ntile * (g.ntile + 1) / 2;
  const int64_t waves = (int64_t)batch * g.ntri;
  int64_t splits = (2048 + waves - 1) / waves;
  const int64_t max_splits = std::max<int64_t>(1, (m + 63) / 64);
  splits = std::min<int64_t>(std::max<int64_t>(splits, 1), max_splits);
  splits = std::min<int64_t>(splits, 64);
  int64_t kc = (m + splits - 1) / splits;
  kc = (kc + 15) / 16 * 16;
  g.splits = (int32_t)((m + kc - 1) / kc);
  if (g.splits < 1) g.splits = 1;
  g.kchunk = kc;
  return g;
}

size_t gram_partials_bytes(int64_t m, int64_t d, int32_t batch, int32_t, int32_t) {
  const GramPlan g = make_gram_plan(m, d, d, batch);
  return (size_t)batch * g.ntri * g.splits * kTile * kTile * sizeof(double);
}

__device__ __forceinline__ void tri_index(int t, int& ti, int& tj) {
  // column-major upper triangle: t = tj*(tj+1)/2 + ti, 0 <= ti <= tj
  int j = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (j * (j + 1) / 2 > t) --j;
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  tj = j;
  ti = t - j * (j + 1) / 2;
}

template <typename TI>
__device__ __forceinline__ double to_f64(TI v);
template <>
__device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <>
__device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }

// Wavefront w = ((p * ntri + t) * splits + split) * 2 + half computes rows
// [16 half, 16 half + 16) of 32 x 32 tile t over its slice of the m rows.
// Two accumulators and a few k-steps of operands keep the register footprint
// small enough to run beside the memory-bound pass.
__device__ __forceinline__ void gram_wave_coords(const GramPlan& G, int64_t w, int& p, int& t,
                                                 int& split, int& half) {
  half = (int)(w & 1);
  const int64_t q = w >> 1;
  split = (int)(q % G.splits);
  t = (int)((q / G.splits) % G.ntri);
  p = (int)(q / ((int64_t)G.splits * G.ntri));
}

// FP64 matrix cores; F64 inputs, or F32 inputs widened exactly to F64.
template <typename TI>
__global__ __launch_bounds__(256, 8) void k_gram_f64(const TI* __restrict__ SA, GramPlan G,
                                                     double* __restrict__ part) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + wv;
  const int64_t total = (int64_t)G.batch * G.ntri * G.splits * 2;
  if (w >= total) return;
  int p, t, split, half;
  gram_wave_coords(G, w, p, t, split, half);
  int ti, tj;
  tri_index(t, ti, tj);
  const int64_t i0 = (int64_t)ti * kTile + 16 * half, j0 = (int64_t)tj * kTile;
  const int64_t kb = (int64_t)split * G.kchunk;
  const int64_t ke = min(G.m, kb + G.kchunk);
  const int r = lane & 15, kk = lane >> 4;
  const TI* base = SA + (int64_t)p * G.m * G.ld;
  const bool ci = i0 + r < G.d, cj0 = j0 + r < G.d, cj1 = j0 + 16 + r < G.d;
  f64x4 c0 = {0, 0, 0, 0}, c1 = c0;
  for (int64_t k = kb; k < ke; k += 8) {
    double a[2], b0[2], b1[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int64_t row = k + 4 * q + kk;
      const bool okr = row < ke;
      const TI* rp = base + row * G.ld;
      a[q] = (okr && ci) ? to_f64(rp[i0 + r]) : 0.0;
      b0[q] = (okr && cj0) ? to_f64(rp[j0 + r]) : 0.0;
      b1[q] = (okr && cj1) ? to_f64(rp[j0 + 16 + r]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b0[q], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b1[q], c1, 0, 0, 0);
    }
  }
  // 16 x 16 f64 output: row 4*reg + lane/16, column lane%16
  double* out = part + (w >> 1) * (kTile * kTile) + 16 * half * kTile;
  const int col = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int reg = 0; reg < 4; ++reg) {
    const int row = 4 * reg + rq;
    out[row * kTile + col] = c0[reg];
    out[row * kTile + 16 + col] = c1[reg];
  }
}

// FP32 accumulation on the matrix cores: F32 inputs (16x16x4) or BF16
// inputs (16x16x32, eight consecutive k per lane).
__global__ __launch_bounds__(256, 8) void k_gram_f32_f32(const float* __restrict__ SA, GramPlan G,
                                                         double* __restrict__ part) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + wv;
  const int64_t total = (int64_t)G.batch * G.ntri * G.splits * 2;
  if (w >= total) return;
  int p, t, split, half;
  gram_wave_coords(G, w, p, t, split, half);
  int ti, tj;
  tri_index(t, ti, tj);
  const int64_t i0 = (int64_t)ti * kTile + 16 * half, j0 = (int64_t)tj * kTile;
  const int64_t kb = (int64_t)split * G.kchunk;
  const int64_t ke = min(G.m, kb + G.kchunk);
  const int r = lane & 15, kk = lane >> 4;
  const float* base = SA + (int64_t)p * G.m * G.ld;
  const bool ci = i0 + r < G.d, cj0 = j0 + r < G.d, cj1 = j0 + 16 + r < G.d;
  f32x4 c0 = {0, 0, 0, 0}, c1 = c0;
  for (int64_t k = kb; k < ke; k += 16) {
    float a[4], b0[4], b1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = k + 4 * q + kk;
      const bool okr = row < ke;
      const float* rp = base + row * G.ld;
      a[q] = (okr && ci) ? rp[i0 + r] : 0.f;
      b0[q] = (okr && cj0) ? rp[j0 + r] : 0.f;
      b1[q] = (okr && cj1) ? rp[j0 + 16 + r] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b0[q], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b1[q], c1, 0, 0, 0);
    }
  }
  // 16 x 16 f32 output: row 4*(lane/16) + reg, column lane%16
  double* out = part + (w >> 1) * (kTile * kTile) + 16 * half * kTile;
  const int col = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int reg = 0; reg < 4; ++reg) {
    const int row = 4 * rq + reg;
    out[row * kTile + col] = (double)c0[reg];
    out[row * kTile + 16 + col] = (double)c1[reg];
  }
}

__global__ __launch_bounds__(256, 6) void k_gram_bf16_f32(const uint16_t* __restrict__ SA,
                                                          GramPlan G, double* __restrict__ part) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + wv;
  const int64_t total = (int64_t)G.batch * G.ntri * G.splits * 2;
  if (w >= total) return;
  int p, t, split, half;
  gram_wave_coords(G, w, p, t, split, half);
  int ti, tj;
  tri_index(t, ti, tj);
  const int64_t i0 = (int64_t)ti * kTile + 16 * half, j0 = (int64_t)tj * kTile;
  const int64_t kb = (int64_t)split * G.kchunk;
  const int64_t ke = min(G.m, kb + G.kchunk);
  const int r = lane & 15, kk = lane >> 4;
  const uint16_t* base = SA + (int64_t)p * G.m * G.ld;
  const bool ci = i0 + r < G.d, cj0 = j0 + r < G.d, cj1 = j0 + 16 + r < G.d;
  f32x4 c0 = {0, 0, 0, 0}, c1 = c0;
  // lane supplies A[i = lane%16][k = 8*(lane/16) + e]; A and B use the same k map
  for (int64_t k = kb; k < ke; k += 32) {
    bf16x8 a, b0, b1;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t row = k + 8 * kk + e;
      const bool okr = row < ke;
      const uint16_t* rp = base + row * G.ld;
      a[e] = (short)((okr && ci) ? rp[i0 + r] : 0);
      b0[e] = (short)((okr && cj0) ? rp[j0 + r] : 0);
      b1[e] = (short)((okr && cj1) ? rp[j0 + 16 + r] : 0);
    }
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, c1, 0, 0, 0);
  }
  double* out = part + (w >> 1) * (kTile * kTile) + 16 * half * kTile;
  const int col = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int reg = 0; reg < 4; ++reg) {
    const int row = 4 * rq + reg;
    out[row * kTile + col] = (double)c0[reg];
    out[row * kTile + 16 + col] = (double)c1[reg];
  }
}

// Sum the split-K partials in ascending split order and write both halves.
// acc32: add the partials in float (the F32-accumulation variants).
__global__ __launch_bounds__(256) void k_gram_reduce(GramPlan G, const double* __restrict__ part,
                                                     double* __restrict__ H, int32_t acc32) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t dd = G.d * G.d;
  if (idx >= (int64_t)G.batch * dd) return;
  const int p = (int)(idx / dd);
  const int64_t e = idx - (int64_t)p * dd;
  const int64_t i = e / G.d, j = e - (e / G.d) * G.d;
  int64_t a = i, b = j;
  if (a / kTile > b / kTile) {
    a = j;
    b = i;
  }
  const int ti = (int)(a / kTile), tj = (int)(b / kTile);
  const int t = tj * (tj + 1) / 2 + ti;
  const int li = (int)(a - (int64_t)ti * kTile), lj = (int)(b - (int64_t)tj * kTile);
  const double* src = part + (((int64_t)p * G.ntri + t) * G.splits) * (kTile * kTile);
  // inside a diagonal tile the lower half mirrors the upper half
  int64_t off = (ti == tj && li > lj) ? (lj * kTile + li) : (li * kTile + lj);
  // loads of eight slices are issued together, then added in ascending order
  const int64_t stride = (int64_t)kTile * kTile;
  if (acc32) {
    float s = 0.f;
    int q = 0;
    for (; q + 8 <= G.splits; q += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)(q + u) * stride + off];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (float)v[u];
    }
    for (; q < G.splits; ++q) s += (float)src[(int64_t)q * stride + off];
    H[idx] = (double)s;
  } else {
    double s = 0.0;
    int q = 0;
    for (; q + 8 <= G.splits; q += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)(q + u) * stride + off];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < G.splits; ++q) s += src[(int64_t)q * stride + off];
    H[idx] = s;
  }
}

hipError_t launch_gram(const void* SA, int32_t in_dtype, int64_t m, int64_t d, int64_t ld,
                       int32_t batch, int32_t acc_dtype, double* H, void* partials,
                       hipStream_t st) {
  const GramPlan G = make_gram_plan(m, d, ld, batch);
  const int64_t waves = (int64_t)batch * G.ntri * G.splits * 2;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  double* part = static_cast<double*>(partials);
  if (acc_dtype == 0) {
    if (in_dtype == 0)
      hipLaunchKernelGGL(k_gram_f64<double>, dim3(blocks), dim3(256), 0, st,
                         static_cast<const double*>(SA), G, part);
    else if (in_dtype == 1)
      hipLaunchKernelGGL(k_gram_f64<float>, dim3(blocks), dim3(256), 0, st,
                         static_cast<const float*>(SA), G, part);
    else
      return hipErrorInvalidValue;
  } else {
    if (in_dtype == 1)
      hipLaunchKernelGGL(k_gram_f32_f32, dim3(blocks), dim3(256), 0, st,
                         static_cast<const float*>(SA), G, part);
    else if (in_dtype == 2)
      hipLaunchKernelGGL(k_gram_bf16_f32, dim3(blocks), dim3(256), 0, st,
                         static_cast<const uint16_t*>(SA), G, part);
    else
      return hipErrorInvalidValue;
  }
  const int64_t n_out = (int64_t)batch * d * d;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st, G,
                     part, H, acc_dtype == 0 ? 0 : 1);
  return hipGetLastError();
}

}  // namespace ihs
