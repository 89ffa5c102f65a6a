// The sketched Hessian H = (SA)^T (SA) (Sec. 1, the T_QP term; App. A.1.1,
// "O(m d^2) to compute the approximate Hessian") on gfx950 matrix cores.
//
// Each wavefront owns one 32 x 32 tile of the upper triangle of H and a
// contiguous slice of the m rows of SA (split-K). Operands come straight from
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

// Operand fetch converting to the MFMA input type.
__device__ __forceinline__ double ld_f64(const void* SA, int32_t dt, int64_t idx) {
  if (dt == 0) return static_cast<const double*>(SA)[idx];
  if (dt == 1) return (double)static_cast<const float*>(SA)[idx];
  return bf16_bits_to_f64(static_cast<const uint16_t*>(SA)[idx]);
}

// FP64 (or F32 inputs widened to FP64) on the FP64 matrix cores.
__global__ __launch_bounds__(256) void k_gram_f64(const void* __restrict__ SA, int32_t in_dt,
                                                  GramPlan G, double* __restrict__ part) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + wv;
  const int64_t total = (int64_t)G.batch * G.ntri * G.splits;
  if (w >= total) return;
  const int split = (int)(w % G.splits);
  const int t = (int)((w / G.splits) % G.ntri);
  const int p = (int)(w / ((int64_t)G.splits * G.ntri));
  int ti, tj;
  tri_index(t, ti, tj);
  const int64_t i0 = (int64_t)ti * kTile, j0 = (int64_t)tj * kTile;
  const int64_t kb = (int64_t)split * G.kchunk;
  const int64_t ke = min(G.m, kb + G.kchunk);
  const int r = lane & 15, kk = lane >> 4;
  const int64_t base = (int64_t)p * G.m * G.ld;
  const bool ci0 = i0 + r < G.d, ci1 = i0 + 16 + r < G.d;
  const bool cj0 = j0 + r < G.d, cj1 = j0 + 16 + r < G.d;
  f64x4 c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
  for (int64_t k = kb; k < ke; k += 16) {
    double a0[4], a1[4], b0[4], b1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = k + 4 * q + kk;
      const bool okr = row < ke;
      const int64_t off = base + row * G.ld;
      a0[q] = (okr && ci0) ? ld_f64(SA, in_dt, off + i0 + r) : 0.0;
      a1[q] = (okr && ci1) ? ld_f64(SA, in_dt, off + i0 + 16 + r) : 0.0;
      b0[q] = (okr && cj0) ? ld_f64(SA, in_dt, off + j0 + r) : 0.0;
      b1[q] = (okr && cj1) ? ld_f64(SA, in_dt, off + j0 + 16 + r) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[q], b0[q], c00, 0, 0, 0);
      c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[q], b1[q], c01, 0, 0, 0);
      c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[q], b0[q], c10, 0, 0, 0);
      c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[q], b1[q], c11, 0, 0, 0);
    }
  }
  // D(i, j) of a 16 x 16 block sits in lane 16*(i%4)... : row 4*reg + lane/16, col lane%16
  double* out = part + w * (kTile * kTile);
  const int col = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int reg = 0; reg < 4; ++reg) {
    const int row = 4 * reg + rq;
    out[row * kTile + col] = c00[reg];
    out[row * kTile + 16 + col] = c01[reg];
    out[(16 + row) * kTile + col] = c10[reg];
    out[(16 + row) * kTile + 16 + col] = c11[reg];
  }
}

// FP32 accumulation on the FP32 matrix cores: F32 inputs (16x16x4) or BF16
// inputs (16x16x32, eight consecutive k per lane).
__global__ __launch_bounds__(256) void k_gram_f32acc(const void* __restrict__ SA, int32_t in_dt,
                                                     GramPlan G, double* __restrict__ part) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + wv;
  const int64_t total = (int64_t)G.batch * G.ntri * G.splits;
  if (w >= total) return;
  const int split = (int)(w % G.splits);
  const int t = (int)((w / G.splits) % G.ntri);
  const int p = (int)(w / ((int64_t)G.splits * G.ntri));
  int ti, tj;
  tri_index(t, ti, tj);
  const int64_t i0 = (int64_t)ti * kTile, j0 = (int64_t)tj * kTile;
  const int64_t kb = (int64_t)split * G.kchunk;
  const int64_t ke = min(G.m, kb + G.kchunk);
  const int r = lane & 15, kk = lane >> 4;
  const int64_t base = (int64_t)p * G.m * G.ld;
  const bool ci0 = i0 + r < G.d, ci1 = i0 + 16 + r < G.d;
  const bool cj0 = j0 + r < G.d, cj1 = j0 + 16 + r < G.d;
  f32x4 c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
  if (in_dt == 1) {
    const float* S = static_cast<const float*>(SA);
    for (int64_t k = kb; k < ke; k += 16) {
      float a0[4], a1[4], b0[4], b1[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = k + 4 * q + kk;
        const bool okr = row < ke;
        const int64_t off = base + row * G.ld;
        a0[q] = (okr && ci0) ? S[off + i0 + r] : 0.f;
        a1[q] = (okr && ci1) ? S[off + i0 + 16 + r] : 0.f;
        b0[q] = (okr && cj0) ? S[off + j0 + r] : 0.f;
        b1[q] = (okr && cj1) ? S[off + j0 + 16 + r] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c00 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[q], b0[q], c00, 0, 0, 0);
        c01 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[q], b1[q], c01, 0, 0, 0);
        c10 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[q], b0[q], c10, 0, 0, 0);
        c11 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[q], b1[q], c11, 0, 0, 0);
      }
    }
  } else {
    const uint16_t* S = static_cast<const uint16_t*>(SA);
    // 16x16x32: lane supplies A[i = lane%16][k = 8*(lane/16) + e], e < 8
    for (int64_t k = kb; k < ke; k += 32) {
      bf16x8 a0, a1, b0, b1;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t row = k + 8 * kk + e;
        const bool okr = row < ke;
        const int64_t off = base + row * G.ld;
        a0[e] = (short)((okr && ci0) ? S[off + i0 + r] : 0);
        a1[e] = (short)((okr && ci1) ? S[off + i0 + 16 + r] : 0);
        b0[e] = (short)((okr && cj0) ? S[off + j0 + r] : 0);
        b1[e] = (short)((okr && cj1) ? S[off + j0 + 16 + r] : 0);
      }
      c00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, c00, 0, 0, 0);
      c01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, c01, 0, 0, 0);
      c10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, c10, 0, 0, 0);
      c11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, c11, 0, 0, 0);
    }
  }
  // 16x16 f32 output: row 4*(lane/16) + reg, col lane%16
  double* out = part + w * (kTile * kTile);
  const int col = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int reg = 0; reg < 4; ++reg) {
    const int row = 4 * rq + reg;
    out[row * kTile + col] = (double)c00[reg];
    out[row * kTile + 16 + col] = (double)c01[reg];
    out[(16 + row) * kTile + col] = (double)c10[reg];
    out[(16 + row) * kTile + 16 + col] = (double)c11[reg];
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
  if (acc32) {
    float s = 0.f;
    for (int q = 0; q < G.splits; ++q) s += (float)src[(int64_t)q * kTile * kTile + off];
    H[idx] = (double)s;
  } else {
    double s = 0.0;
    for (int q = 0; q < G.splits; ++q) s += src[(int64_t)q * kTile * kTile + off];
    H[idx] = s;
  }
}

hipError_t launch_gram(const void* SA, int32_t in_dtype, int64_t m, int64_t d, int64_t ld,
                       int32_t batch, int32_t acc_dtype, double* H, void* partials,
                       hipStream_t st) {
  const GramPlan G = make_gram_plan(m, d, ld, batch);
  const int64_t waves = (int64_t)batch * G.ntri * G.splits;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  double* part = static_cast<double*>(partials);
  if (acc_dtype == 0) {
    hipLaunchKernelGGL(k_gram_f64, dim3(blocks), dim3(256), 0, st, SA, in_dtype, G, part);
  } else {
    hipLaunchKernelGGL(k_gram_f32acc, dim3(blocks), dim3(256), 0, st, SA, in_dtype, G, part);
  }
  const int64_t n_out = (int64_t)batch * d * d;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, st, G,
                     part, H, acc_dtype == 0 ? 0 : 1);
  return hipGetLastError();
}

}  // namespace ihs
