// The sketched Hessian H = (SA)^T (SA) (Sec. 1, the T_QP term; App. A.1.1:
// forming it costs O(m d^2)) on gfx950 matrix cores.
//
// One workgroup owns a tile of the upper triangle of H (64 x 64, or 128 x 128
// from d = 1024 on, for FP64 accumulation; 64 x 64 for FP32 products; 128 x
// 128 for BF16 products) for a contiguous slice
// of the m rows of SA (split-K). Both operand panels of a stage are staged
// through LDS with coalesced row loads and reused by all four wavefronts;
// diagonal tiles stage one panel. Partial tiles are summed over the slices
// in a fixed order and mirrored into both triangles, so H is exactly
// symmetric and bitwise reproducible.
#include <algorithm>

#include "kernels.hpp"

namespace ihs {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

// Output tile edge: 64 for the FP64 and FP32 products (16 x 16 x 4), 128 for
// the BF16 ones (16 x 16 x 32, eight times the work per operand load, so a
// tile must reuse each staged operand more to keep the matrix cores fed).
// From d = 1024 on the FP64 products also take 128 x 128 tiles: every tile
// re-reads its two panels of SA, so the panels' traffic from L2 halves (at
// d = 512 the wide tiles leave too few workgroups to fill the chip).
constexpr int kTileF64 = 64;
constexpr int kTileF64Wide = 128;
constexpr int kF64WideMinD = 1024;
constexpr int kTileF32 = 64;
constexpr int kTileBf16 = 128;

struct GramPlan {
  int64_t m, d, ld;
  int32_t batch, tile, ntile, ntri, splits;
  int64_t kchunk;
};

static int tile_of(int32_t in_dtype, int32_t acc, int64_t d) {
  if (in_dtype == 2) return kTileBf16;
  if (acc == 1) return kTileF32;
  return d >= kF64WideMinD ? kTileF64Wide : kTileF64;
}

// Workgroups of each kernel that fit on one CU at once (LDS and registers):
// the slices are sized so that all workgroups run in one round, since a
// second, partly filled round would double the time. `per_cu` caps the
// workgroups per CU below that (a Gram that runs beside latency-bound work
// leaves registers free for it).
constexpr int kCUs = 256;

static GramPlan make_gram_plan(int64_t m, int64_t d, int64_t ld, int32_t batch, int32_t acc,
                               int32_t in, int32_t per_cu = 4) {
  GramPlan g;
  g.m = m;
  g.d = d;
  g.ld = ld;
  g.batch = batch;
  g.tile = tile_of(in, acc, d);
  g.ntile = (int32_t)((d + g.tile - 1) / g.tile);
  g.ntri = g.ntile * (g.ntile + 1) / 2;
  // the wide FP64 tiles: two workgroups per CU (LDS and registers); BF16
  // products: two per CU as well, since each extra slice adds a tile of FP32
  // partials to write and reduce (8192 x 1024: 51 us at four, 42 at two)
  const int32_t cap = (g.tile == kTileF64Wide || in == 2) ? 2 : 4;
  const int64_t slots = (int64_t)kCUs * std::max(1, std::min(per_cu, cap));
  const int64_t tiles = (int64_t)batch * g.ntri;
  int64_t splits = std::max<int64_t>(1, slots / tiles);
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, m / 128));  // >= 128 rows a slice
  splits = std::max<int64_t>(1, std::min<int64_t>(splits, 64));
  int64_t kc = (m + splits - 1) / splits;
  kc = (kc + 31) / 32 * 32;
  g.kchunk = std::max<int64_t>(kc, 32);
  g.splits = (int32_t)std::max<int64_t>(1, (m + g.kchunk - 1) / g.kchunk);
  return g;
}

// BF16 inputs are first copied into rows of eight: element (k, c) of a
// problem's m x d block at ((k / 8) * d + c) * 8 + k % 8, zero-padded to a
// multiple of 8 rows, so a lane's eight consecutive k of one column (the
// operand of a 16 x 16 x 32 product) are one 16-byte load.
__host__ __device__ __forceinline__ int64_t bf16_rows8(int64_t m) { return (m + 7) / 8 * 8; }

size_t gram_partials_bytes(int64_t m, int64_t d, int32_t batch, int32_t in, int32_t acc) {
  const GramPlan g = make_gram_plan(m, d, d, batch, acc, in);
  const size_t es = acc == 0 ? sizeof(double) : sizeof(float);
  size_t bytes = (size_t)batch * g.ntri * g.splits * g.tile * g.tile * es;
  if (in == 2) bytes = (bytes + 255) / 256 * 256 + (size_t)batch * bf16_rows8(m) * d * 2;
  return bytes;
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

// Workgroup -> (problem, upper-triangle tile, slice of the m rows).
__device__ __forceinline__ void gram_coords(const GramPlan& G, int& p, int& ti, int& tj,
                                            int& split) {
  const int64_t q = blockIdx.x;
  split = (int)(q % G.splits);
  const int t = (int)((q / G.splits) % G.ntri);
  p = (int)(q / ((int64_t)G.splits * G.ntri));
  tri_index(t, ti, tj);
}

// ---------------------------------------------------------------------------
// FP64 matrix cores (16 x 16 x 4), F64 inputs or F32 inputs widened exactly.
// One workgroup of four wavefronts owns a 64 x 64 tile of H for one slice of
// rows; each wavefront a 32 x 32 quarter (2 x 2 products). The two 16 x 64
// operand panels of a stage go through LDS (coalesced row loads), double
// buffered: the next stage's loads are issued before the current stage's
// products, and written to the other buffer after them.
// ---------------------------------------------------------------------------
constexpr int kKcF64 = 16;            // rows per stage

template <typename TI, int TILE>
__global__ __launch_bounds__(256, TILE == 128 ? 2 : 4) void k_gram_f64(
    const TI* __restrict__ SA, GramPlan G, double* __restrict__ part) {
  constexpr int kPad = TILE + 1;  // LDS row pitch (doubles)
  constexpr int MT = TILE / 32;   // 16 x 16 output blocks per wavefront edge
  __shared__ double As[2][kKcF64][kPad];
  __shared__ double Bs[2][kKcF64][kPad];
  int p, ti, tj, split;
  gram_coords(G, p, ti, tj, split);
  const bool diag = ti == tj;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int64_t i0 = (int64_t)ti * TILE, j0 = (int64_t)tj * TILE;
  const int64_t kb = (int64_t)split * G.kchunk;
  const int64_t ke = min(G.m, kb + G.kchunk);
  const TI* base = SA + (int64_t)p * G.m * G.ld;
  // thread tid stages elements e = tid + 256 u of each kKcF64 x TILE panel
  constexpr int kPer = kKcF64 * TILE / 256;
  double ra[kPer], rb[kPer];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int r = e / TILE, c = e % TILE;
      const int64_t row = k0 + r;
      const bool ok = row < ke;
      ra[u] = (ok && i0 + c < G.d) ? to_f64(base[row * G.ld + i0 + c]) : 0.0;
      if (!diag) rb[u] = (ok && j0 + c < G.d) ? to_f64(base[row * G.ld + j0 + c]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int r = e / TILE, c = e % TILE;
      As[buf][r][c] = ra[u];
      if (!diag) Bs[buf][r][c] = rb[u];
    }
  };
  // wavefront (wr, wc) of the 2 x 2 grid owns a (TILE/2) x (TILE/2) block
  const int wr = wv >> 1, wc = wv & 1;
  constexpr int HALF = TILE / 2;
  f64x4 acc[MT][MT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < MT; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nstage = (int)((ke - kb + kKcF64 - 1) / kKcF64);
  if (nstage > 0) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int sidx = 0; sidx < nstage; ++sidx) {
    const int buf = sidx & 1;
    if (sidx + 1 < nstage) load(kb + (int64_t)(sidx + 1) * kKcF64);
    const double(*Bp)[kPad] = diag ? As[buf] : Bs[buf];
#pragma unroll
    for (int k4 = 0; k4 < kKcF64; k4 += 4) {
      const int kr = k4 + (lane >> 4), cl = lane & 15;
      double a[MT], b[MT];
#pragma unroll
      for (int q = 0; q < MT; ++q) {
        a[q] = As[buf][kr][HALF * wr + 16 * q + cl];
        b[q] = Bp[kr][HALF * wc + 16 * q + cl];
      }
#pragma unroll
      for (int x = 0; x < MT; ++x)
#pragma unroll
        for (int y = 0; y < MT; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    if (sidx + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }
  // 16 x 16 f64 output blocks: row 4*reg + lane/16, column lane%16
  double* out = part + ((((int64_t)p * G.ntri) + (blockIdx.x / G.splits) % G.ntri) * G.splits +
                        split) * (TILE * TILE);
#pragma unroll
  for (int x = 0; x < MT; ++x)
#pragma unroll
    for (int y = 0; y < MT; ++y)
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) {
        const int row = HALF * wr + 16 * x + 4 * reg + (lane >> 4);
        const int col = HALF * wc + 16 * y + (lane & 15);
        out[row * TILE + col] = acc[x][y][reg];
      }
}

// ---------------------------------------------------------------------------
// FP32 accumulation of F32 inputs (16 x 16 x 4 products): the FP64 kernel's
// 64 x 64 tiles and staging, in single precision.
// ---------------------------------------------------------------------------
constexpr int kKcF32 = 16;
constexpr int kPadF32 = kTileF32 + 4;

__global__ __launch_bounds__(256, 4) void k_gram_f32_f32(const float* __restrict__ SA, GramPlan G,
                                                         float* __restrict__ part) {
  __shared__ float As[2][kKcF32][kPadF32];
  __shared__ float Bs[2][kKcF32][kPadF32];
  int p, ti, tj, split;
  gram_coords(G, p, ti, tj, split);
  const bool diag = ti == tj;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int64_t i0 = (int64_t)ti * kTileF32, j0 = (int64_t)tj * kTileF32;
  const int64_t kb = (int64_t)split * G.kchunk;
  const int64_t ke = min(G.m, kb + G.kchunk);
  const float* base = SA + (int64_t)p * G.m * G.ld;
  constexpr int kPer = kKcF32 * kTileF32 / 256;  // 4
  float ra[kPer], rb[kPer];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int r = e / kTileF32, c = e % kTileF32;
      const int64_t row = k0 + r;
      const bool ok = row < ke;
      ra[u] = (ok && i0 + c < G.d) ? base[row * G.ld + i0 + c] : 0.f;
      if (!diag) rb[u] = (ok && j0 + c < G.d) ? base[row * G.ld + j0 + c] : 0.f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int r = e / kTileF32, c = e % kTileF32;
      As[buf][r][c] = ra[u];
      if (!diag) Bs[buf][r][c] = rb[u];
    }
  };
  const int wr = wv >> 1, wc = wv & 1;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nstage = (int)((ke - kb + kKcF32 - 1) / kKcF32);
  if (nstage > 0) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int sidx = 0; sidx < nstage; ++sidx) {
    const int buf = sidx & 1;
    if (sidx + 1 < nstage) load(kb + (int64_t)(sidx + 1) * kKcF32);
    const float(*Bp)[kPadF32] = diag ? As[buf] : Bs[buf];
#pragma unroll
    for (int k4 = 0; k4 < kKcF32; k4 += 4) {
      const int kr = k4 + (lane >> 4), cl = lane & 15;
      float a[2], b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        a[q] = As[buf][kr][32 * wr + 16 * q + cl];
        b[q] = Bp[kr][32 * wc + 16 * q + cl];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    if (sidx + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }
  // 16 x 16 f32 output blocks: row 4*(lane/16) + reg, column lane%16
  float* out = part + ((((int64_t)p * G.ntri) + (blockIdx.x / G.splits) % G.ntri) * G.splits +
                       split) * (kTileF32 * kTileF32);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) {
        const int row = 32 * wr + 16 * x + 4 * (lane >> 4) + reg;
        const int col = 32 * wc + 16 * y + (lane & 15);
        out[row * kTileF32 + col] = acc[x][y][reg];
      }
}

// ---------------------------------------------------------------------------
// FP32 accumulation of BF16 inputs (16 x 16 x 32 products). The inputs are
// first regrouped into rows of eight (k_bf16_rows8), so every staging load
// and every operand read is 16 bytes. One workgroup of four wavefronts owns
// a 128 x 128 tile; each wavefront a 64 x 64 quarter (4 x 4 products); a
// stage is 32 rows (four groups of eight).
// ---------------------------------------------------------------------------
constexpr int kKcBf16 = 32;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One thread per 16-byte cell (eight rows of one column): the eight reads of
// a wavefront's threads cover eight rows of 64 consecutive columns.
__global__ __launch_bounds__(256) void k_bf16_rows8(const uint16_t* __restrict__ SA, int64_t m,
                                                    int64_t d, int64_t ld, int32_t batch,
                                                    u32x4* __restrict__ out) {
  const int64_t groups = bf16_rows8(m) / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;  // output cell
  if (idx >= (int64_t)batch * groups * d) return;
  const int64_t p = idx / (groups * d);
  const int64_t rem = idx - p * groups * d;
  const int64_t g = rem / d, c = rem - (rem / d) * d;
  uint32_t w[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int64_t k0 = 8 * g + 2 * h;
    const uint32_t lo = k0 < m ? SA[(p * m + k0) * ld + c] : 0u;
    const uint32_t hi = k0 + 1 < m ? SA[(p * m + k0 + 1) * ld + c] : 0u;
    w[h] = lo | (hi << 16);
  }
  out[idx] = u32x4{w[0], w[1], w[2], w[3]};
}

__global__ __launch_bounds__(256, 4) void k_gram_bf16_f32(const uint16_t* __restrict__ S8,
                                                          GramPlan G, float* __restrict__ part) {
  // [buffer][group of 8 rows][column] of 16-byte cells
  __shared__ u32x4 At[2][kKcBf16 / 8][kTileBf16];
  __shared__ u32x4 Bt[2][kKcBf16 / 8][kTileBf16];
  int p, ti, tj, split;
  gram_coords(G, p, ti, tj, split);
  const bool diag = ti == tj;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int64_t i0 = (int64_t)ti * kTileBf16, j0 = (int64_t)tj * kTileBf16;
  const int64_t kb = (int64_t)split * G.kchunk;  // a multiple of 32
  const int64_t ke = min(bf16_rows8(G.m), kb + G.kchunk);
  const u32x4* base = reinterpret_cast<const u32x4*>(S8) + (int64_t)p * (bf16_rows8(G.m) / 8) * G.d;
  constexpr int kPer = (kKcBf16 / 8) * kTileBf16 / 256;  // 2 cells per thread and panel
  u32x4 ra[kPer], rb[kPer];
  const u32x4 zero = {0u, 0u, 0u, 0u};
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int g = e / kTileBf16, c = e % kTileBf16;
      const int64_t row = k0 + 8 * g;
      const bool ok = row < ke;
      ra[u] = (ok && i0 + c < G.d) ? base[(row / 8) * G.d + i0 + c] : zero;
      if (!diag) rb[u] = (ok && j0 + c < G.d) ? base[(row / 8) * G.d + j0 + c] : zero;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int g = e / kTileBf16, c = e % kTileBf16;
      At[buf][g][c] = ra[u];
      if (!diag) Bt[buf][g][c] = rb[u];
    }
  };
  const int wr = wv >> 1, wc = wv & 1;
  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nstage = (int)((ke - kb + kKcBf16 - 1) / kKcBf16);
  if (nstage > 0) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int sidx = 0; sidx < nstage; ++sidx) {
    const int buf = sidx & 1;
    if (sidx + 1 < nstage) load(kb + (int64_t)(sidx + 1) * kKcBf16);
    const u32x4(*Bp)[kTileBf16] = diag ? At[buf] : Bt[buf];
    // lane supplies operand row lane%16 at rows 8*(lane/16) .. +7 of the stage
    const int g = lane >> 4, cl = lane & 15;
    bf16x8 a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const u32x4 av = At[buf][g][64 * wr + 16 * q + cl];
      const u32x4 bv = Bp[g][64 * wc + 16 * q + cl];
      a[q] = __builtin_bit_cast(bf16x8, av);
      b[q] = __builtin_bit_cast(bf16x8, bv);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
    if (sidx + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }
  float* out = part + ((((int64_t)p * G.ntri) + (blockIdx.x / G.splits) % G.ntri) * G.splits +
                       split) * (kTileBf16 * kTileBf16);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) {
        const int row = 64 * wr + 16 * x + 4 * (lane >> 4) + reg;
        const int col = 64 * wc + 16 * y + (lane & 15);
        out[row * kTileBf16 + col] = acc[x][y][reg];
      }
}

// Sum the split-K partials in ascending split order and write both halves.
// One workgroup per 64 x 16 strip of a 64 x 64 block of a tile, four
// elements per thread with all their loads in flight together: the partials
// are read along rows, the strip is written in place and, through LDS,
// transposed into the lower triangle, so every global access is coalesced.
// Diagonal tiles keep their upper half and mirror it. TP: the partials' type
// (double for FP64 accumulation; float otherwise, added in float).
constexpr int kRedStrip = 16;

template <typename TP>
__global__ __launch_bounds__(256) void k_gram_reduce(GramPlan G, const TP* __restrict__ part,
                                                     double* __restrict__ H) {
  __shared__ double S[64][kRedStrip + 1];
  const int T = G.tile, per = T / 64, nstrip = 64 / kRedStrip;
  int64_t q = blockIdx.x;
  const int strip = (int)(q % nstrip);
  q /= nstrip;
  const int sb = (int)(q % (per * per));
  q /= per * per;
  const int t = (int)(q % G.ntri);
  const int p = (int)(q / G.ntri);
  int ti, tj;
  tri_index(t, ti, tj);
  const bool diag = ti == tj;
  const int sr = sb / per, sc = sb % per;
  if (diag && sr > sc) return;  // below the diagonal of a diagonal tile: mirrored
  const int64_t i0 = (int64_t)ti * T + 64 * sr, j0 = (int64_t)tj * T + 64 * sc + kRedStrip * strip;
  const TP* src = part + (((int64_t)p * G.ntri + t) * G.splits) * ((int64_t)T * T);
  const int64_t stride = (int64_t)T * T;
  double* Hp = H + (int64_t)p * G.d * G.d;
  constexpr int kE = 64 * kRedStrip / 256;  // 4 elements per thread
  int64_t off[kE];
  TP s[kE];
#pragma unroll
  for (int u = 0; u < kE; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int r = e / kRedStrip, c = e % kRedStrip;
    off[u] = (int64_t)(64 * sr + r) * T + 64 * sc + kRedStrip * strip + c;
    s[u] = (TP)0;
  }
  // loads of two slices of every element are issued together, then added in
  // ascending slice order
  int k = 0;
  for (; k + 2 <= G.splits; k += 2) {
    TP v[2][kE];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < kE; ++u) v[h][u] = src[(int64_t)(k + h) * stride + off[u]];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < kE; ++u) s[u] += v[h][u];
  }
  for (; k < G.splits; ++k)
#pragma unroll
    for (int u = 0; u < kE; ++u) s[u] += src[(int64_t)k * stride + off[u]];
  const int cdiag = kRedStrip * strip;  // this strip's first column within the block
#pragma unroll
  for (int u = 0; u < kE; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int r = e / kRedStrip, c = e % kRedStrip;
    const double v = (double)s[u];
    S[r][c] = v;
    const int64_t gi = i0 + r, gj = j0 + c;
    if (gi < G.d && gj < G.d && (!diag || sr < sc || r <= cdiag + c)) Hp[gi * G.d + gj] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * kRedStrip; e += 256) {
    const int c = e / 64, r = e % 64;  // write row j0 + c, column i0 + r
    const int64_t gi = i0 + r, gj = j0 + c;
    if (gi < G.d && gj < G.d && (!diag || sr < sc || r < cdiag + c)) Hp[gj * G.d + gi] = S[r][c];
  }
}

hipError_t launch_gram(const void* SA, int32_t in_dtype, int64_t m, int64_t d, int64_t ld,
                       int32_t batch, int32_t acc_dtype, double* H, void* partials,
                       hipStream_t st, int32_t per_cu) {
  const GramPlan G = make_gram_plan(m, d, ld, batch, acc_dtype, in_dtype, per_cu);
  const unsigned blocks = (unsigned)((int64_t)batch * G.ntri * G.splits);
  const dim3 rgrid((unsigned)((int64_t)batch * G.ntri * (G.tile / 64) * (G.tile / 64) *
                              (64 / kRedStrip)));
  if (acc_dtype == 0) {
    double* part = static_cast<double*>(partials);
    const bool wide = G.tile == kTileF64Wide;
    if (in_dtype == 0 && wide)
      hipLaunchKernelGGL((k_gram_f64<double, kTileF64Wide>), dim3(blocks), dim3(256), 0, st,
                         static_cast<const double*>(SA), G, part);
    else if (in_dtype == 0)
      hipLaunchKernelGGL((k_gram_f64<double, kTileF64>), dim3(blocks), dim3(256), 0, st,
                         static_cast<const double*>(SA), G, part);
    else if (in_dtype == 1 && wide)
      hipLaunchKernelGGL((k_gram_f64<float, kTileF64Wide>), dim3(blocks), dim3(256), 0, st,
                         static_cast<const float*>(SA), G, part);
    else if (in_dtype == 1)
      hipLaunchKernelGGL((k_gram_f64<float, kTileF64>), dim3(blocks), dim3(256), 0, st,
                         static_cast<const float*>(SA), G, part);
    else
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gram_reduce<double>, rgrid, dim3(256), 0, st, G, part, H);
  } else {
    float* part = static_cast<float*>(partials);
    if (in_dtype == 1) {
      hipLaunchKernelGGL(k_gram_f32_f32, dim3(blocks), dim3(256), 0, st,
                         static_cast<const float*>(SA), G, part);
    } else if (in_dtype == 2) {
      const size_t pbytes = (size_t)batch * G.ntri * G.splits * G.tile * G.tile * sizeof(float);
      uint16_t* s8 = reinterpret_cast<uint16_t*>(static_cast<char*>(partials) +
                                                 (pbytes + 255) / 256 * 256);
      const int64_t cells = (int64_t)batch * (bf16_rows8(m) / 8) * d;
      hipLaunchKernelGGL(k_bf16_rows8, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st,
                         static_cast<const uint16_t*>(SA), m, d, ld, batch,
                         reinterpret_cast<u32x4*>(s8));
      hipLaunchKernelGGL(k_gram_bf16_f32, dim3(blocks), dim3(256), 0, st, s8, G, part);
    } else {
      return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_gram_reduce<float>, rgrid, dim3(256), 0, st, G, part, H);
  }
  return hipGetLastError();
}

}  // namespace ihs
