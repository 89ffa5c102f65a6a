// The two dense sketches of Sec. 2 ("Sketching Results") that the paper
// compares the sparse embeddings with, on gfx950.
//
// SRHT, S = (1/sqrt(m)) P H D (Sec. 2; "Time Complexity of sketching
// methods": a fast Hadamard transform plus O(n) for P and D). The rows of A,
// signed by D and padded with zero rows to N = 2^ceil(log2 n), are
// transformed along the row index for every column by the radix-2 recursion
// (stages h = 1, 2, 4, ..., each pair (y_i, y_{i+h}) -> (y_i + y_{i+h},
// y_i - y_{i+h})), then P picks m rows and the scale is applied once. A pass
// over the N x d buffer takes up to kPassBits consecutive stages: a tile is
// the 2^k rows that differ only in those index bits, times 16 columns (one
// 128-byte segment per row), held in LDS while its stages run. Every
// butterfly is the one of the recursion, so the result is bitwise that of a
// sequential radix-2 transform.
//
// Gaussian, S = G / sqrt(m) (Sec. 2; a dense product, O(m n d)). G is never
// stored: each workgroup draws the 64 x 32 block of G it needs next into LDS
// (Philox4x64-10, four normals per call by the Box-Muller method) beside the
// matching 32 x 64 block of A, and multiplies them on the FP64 matrix cores
// (16 x 16 x 4). Slices of the n rows are summed in a fixed order, so S A is
// bitwise reproducible.
//
// Random choices: Philox4x64-10 under key (seed, iteration), counter
// (index, word, problem, stream): stream 1 gives D (bit 63 of word 1), stream
// 2 the rows of P (floor(word 0 * N / 2^64)), stream 3 the entries of G
// (rows 4q .. 4q+3 of column i from counter (i, q, problem, 3)).
#include <algorithm>

#include "kernels.hpp"

namespace ihs {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr uint64_t kStreamSign = 1, kStreamRows = 2, kStreamGauss = 3;

// ---------------------------------------------------------------------------
// SRHT
// ---------------------------------------------------------------------------
constexpr int kFwhtCols = 16;   // columns per tile: one 128-byte segment per row
constexpr int kPassBits = 8;    // stages per pass: 256 rows x 16 columns = 32 KiB LDS
constexpr int kFwhtThreads = 256;

__device__ __forceinline__ double srht_sign(uint64_t row, int32_t problem, uint64_t seed,
                                            uint64_t iter) {
  const U64x4 w = philox4x64_10(row, 0ull, (uint64_t)problem, kStreamSign, seed, iter);
  return (w.w[1] >> 63) ? -1.0 : 1.0;
}

// One pass: stages b0 .. b0 + kb - 1 of the transform on tiles of 2^kb rows.
// SOURCE: 0 reads Y, 1 reads dense A (F64), 2 dense A (F32); the first pass
// applies D and the zero padding while loading.
template <int SOURCE>
__global__ __launch_bounds__(kFwhtThreads) void k_fwht_pass(const void* __restrict__ A,
                                                           int64_t lda, int64_t n, int64_t d,
                                                           double* Y, int32_t b0, int32_t kb,
                                                           int64_t ntile_rows, uint64_t seed,
                                                           uint64_t iter, int32_t problem) {
  extern __shared__ double tile[];  // [T][kFwhtCols]
  __shared__ double sgn[1 << kPassBits];
  const int T = 1 << kb;
  const int64_t tr = blockIdx.x % ntile_rows;   // which set of 2^kb rows
  const int64_t c0 = (blockIdx.x / ntile_rows) * kFwhtCols;
  const int64_t lo_mask = ((int64_t)1 << b0) - 1;
  const int64_t lo = tr & lo_mask, hi = tr >> b0;
  auto row_of = [&](int j) -> int64_t {
    return lo + ((int64_t)j << b0) + (hi << (b0 + kb));
  };
  if (SOURCE != 0) {
    for (int j = threadIdx.x; j < T; j += kFwhtThreads) {
      const int64_t r = row_of(j);
      sgn[j] = r < n ? srht_sign((uint64_t)r, problem, seed, iter) : 0.0;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < T * kFwhtCols; e += kFwhtThreads) {
    const int j = e / kFwhtCols, c = e % kFwhtCols;
    const int64_t r = row_of(j), col = c0 + c;
    double v = 0.0;
    if (col < d) {
      if (SOURCE == 0) {
        v = Y[r * d + col];
      } else if (r < n) {
        const double a = SOURCE == 1 ? static_cast<const double*>(A)[r * lda + col]
                                     : (double)static_cast<const float*>(A)[r * lda + col];
        v = sgn[j] * a;
      }
    }
    tile[j * kFwhtCols + c] = v;
  }
  __syncthreads();
  // two stages per round where possible (radix 4): the four values of a
  // group take the two butterflies of stage s and then the two of stage s+1
  int s = 0;
  for (; s + 1 < kb; s += 2) {
    const int h = 1 << s;
    for (int e = threadIdx.x; e < (T / 4) * kFwhtCols; e += kFwhtThreads) {
      const int g = e / kFwhtCols, c = e % kFwhtCols;
      const int base = ((g >> s) << (s + 2)) | (g & (h - 1));  // bits s and s+1 clear
      double* p0 = &tile[base * kFwhtCols + c];
      const int step = h * kFwhtCols;
      const double a0 = p0[0], a1 = p0[step], a2 = p0[2 * step], a3 = p0[3 * step];
      const double b0v = a0 + a1, b1v = a0 - a1, b2v = a2 + a3, b3v = a2 - a3;
      p0[0] = b0v + b2v;
      p0[2 * step] = b0v - b2v;
      p0[step] = b1v + b3v;
      p0[3 * step] = b1v - b3v;
    }
    __syncthreads();
  }
  if (s < kb) {  // one stage left
    const int h = 1 << s;
    for (int e = threadIdx.x; e < (T / 2) * kFwhtCols; e += kFwhtThreads) {
      const int g = e / kFwhtCols, c = e % kFwhtCols;
      const int base = ((g >> s) << (s + 1)) | (g & (h - 1));
      double* p0 = &tile[base * kFwhtCols + c];
      const double a0 = p0[0], a1 = p0[h * kFwhtCols];
      p0[0] = a0 + a1;
      p0[h * kFwhtCols] = a0 - a1;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < T * kFwhtCols; e += kFwhtThreads) {
    const int j = e / kFwhtCols, c = e % kFwhtCols;
    const int64_t col = c0 + c;
    if (col < d) Y[row_of(j) * d + col] = tile[j * kFwhtCols + c];
  }
}

__device__ __forceinline__ void store_out(void* SA, int32_t dt, int64_t idx, double v) {
  if (dt == 0) {
    static_cast<double*>(SA)[idx] = v;
  } else if (dt == 1) {
    static_cast<float*>(SA)[idx] = (float)v;
  } else {
    static_cast<uint16_t*>(SA)[idx] = f64_to_bf16_bits(v);
  }
}

// SA[k, :] = scale * Y[row_k, :], one wavefront per sampled row.
__global__ __launch_bounds__(256) void k_srht_sample(const double* __restrict__ Y, int64_t N,
                                                     int64_t d, int64_t m, double scale,
                                                     void* SA, int32_t sa_dtype, int64_t ld_sa,
                                                     uint64_t seed, uint64_t iter,
                                                     int32_t problem) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + wv;
  if (k >= m) return;
  const U64x4 w = philox4x64_10((uint64_t)k, 0ull, (uint64_t)problem, kStreamRows, seed, iter);
  const int64_t r = (int64_t)__umul64hi(w.w[0], (uint64_t)N);
  for (int64_t c = lane; c < d; c += 64)
    store_out(SA, sa_dtype, k * ld_sa + c, Y[r * d + c] * scale);
}

// Y (N x d) = D times the rows of a CSR matrix, zero elsewhere (Y zeroed first).
__global__ __launch_bounds__(256) void k_csr_scatter_signed(const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col_idx,
                                                            const double* __restrict__ vals,
                                                            int64_t n, int64_t d, double* Y,
                                                            int32_t signed_rows, uint64_t seed,
                                                            uint64_t iter, int32_t problem) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + wv;
  if (r >= n) return;
  const double sg = signed_rows ? srht_sign((uint64_t)r, problem, seed, iter) : 1.0;
  for (int64_t e = row_ptr[r] + lane; e < row_ptr[r + 1]; e += 64)
    Y[r * d + col_idx[e]] = sg * vals[e];
}

__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

size_t srht_workspace_bytes(int64_t n, int64_t d) {
  int64_t N = 1;
  while (N < n) N <<= 1;
  return (size_t)N * d * sizeof(double);
}

hipError_t launch_srht(const DenseSketchArgs& a, hipStream_t st) {
  int64_t N = 1;
  int32_t logN = 0;
  while (N < a.n) {
    N <<= 1;
    ++logN;
  }
  const int64_t col_tiles = (a.d + kFwhtCols - 1) / kFwhtCols;
  int32_t npass = std::max<int32_t>(1, (logN + kPassBits - 1) / kPassBits);
  bool loaded = false;
  if (a.csr) {  // densify with the signs into Y; every pass then reads Y
    const int64_t total = N * a.d;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a.work, total);
    if (a.n > 0)
      hipLaunchKernelGGL(k_csr_scatter_signed, dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0, st,
                         a.row_ptr, a.col_idx, static_cast<const double*>(a.A), a.n, a.d, a.work,
                         1, a.seed, a.iter, a.problem);
    loaded = true;
  }
  int32_t b0 = 0;
  for (int32_t p = 0; p < npass || (!loaded && p == 0); ++p) {
    // spread the stages evenly over the passes (a single pass when N = 1)
    const int32_t left = logN - b0, passes_left = std::max<int32_t>(1, npass - p);
    const int32_t kb = std::max<int32_t>(0, (left + passes_left - 1) / passes_left);
    const int64_t ntile_rows = N >> kb;
    const dim3 grid((unsigned)(ntile_rows * col_tiles));
    const size_t lds = (size_t)(1 << kb) * kFwhtCols * sizeof(double);
    if (!loaded) {
      if (a.a_dtype == 0)
        hipLaunchKernelGGL(k_fwht_pass<1>, grid, dim3(kFwhtThreads), lds, st, a.A, a.lda, a.n,
                           a.d, a.work, b0, kb, ntile_rows, a.seed, a.iter, a.problem);
      else
        hipLaunchKernelGGL(k_fwht_pass<2>, grid, dim3(kFwhtThreads), lds, st, a.A, a.lda, a.n,
                           a.d, a.work, b0, kb, ntile_rows, a.seed, a.iter, a.problem);
      loaded = true;
    } else if (kb > 0) {
      hipLaunchKernelGGL(k_fwht_pass<0>, grid, dim3(kFwhtThreads), lds, st, nullptr, a.d, a.n,
                         a.d, a.work, b0, kb, ntile_rows, a.seed, a.iter, a.problem);
    }
    b0 += kb;
  }
  if (a.m > 0)
    hipLaunchKernelGGL(k_srht_sample, dim3((unsigned)((a.m + 3) / 4)), dim3(256), 0, st, a.work, N,
                       a.d, a.m, a.scale, a.SA, a.sa_dtype, a.ld_sa, a.seed, a.iter, a.problem);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gaussian
// ---------------------------------------------------------------------------
constexpr int kGTm = 64;   // output rows per workgroup (4 wavefronts x 16)
constexpr int kGTd = 64;   // output columns per workgroup (4 blocks of 16)
constexpr int kGKc = 32;   // rows of A per LDS stage

struct GaussPlan {
  int64_t m, n, d;
  int32_t mt, dt, splits;
  int64_t kchunk;
};

static GaussPlan make_gauss_plan(int64_t m, int64_t n, int64_t d) {
  GaussPlan g;
  g.m = m;
  g.n = n;
  g.d = d;
  g.mt = (int32_t)((m + kGTm - 1) / kGTm);
  g.dt = (int32_t)((d + kGTd - 1) / kGTd);
  const int64_t tiles = (int64_t)g.mt * g.dt;
  int64_t splits = std::max<int64_t>(1, (2048 + tiles - 1) / tiles);
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, (n + 1023) / 1024));
  splits = std::min<int64_t>(splits, 64);
  int64_t kc = (n + splits - 1) / splits;
  kc = std::max<int64_t>(kGKc, (kc + kGKc - 1) / kGKc * kGKc);
  g.kchunk = kc;
  g.splits = (int32_t)std::max<int64_t>(1, (n + kc - 1) / kc);
  return g;
}

size_t gauss_workspace_bytes(int64_t m, int64_t n, int64_t d) {
  const GaussPlan g = make_gauss_plan(m, n, d);
  return (size_t)g.splits * g.mt * kGTm * g.dt * kGTd * sizeof(double);
}

// Two normals from one pair of 64-bit words (Box and Muller, 1958).
__device__ __forceinline__ void box_muller(uint64_t wa, uint64_t wb, double& z0, double& z1) {
  const double u1 = ((double)(wa >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(wb >> 11) * 0x1.0p-53;
  const double rho = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  z0 = rho * c;
  z1 = rho * s;
}

// Workgroup (tile, split): rows [r0, r0 + 64) x columns [c0, c0 + 64) of
// G A over the slice of A's rows of `split`, written to part[split][tile].
template <typename TA>
__global__ __launch_bounds__(256) void k_gauss_gemm(const TA* __restrict__ A, int64_t lda,
                                                    GaussPlan P, double* __restrict__ part,
                                                    uint64_t seed, uint64_t iter,
                                                    int32_t problem) {
  __shared__ double Gs[kGTm][kGKc + 1];
  __shared__ double As[kGKc][kGTd + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = blockIdx.x % ((int64_t)P.mt * P.dt);
  const int split = (int)(blockIdx.x / ((int64_t)P.mt * P.dt));
  const int64_t r0 = (tile / P.dt) * kGTm, c0 = (tile % P.dt) * kGTd;
  const int64_t kb = (int64_t)split * P.kchunk;
  const int64_t ke = min(P.n, kb + P.kchunk);
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int t = threadIdx.x;
  for (int64_t i0 = kb; i0 < ke; i0 += kGKc) {
    // G block: 64 rows x 32 columns of G = 16 groups of 4 rows per column,
    // 512 Philox calls, two per thread
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = (t >> 5) + 8 * h;   // group of rows 4q .. 4q+3 of the tile
      const int kk = t & 31;            // column of G within the block
      const int64_t i = i0 + kk;
      double z[4] = {0.0, 0.0, 0.0, 0.0};
      if (i < ke) {
        const U64x4 w = philox4x64_10((uint64_t)i, (uint64_t)(r0 / 4 + q), (uint64_t)problem,
                                      kStreamGauss, seed, iter);
        box_muller(w.w[0], w.w[1], z[0], z[1]);
        box_muller(w.w[2], w.w[3], z[2], z[3]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) Gs[4 * q + j][kk] = z[j];
    }
    // A block: 32 rows x 64 columns, 64 consecutive columns per row
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int rr = (t >> 6) + 4 * u, cc = t & 63;
      const int64_t i = i0 + rr, col = c0 + cc;
      As[rr][cc] = (i < ke && col < P.d) ? (double)A[i * lda + col] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < kGKc; k4 += 4) {
      const double a = Gs[16 * wv + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double bv = As[k4 + (lane >> 4)][16 * b + (lane & 15)];
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // 16 x 16 output blocks: row 4*reg + lane/16, column lane%16
  double* out = part + ((int64_t)split * P.mt * P.dt + tile) * (kGTm * kGTd);
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int reg = 0; reg < 4; ++reg) {
      const int row = 16 * wv + 4 * reg + (lane >> 4);
      out[row * kGTd + 16 * b + (lane & 15)] = acc[b][reg];
    }
}

// SA = scale * sum over the splits, in order, of the partial tiles.
__global__ __launch_bounds__(256) void k_gauss_reduce(const double* __restrict__ part,
                                                      GaussPlan P, double scale, void* SA,
                                                      int32_t sa_dtype, int64_t ld_sa) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= P.m * P.d) return;
  const int64_t r = idx / P.d, c = idx % P.d;
  const int64_t tile = (r / kGTm) * P.dt + c / kGTd;
  const int64_t off = tile * (kGTm * kGTd) + (r % kGTm) * kGTd + (c % kGTd);
  const int64_t stride = (int64_t)P.mt * P.dt * (kGTm * kGTd);
  double s = 0.0;
  for (int q = 0; q < P.splits; ++q) s += part[off + q * stride];
  store_out(SA, sa_dtype, r * ld_sa + c, s * scale);
}

hipError_t launch_gaussian(const DenseSketchArgs& a, hipStream_t st) {
  const GaussPlan P = make_gauss_plan(a.m, a.n, a.d);
  const void* src = a.A;
  int64_t lda = a.lda;
  int32_t dt = a.a_dtype;
  double* part = a.work;
  if (a.csr) {  // densify into the buffer after the partial tiles
    double* dense = a.work + gauss_workspace_bytes(a.m, a.n, a.d) / sizeof(double);
    const int64_t total = a.n * a.d;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, dense,
                       total);
    if (a.n > 0)
      hipLaunchKernelGGL(k_csr_scatter_signed, dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0, st,
                         a.row_ptr, a.col_idx, static_cast<const double*>(a.A), a.n, a.d, dense, 0,
                         a.seed, a.iter, a.problem);
    src = dense;
    lda = a.d;
    dt = 0;
  }
  const dim3 grid((unsigned)((int64_t)P.mt * P.dt * P.splits));
  if (dt == 0)
    hipLaunchKernelGGL(k_gauss_gemm<double>, grid, dim3(256), 0, st,
                       static_cast<const double*>(src), lda, P, part, a.seed, a.iter, a.problem);
  else
    hipLaunchKernelGGL(k_gauss_gemm<float>, grid, dim3(256), 0, st, static_cast<const float*>(src),
                       lda, P, part, a.seed, a.iter, a.problem);
  const int64_t total = a.m * a.d;
  if (total > 0)
    hipLaunchKernelGGL(k_gauss_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       part, P, a.scale, a.SA, a.sa_dtype, a.ld_sa);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Read ceiling: every byte of a buffer read once with 16-byte loads, spread
// evenly over the grid (the pattern of the passes over A), for measurement.
// ---------------------------------------------------------------------------
// Each workgroup reads one contiguous chunk, eight independent 16-byte loads
// per lane in flight (the gather keeps several rows of its buckets in flight
// the same way).
constexpr int kProbeLoads = 8;

__global__ __launch_bounds__(256) void k_read_probe(const double2* __restrict__ p, int64_t n16,
                                                    int64_t per_block, double* sink) {
  double2 acc[kProbeLoads];
#pragma unroll
  for (int u = 0; u < kProbeLoads; ++u) acc[u] = double2{0.0, 0.0};
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = min(n16, b0 + per_block);
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256 * kProbeLoads) {
    double2 v[kProbeLoads];
#pragma unroll
    for (int u = 0; u < kProbeLoads; ++u) {
      const int64_t k = i + 256 * u;
      v[u] = k < b1 ? p[k] : double2{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kProbeLoads; ++u) {
      acc[u].x += v[u].x;
      acc[u].y += v[u].y;
    }
  }
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int u = 0; u < kProbeLoads; ++u) {
    sx += acc[u].x;
    sy += acc[u].y;
  }
  // never true for finite data; keeps the loads from being dropped
  if (sx == 1.0e300 && sy == -1.0e300) sink[0] = sx;
}

hipError_t launch_read_probe(const void* buf, int64_t bytes, double* sink, hipStream_t st) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(8192, (n16 + 4095) / 4096);
  const int64_t per_block = (n16 + blocks - 1) / blocks;
  hipLaunchKernelGGL(k_read_probe, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const double2*>(buf), n16, per_block, sink);
  return hipGetLastError();
}

size_t dense_sketch_workspace_bytes(int32_t kind, int64_t m, int64_t n, int64_t d, bool csr) {
  if (kind == 2) return srht_workspace_bytes(n, d);
  return gauss_workspace_bytes(m, n, d) + (csr ? (size_t)n * d * sizeof(double) : 0);
}

hipError_t launch_dense_sketch(const DenseSketchArgs& a, hipStream_t st) {
  return a.kind == 2 ? launch_srht(a, st) : launch_gaussian(a, st);
}

}  // namespace ihs
