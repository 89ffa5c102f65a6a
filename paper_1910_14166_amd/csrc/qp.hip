// The small d x d quadratic program of Eq.(2) (Sec. 1: T_solve = O(d^3);
// App. A.1.1 on the cost of the QP, polynomial in d) and the fixed-order
// reduction of the gradient partials produced by the row passes.
//
// Unconstrained step: x^{t+1} = x^t + H^{-1} g with H = L L^T.
//  * Right-looking blocked Cholesky, 64-column panels: per panel one launch
//    factors the 64 x 64 diagonal block (padded with the identity when d is
//    not a multiple of 64, so d <= 64 is one such launch), one solves the
//    panel rows below it, and one subtracts P P^T from the trailing lower
//    triangle with FP64 matrix-core tiles.
//  * Triangular solves: one workgroup; each 64-block is solved by one
//    wavefront with cross-lane reads, the rest of the vector is updated by all.
#include <algorithm>

#include "kernels.hpp"
#include "rowdot.hpp"

namespace ihs {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Sum four per-lane partial values across the wavefront (transposing
// butterfly, fixed order): afterwards lane row_lane4(u) holds row u's total.
__device__ __forceinline__ double multi_row_sum4(const double (&v)[4], int lane) {
  const bool h32 = (lane & 32) != 0;
  double a0 = (h32 ? v[2] : v[0]) + __shfl_xor(h32 ? v[0] : v[2], 32, 64);
  double a1 = (h32 ? v[3] : v[1]) + __shfl_xor(h32 ? v[1] : v[3], 32, 64);
  const bool h16 = (lane & 16) != 0;
  double s = (h16 ? a1 : a0) + __shfl_xor(h16 ? a0 : a1, 16, 64);
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}
__device__ __forceinline__ int row_lane4(int u) { return ((u >> 1) & 1) * 32 + (u & 1) * 16; }  // d*d doubles within 64 KiB of LDS
constexpr int kNb = 64;

// Per-problem state of the l2-ball shift iteration: trs[4p] is the shift mu
// added to the diagonal, trs[4p+1] >= 2 marks a problem that needs no factor.
__device__ __forceinline__ bool trs_skip(const double* trs, int p) {
  return trs != nullptr && trs[4 * p + 1] >= 2.0;
}

// Stages the lower triangle (with the diagonal) of the nb x nb block at
// (r0, r0) of the d x d row-major matrix M into D, zeros elsewhere. Every
// thread issues its 16 loads before the first LDS store, so the staging
// costs one memory round trip. 256 threads.
__device__ __forceinline__ void stage_lower64(double (*D)[kNb + 1], const double* __restrict__ M,
                                              int64_t d, int64_t r0, int nb) {
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q, i = e >> 6, j = e & 63;
    v[q] = (i < nb && j <= i) ? M[(r0 + i) * d + r0 + j] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    D[e >> 6][e & 63] = v[q];
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Gradient partial reduction, g[p][:] = sum_w gpart[p][w][:], in a fixed
// two-level order: kRedSplit x 4 contiguous groups of parts are summed in
// ascending order (first kernel), then the group sums in ascending order
// (second kernel). The objective f[p] follows the same pattern.
// ---------------------------------------------------------------------------
constexpr int kRedSplit = 16;
constexpr int kRedBatch = 16;

__global__ __launch_bounds__(256) void k_reduce_a(const double* __restrict__ gpart,
                                                  const double* __restrict__ fpart,
                                                  int64_t parts_fixed, const ProbInfo* probs,
                                                  int64_t d, double* red, double* fred) {
  const int p = blockIdx.z;
  const int split = blockIdx.y;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t nparts = parts_fixed > 0 ? parts_fixed : (int64_t)probs[p].nseg;
  const int64_t pbase = parts_fixed > 0 ? (int64_t)p * parts_fixed : (int64_t)probs[p].seg0;
  const int grp = split * 4 + q;  // 0 .. 4*kRedSplit-1
  const int64_t per = (nparts + 4 * kRedSplit - 1) / (4 * kRedSplit);
  const int64_t w0 = min((int64_t)grp * per, nparts), w1 = min(w0 + per, nparts);
  {
    const int64_t col = (int64_t)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (col < d) {
      for (int64_t w = w0; w < w1; w += kRedBatch) {
        double v[kRedBatch];
#pragma unroll
        for (int u = 0; u < kRedBatch; ++u)
          v[u] = w + u < w1 ? gpart[(pbase + w + u) * d + col] : 0.0;
#pragma unroll
        for (int u = 0; u < kRedBatch; ++u)
          if (w + u < w1) s += v[u];
      }
      red[((int64_t)p * 4 * kRedSplit + grp) * d + col] = s;
    }
  }
  if (blockIdx.x == 0 && lane == 0) {
    // loads requested kRedBatch at a time, summed in ascending order
    double fs = 0.0;
    for (int64_t w = w0; w < w1; w += kRedBatch) {
      double v[kRedBatch];
#pragma unroll
      for (int u = 0; u < kRedBatch; ++u) v[u] = w + u < w1 ? fpart[pbase + w + u] : 0.0;
#pragma unroll
      for (int u = 0; u < kRedBatch; ++u)
        if (w + u < w1) fs += v[u];
    }
    fred[(int64_t)p * 4 * kRedSplit + grp] = fs;
  }
}

__global__ __launch_bounds__(64) void k_reduce_b(const double* __restrict__ red,
                                                 const double* __restrict__ fred, int64_t d,
                                                 double* g, double* f, DeviceStatus* st,
                                                 int32_t iter) {
  const int p = blockIdx.y;
  const int64_t col = (int64_t)blockIdx.x * 64 + threadIdx.x;
  // after the tolerance stop the pass did not run: keep g, f and the objective
  if (st != nullptr && status_word(&st->done) != 0) return;
  // every group sum is requested before the first addition (one round trip
  // instead of one per group); the additions keep the ascending order
  if (col < d) {
    double v[4 * kRedSplit];
#pragma unroll
    for (int q = 0; q < 4 * kRedSplit; ++q) v[q] = red[((int64_t)p * 4 * kRedSplit + q) * d + col];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4 * kRedSplit; ++q) s += v[q];
    g[(int64_t)p * d + col] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double v[4 * kRedSplit];
#pragma unroll
    for (int q = 0; q < 4 * kRedSplit; ++q) v[q] = fred[(int64_t)p * 4 * kRedSplit + q];
    double fs = 0.0;
#pragma unroll
    for (int q = 0; q < 4 * kRedSplit; ++q) fs += v[q];
    const double fv = 0.5 * fs;
    if (f != nullptr) f[p] = fv;
    if (st != nullptr) {
      if (p == 0) st->objective = fv;
      if (!isfinite(fv)) status_fail(st, 7 /* IHS_ERR_NONFINITE */, iter, p);
    }
  }
}

size_t reduce_scratch_doubles(int32_t batch, int64_t d) {
  return (size_t)batch * 4 * kRedSplit * (d + 1);
}

hipError_t launch_reduce_partials(const double* gpart, const double* fpart, int32_t batch,
                                  int64_t parts_fixed, const ProbInfo* probs, int64_t d,
                                  double* g, double* f, DeviceStatus* status, int32_t iter,
                                  double* scratch, hipStream_t st) {
  double* red = scratch;
  double* fred = scratch + (int64_t)batch * 4 * kRedSplit * d;
  hipLaunchKernelGGL(k_reduce_a, dim3((unsigned)((d + 63) / 64), kRedSplit, batch), dim3(256), 0,
                     st, gpart, fpart,
                     parts_fixed, probs, d, red, fred);
  hipLaunchKernelGGL(k_reduce_b, dim3((unsigned)((d + 63) / 64), batch), dim3(64), 0, st, red,
                     fred, d, g, f, status, iter);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Blocked Cholesky, in place on L (lower triangle).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol_init(const double* __restrict__ H, double* L,
                                                   int64_t d, int32_t batch, double shift,
                                                   const double* __restrict__ trs) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)batch * d * d) return;
  const int p = (int)(idx / (d * d));
  if (trs_skip(trs, p)) return;
  if (trs) shift = trs[4 * p];
  const int64_t e = idx % (d * d);
  const int64_t i = e / d, j = e - (e / d) * d;
  L[idx] = (j <= i) ? H[idx] + (i == j ? shift : 0.0) : 0.0;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = readlane_u32((uint32_t)u, lane);
  const uint64_t hi = readlane_u32((uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)((hi << 32) | lo));
}

// 1/sqrt(x) and sqrt(x) for positive finite x: the hardware estimate of
// 1/sqrt (about 2^-23 relative error) refined by two steps of Goldschmidt's
// coupled iteration (g -> sqrt(x), h -> 1/(2 sqrt(x))), then one residual
// correction of the root. Measured over 2^20 values spread over 2^-600 ..
// 2^600 and the extremes of the range: within 1.6 ulp for 1/sqrt and 0.6 ulp
// for sqrt. The chain is about 60% of that of a rounded sqrt and a division,
// and the pivots of the diagonal block are one long chain of these.
__device__ __forceinline__ void rsqrt_sqrt(double x, double& r, double& s) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  s = fma(fma(-g, g, x), h, g);
  r = 2.0 * h;
}

// Diagonal block of panel kb: one workgroup of 512 threads per problem
// factors the 64 x 64 block right-looking in steps of four columns. Thread t
// keeps row t/8, columns 8*(t%8) .. +7, in registers. At each step:
//  1. the threads holding the four columns publish them to LDS;
//  2. every thread factors the 4 x 4 pivot block itself and forms its row's
//     panel entries L_iJ = A_iJ L_JJ^{-T}; the holder of the four columns
//     keeps them and publishes them;
//  3. every thread applies the rank-4 update to its entries with the
//     published panel entries of their columns.
// The steps run as eight groups of two with the inner two unrolled, so every
// register index is a constant. L_jj and 1/L_jj come from rsqrt_sqrt. Writes
// L_kk and 1/L_jj back. The block is loaded before the status is read (one
// memory round trip), and two waves per SIMD of at most 96 registers fit
// beside the bucket gather.
constexpr int kDiagThreads = 512;

// The factor of problem p's diagonal block at kb, by one kDiagThreads workgroup.
// UPDATE: the block first takes its share of the trailing update of the
// panel before it, B -= P P^T with P = W[kb:kb+64, kb-64:kb]: P is staged in
// LDS with the block's own loads (one memory round trip), each wavefront forms
// one or two of the block's ten lower 16 x 16 tiles on MFMA from LDS, in the
// operand and accumulation order of chol_update_tile (so the factor is
// bitwise that of a separate update), and the tiles return through LDS to the
// threads that hold the block's rows.
template <bool UPDATE>
__device__ __forceinline__ void chol_diag_block(double* L, int64_t d, int64_t kb, double* rdiag,
                                                DeviceStatus* st, int32_t iter,
                                                const double* __restrict__ trs, int p) {
  __shared__ double Pb[kNb][4];  // the step's four columns of every row
  __shared__ double Zb[kNb][4];  // the step's panel entries of every row
  __shared__ double rd[kNb];
  __shared__ int flag;
  const int tid = threadIdx.x;
  double* W = L + (int64_t)p * d * d;
  const int nb = (int)min((int64_t)kNb, d - kb);
  const int i = tid >> 3, seg = tid & 7, k0 = 8 * seg;
  double a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q)
    a[q] = (i < nb && k0 + q <= i) ? W[(kb + i) * d + kb + k0 + q] : 0.0;
  if constexpr (UPDATE) {
    __shared__ double Ps[kNb][kNb + 1];  // P, then the update's tiles
    constexpr int kPer = kNb * kNb / kDiagThreads;
    double pv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = u * kDiagThreads + tid, r = e / kNb, c = e % kNb;
      pv[u] = r < nb ? W[(kb + r) * d + kb - kNb + c] : 0.0;
    }
    if (tid == 0) flag = (st->code != 0 || trs_skip(trs, p)) ? 1 : 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = u * kDiagThreads + tid;
      Ps[e / kNb][e % kNb] = pv[u];
    }
    __syncthreads();
    if (flag != 0) return;
    const int wv = tid >> 6, lane = tid & 63;
    const int r = lane & 15, kk = lane >> 4, rq = lane >> 4, col = lane & 15;
    constexpr int kTiles = (kNb / 16) * (kNb / 16 + 1) / 2;
    constexpr int kWaves = kDiagThreads / 64;
    f64x4 acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = wv + h * kWaves;
      if (t < kTiles) {
        const int ti = t >= 6 ? 3 : (t >= 3 ? 2 : (t >= 1 ? 1 : 0));
        const int tj = t - ti * (ti + 1) / 2;
#pragma unroll
        for (int k = 0; k < kNb / 4; ++k)
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ps[ti * 16 + r][4 * k + kk],
                                                        Ps[tj * 16 + r][4 * k + kk], acc[h], 0, 0,
                                                        0);
      }
    }
    __syncthreads();  // every read of P is done
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = wv + h * kWaves;
      if (t < kTiles) {
        const int ti = t >= 6 ? 3 : (t >= 3 ? 2 : (t >= 1 ? 1 : 0));
        const int tj = t - ti * (ti + 1) / 2;
#pragma unroll
        for (int reg = 0; reg < 4; ++reg) Ps[ti * 16 + 4 * reg + rq][tj * 16 + col] = acc[h][reg];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (i < nb && k0 + q <= i) a[q] = a[q] - Ps[i][k0 + q];
  } else {
    if (tid == 0) flag = (st->code != 0 || trs_skip(trs, p)) ? 1 : 0;
    __syncthreads();
    if (flag != 0) return;
  }
  int bad = 0;
  for (int S = 0; S < 8 && !bad; ++S) {
#pragma unroll
    for (int JJ = 0; JJ < 2; ++JJ) {
      const int j0 = 8 * S + 4 * JJ, jend = j0 + 4;
      if (j0 >= nb) break;  // uniform
      if (seg == S) {
#pragma unroll
        for (int c = 0; c < 4; ++c) Pb[i][c] = a[4 * JJ + c];
      }
      __syncthreads();
      // the 4 x 4 pivot block, padded with the identity past nb
      double pv[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          pv[r][c] = (j0 + r < nb) ? Pb[j0 + r][c] : (r == c ? 1.0 : 0.0);
      const double d0 = pv[0][0];
      if (!(d0 > 0.0) || !isfinite(d0)) {  // the same pivots in every thread
        bad = 1;
        break;
      }
      double l00, r0;
      rsqrt_sqrt(d0, r0, l00);
      const double l10 = pv[1][0] * r0, l20 = pv[2][0] * r0, l30 = pv[3][0] * r0;
      const double d1 = fma(-l10, l10, pv[1][1]);
      if (!(d1 > 0.0) || !isfinite(d1)) {
        bad = 1;
        break;
      }
      double l11, r1;
      rsqrt_sqrt(d1, r1, l11);
      const double l21 = fma(-l20, l10, pv[2][1]) * r1, l31 = fma(-l30, l10, pv[3][1]) * r1;
      const double d2 = fma(-l21, l21, fma(-l20, l20, pv[2][2]));
      if (!(d2 > 0.0) || !isfinite(d2)) {
        bad = 1;
        break;
      }
      double l22, r2;
      rsqrt_sqrt(d2, r2, l22);
      const double l32 = fma(-l31, l21, fma(-l30, l20, pv[3][2])) * r2;
      const double d3 = fma(-l32, l32, fma(-l31, l31, fma(-l30, l30, pv[3][3])));
      if (!(d3 > 0.0) || !isfinite(d3)) {
        bad = 1;
        break;
      }
      double l33, r3;
      rsqrt_sqrt(d3, r3, l33);
      double zi[4] = {0.0, 0.0, 0.0, 0.0};
      if (i >= jend && i < nb) {
        // z = L_JJ^{-1} u: the panel entries of row i from its four A entries
        const double* u = Pb[i];
        zi[0] = u[0] * r0;
        zi[1] = fma(-l10, zi[0], u[1]) * r1;
        zi[2] = fma(-l21, zi[1], fma(-l20, zi[0], u[2])) * r2;
        zi[3] = fma(-l32, zi[2], fma(-l31, zi[1], fma(-l30, zi[0], u[3]))) * r3;
        if (seg == S) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            a[4 * JJ + c] = zi[c];
            Zb[i][c] = zi[c];
          }
        }
      } else if (i >= j0 && i < jend && i < nb && seg == S) {
        // row i - j0 of the 4 x 4 factor
        const int rr = i - j0;
        a[4 * JJ + 0] = rr == 0 ? l00 : (rr == 1 ? l10 : (rr == 2 ? l20 : l30));
        a[4 * JJ + 1] = rr == 0 ? 0.0 : (rr == 1 ? l11 : (rr == 2 ? l21 : l31));
        a[4 * JJ + 2] = rr <= 1 ? 0.0 : (rr == 2 ? l22 : l32);
        a[4 * JJ + 3] = rr <= 2 ? 0.0 : l33;
      }
      if (tid == 0) {
        rd[j0] = r0;
        rd[j0 + 1] = r1;
        rd[j0 + 2] = r2;
        rd[j0 + 3] = r3;
      }
      __syncthreads();
      if (i >= jend && i < nb && seg >= S) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = k0 + q;
          if (k >= jend && k <= i) {
            const double* zk = Zb[k];
            a[q] = fma(-zi[3], zk[3], fma(-zi[2], zk[2], fma(-zi[1], zk[1], fma(-zi[0], zk[0], a[q]))));
          }
        }
      }
    }
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) status_fail(st, 5 /* IHS_ERR_NOT_PD */, iter, p);
    return;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (i < nb && k0 + q <= i) W[(kb + i) * d + kb + k0 + q] = a[q];
  if (tid < nb) rdiag[(int64_t)p * d + kb + tid] = rd[tid];
}

__global__ __launch_bounds__(kDiagThreads) void k_chol_diag(double* L, int64_t d, int64_t kb,
                                                            double* rdiag, DeviceStatus* st,
                                                            int32_t iter,
                                                            const double* __restrict__ trs) {
  chol_diag_block<false>(L, d, kb, rdiag, st, iter, trs, blockIdx.x);
}

// Panel rows below the diagonal block: x L_kk^T = a for each row, one row per
// wavefront pass with lanes over the 64 columns; the factored block is staged
// in LDS and x_c is read from lane c (column-oriented substitution).
// Four rows are interleaved per wavefront for independent dependency chains.
// The rows, the block and the pivots are requested together with the status,
// so the kernel waits for memory once.
__global__ __launch_bounds__(256) void k_chol_trsm(double* L, int64_t d, int64_t kb,
                                                   const double* __restrict__ rdiag,
                                                   DeviceStatus* st, const double* __restrict__ trs) {
  __shared__ double D[kNb][kNb + 1];
  __shared__ double rd[kNb];
  __shared__ int flag;
  const int p = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* W = L + (int64_t)p * d * d;
  const int64_t rows0 = kb + kNb;
  const int64_t r_first = rows0 + ((int64_t)blockIdx.x * 4 + wv) * 4;
  double a[4];
  bool ok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    ok[u] = r_first + u < d;
    a[u] = ok[u] ? W[(r_first + u) * d + kb + lane] : 0.0;
  }
  const double rdv = tid < kNb ? rdiag[(int64_t)p * d + kb + tid] : 0.0;
  if (tid == 0) flag = (st->code != 0 || trs_skip(trs, p)) ? 1 : 0;
  stage_lower64(D, W, d, kb, kNb);  // below > 0, so the block is full
  if (tid < kNb) rd[tid] = rdv;
  __syncthreads();
  if (flag != 0) return;
  for (int c = 0; c < kNb; ++c) {
    const double lkc = D[lane][c];
    const double rc = rd[c];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double xc = readlane_f64(a[u], c) * rc;
      a[u] = lane == c ? xc : (lane > c ? fma(-xc, lkc, a[u]) : a[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (ok[u]) W[(r_first + u) * d + kb + lane] = a[u];
}

// Trailing update W[i][j] -= sum_k P[i][k] P[j][k], kb+64 <= j <= i < d, with
// P = W[:, kb:kb+64]. One wavefront per 16 x 16 lower tile (small register
// footprint, so these tiles also run beside a memory-bound pass). All operand
// loads, the tile's own entries and the status are requested up front: one
// memory round trip before the MFMA chain. Tile t of the lower triangle of
// T x T tiles is (ti, tj), t = ti (ti + 1) / 2 + tj.
__device__ __forceinline__ void chol_update_tile(double* W, int64_t d, int64_t kb, int64_t t,
                                                 int lane, const DeviceStatus* st,
                                                 const double* __restrict__ trs, int p) {
  const int64_t t0 = kb + kNb;
  int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > t) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  const int64_t r0 = t0 + ti * 16, c0 = t0 + tj * 16;
  const int r = lane & 15, kk = lane >> 4;
  const bool ra = r0 + r < d, rb = c0 + r < d;
  const double* pa = W + (r0 + r) * d + kb + kk;
  const double* pb = W + (c0 + r) * d + kb + kk;
  const int col = lane & 15, rq = lane >> 4;
  double cur[4];
#pragma unroll
  for (int reg = 0; reg < 4; ++reg) {
    const int64_t ii = r0 + 4 * reg + rq, jj = c0 + col;
    cur[reg] = (ii < d && jj < d && jj <= ii) ? W[ii * d + jj] : 0.0;
  }
  // the panel's 64 columns in four chunks of 16, each chunk's operands
  // requested before the previous chunk's products (few registers, so a
  // workgroup of the diagonal factor's size fits beside a memory-bound pass)
  constexpr int KC = kNb / 16;  // MFMA steps per chunk
  double av[KC], bv[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    av[k] = ra ? pa[4 * k] : 0.0;
    bv[k] = rb ? pb[4 * k] : 0.0;
  }
  if (st->code != 0 || trs_skip(trs, p)) return;
  f64x4 acc = {0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double an[KC], bn[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      an[k] = (c + 1 < 4 && ra) ? pa[4 * (KC * (c + 1) + k)] : 0.0;
      bn[k] = (c + 1 < 4 && rb) ? pb[4 * (KC * (c + 1) + k)] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[k], bv[k], acc, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      av[k] = an[k];
      bv[k] = bn[k];
    }
  }
#pragma unroll
  for (int reg = 0; reg < 4; ++reg) {
    const int64_t ii = r0 + 4 * reg + rq, jj = c0 + col;
    if (ii < d && jj < d && jj <= ii) W[ii * d + jj] = cur[reg] - acc[reg];
  }
}

// The trailing update after panel kb fused with the factor of the next
// diagonal block (kb + 64): workgroup p < batch updates that block (the first
// tiles of the triangle) and factors it, while the other workgroups update the
// rest of the trailing matrix, which that block does not read. One launch per
// block step instead of two, and the block's factor runs beside the update
// instead of after it. At most 96 registers, so that two of these 512-thread
// workgroups' waves per SIMD fit beside the bucket gather.
__global__ __launch_bounds__(kDiagThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_chol_update_diag(
    double* L, int64_t d, int64_t kb, int32_t batch, double* rdiag, DeviceStatus* st,
    int32_t iter, const double* __restrict__ trs) {
  constexpr int kWaves = kDiagThreads / 64;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t0 = kb + kNb;
  const int64_t T = (d - t0 + 15) / 16;
  const int64_t Tn = min(T, (int64_t)(kNb / 16));
  const int64_t ndiag = Tn * (Tn + 1) / 2;  // tiles of the next diagonal block
  const int64_t ntri = T * (T + 1) / 2;
  if ((int)blockIdx.x < batch) {
    chol_diag_block<true>(L, d, t0, rdiag, st, iter, trs, blockIdx.x);
    return;
  }
  const int64_t per = ntri - ndiag;
  const int64_t w = (int64_t)(blockIdx.x - batch) * kWaves + wv;
  if (w >= per * batch) return;
  const int p = (int)(w / per);
  chol_update_tile(L + (int64_t)p * d * d, d, kb, ndiag + (w - (int64_t)p * per), lane, st, trs,
                   p);
}

hipError_t launch_cholesky(const double* H, double* L, int64_t d, int32_t batch,
                           DeviceStatus* status, int32_t iter, double shift, double* scratch,
                           hipStream_t st, const double* trs) {
  double* rdiag = chol_rdiag(scratch, batch);
  const int64_t tot = (int64_t)batch * d * d;
  hipLaunchKernelGGL(k_chol_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, H, L, d,
                     batch, shift, trs);
  hipLaunchKernelGGL(k_chol_diag, dim3(batch), dim3(kDiagThreads), 0, st, L, d, (int64_t)0, rdiag,
                     status, iter, trs);
  for (int64_t kb = 0; kb + kNb < d; kb += kNb) {
    const int64_t below = d - kb - kNb;
    const unsigned gx = (unsigned)((below + 15) / 16);  // 16 rows per workgroup
    hipLaunchKernelGGL(k_chol_trsm, dim3(gx, batch), dim3(256), 0, st, L, d, kb, rdiag, status,
                       trs);
    // the update after panel kb and the factor of the diagonal block at kb + 64
    const int64_t T = (below + 15) / 16;
    const int64_t Tn = std::min<int64_t>(T, kNb / 16);
    const int64_t rest = (T * (T + 1) / 2 - Tn * (Tn + 1) / 2) * batch;
    constexpr int64_t kWaves = kDiagThreads / 64;
    hipLaunchKernelGGL(k_chol_update_diag, dim3((unsigned)(batch + (rest + kWaves - 1) / kWaves)),
                       dim3(kDiagThreads), 0, st, L, d, kb, batch, rdiag, status, iter, trs);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// out = base + (L L^T)^{-1} v, one workgroup (256 threads) per problem.
// Per 64-row block: the diagonal block is staged in LDS and solved by
// wavefront 0 (lane c holds y_c; x_c is read from lane c, reciprocal
// pivots from the factorisation); the remaining rows are updated by all four
// wavefronts, four rows at a time with one transposing butterfly. The loads
// of several passes are issued together (kSolveGroups passes forward,
// kSolveCols columns backward), so fewer of one workgroup's reads of L wait
// one after the other.
// Also records sqrt(dx^T v) for problem 0.
// ---------------------------------------------------------------------------
constexpr int kSolveGroups = 4, kSolveCols = 32;

__global__ __launch_bounds__(256) void k_chol_solve(const double* __restrict__ L, int64_t d,
                                                    const double* __restrict__ rdiag,
                                                    const double* __restrict__ v,
                                                    const double* base, double* out,
                                                    DeviceStatus* st, const DeviceStatus* gate,
                                                    int32_t gate_iter) {
  extern __shared__ double y[];
  __shared__ double D[64][65];
  __shared__ double red[256];
  __shared__ int code;
  const int p = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* Lp = L + (int64_t)p * d * d;
  const double* rp = rdiag + (int64_t)p * d;
  const double* vp = v + (int64_t)p * d;
  const double* bp = base + (int64_t)p * d;
  double* op = out + (int64_t)p * d;
  if (tid == 0) {
    code = status_halted(st) ? 1 : 0;
    if (gate != nullptr && status_failed_by(gate, gate_iter)) code = 1;
  }
  __syncthreads();
  if (code != 0) {
    if (op != bp)
      for (int64_t i = tid; i < d; i += 256) op[i] = bp[i];
    return;
  }
  for (int64_t i = tid; i < d; i += 256) y[i] = vp[i];
  const int64_t nblk = (d + 63) / 64;
  // forward: L y = v
  for (int64_t bi = 0; bi < nblk; ++bi) {
    const int64_t jb = bi * 64;
    const int nb = (int)min((int64_t)64, d - jb);
    stage_lower64(D, Lp, d, jb, nb);
    __syncthreads();
    if (wv == 0) {
      double yl = lane < nb ? y[jb + lane] : 0.0;
      const double rl = lane < nb ? rp[jb + lane] : 0.0;
      for (int c = 0; c < nb; ++c) {
        const double lkc = D[lane][c];
        const double xc = readlane_f64(yl, c) * readlane_f64(rl, c);
        yl = lane == c ? xc : (lane > c ? fma(-xc, lkc, yl) : yl);
      }
      if (lane < nb) y[jb + lane] = yl;
    }
    __syncthreads();
    const double yb = lane < nb ? y[jb + lane] : 0.0;
    for (int64_t i0 = jb + nb + (int64_t)wv * 4; i0 < d; i0 += 16 * kSolveGroups) {
      // the rows of kSolveGroups passes are requested before any is reduced
      double t[kSolveGroups][4];
#pragma unroll
      for (int g = 0; g < kSolveGroups; ++g)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t r = i0 + 16 * g + u;
          t[g][u] = (r < d && lane < nb) ? Lp[r * d + jb + lane] * yb : 0.0;
        }
#pragma unroll
      for (int g = 0; g < kSolveGroups; ++g) {
        const double s = multi_row_sum4(t[g], lane);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t r = i0 + 16 * g + u;
          if (lane == row_lane4(u) && r < d) y[r] -= s;
        }
      }
    }
    __syncthreads();
  }
  // backward: L^T z = y
  for (int64_t bi = nblk - 1; bi >= 0; --bi) {
    const int64_t jb = bi * 64;
    const int nb = (int)min((int64_t)64, d - jb);
    stage_lower64(D, Lp, d, jb, nb);
    __syncthreads();
    if (wv == 0) {
      double yl = lane < nb ? y[jb + lane] : 0.0;
      const double rl = lane < nb ? rp[jb + lane] : 0.0;
      for (int c = nb - 1; c >= 0; --c) {
        const double lck = D[c][lane];
        const double xc = readlane_f64(yl, c) * readlane_f64(rl, c);
        yl = lane == c ? xc : (lane < c ? fma(-xc, lck, yl) : yl);
      }
      if (lane < nb) y[jb + lane] = yl;
    }
    __syncthreads();
    for (int64_t i = tid; i < jb; i += 256) {
      double s = 0.0;
      for (int c0 = 0; c0 < nb; c0 += kSolveCols) {
        double lv[kSolveCols];  // requested together, summed in column order
#pragma unroll
        for (int q = 0; q < kSolveCols; ++q)
          lv[q] = c0 + q < nb ? Lp[(jb + c0 + q) * d + i] : 0.0;
#pragma unroll
        for (int q = 0; q < kSolveCols; ++q)
          if (c0 + q < nb) s = fma(lv[q], y[jb + c0 + q], s);
      }
      y[i] -= s;
    }
    __syncthreads();
  }
  double part = 0.0;
  bool finite = true;
  for (int64_t i = tid; i < d; i += 256) {
    const double xi = bp[i] + y[i];
    part = fma(y[i], vp[i], part);
    finite = finite && isfinite(xi);
  }
  red[tid] = part;
  const int all_finite = __syncthreads_and(finite ? 1 : 0);
  for (int stride = 128; stride > 0; stride >>= 1) {
    if (tid < stride) red[tid] += red[tid + stride];
    __syncthreads();
  }
  if (!all_finite) {
    if (tid == 0) status_fail(st, 7 /* IHS_ERR_NONFINITE */, -1, p);
    if (op != bp)
      for (int64_t i = tid; i < d; i += 256) op[i] = bp[i];
    return;
  }
  for (int64_t i = tid; i < d; i += 256) op[i] = bp[i] + y[i];
  if (p == 0 && tid == 0) st->last_step = sqrt(fmax(red[0], 0.0));
}

hipError_t launch_chol_solve_update(const double* L, const double* rdiag, int64_t d,
                                    int32_t batch, const double* v, const double* base,
                                    double* out, DeviceStatus* status, hipStream_t st,
                                    const DeviceStatus* gate, int32_t gate_iter) {
  hipLaunchKernelGGL(k_chol_solve, dim3(batch), dim3(256), (size_t)(d * sizeof(double)),
                     st, L, d, rdiag, v, base, out, status, gate, gate_iter);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Explicit inverse H^{-1} = L^{-T} L^{-1} from the Cholesky factor, in three
// stages over 64 x 64 blocks, the last two on f64 MFMA:
//   1. diagonal blocks Linv_ii = L_ii^{-1}, one workgroup per block;
//   2. recursive doubling: adjacent inverted segments A (h blocks) and C
//      (up to h blocks) of L = [[A, 0], [B, C]] merge into one by
//      [[A, 0], [B, C]]^{-1} = [[A^{-1}, 0], [-C^{-1} B A^{-1}, C^{-1}]],
//      T = B A^{-1} first and then -C^{-1} T, every 64 x 64 output tile in
//      parallel; h = 1, 2, 4, ... so there are log2(blocks) merge stages;
//   3. H^{-1}_{IJ} = sum_{k >= I} Linv_{kI}^T Linv_{kJ} for I >= J, mirrored.
// T is kept in the H^{-1} buffer at the position of its block, which the
// last stage overwrites. Entries at or beyond d read as zero, so a ragged last
// block needs no padding. Problems with trs[4p+1] >= 2 (nullable) are skipped.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool inv_skip(const DeviceStatus* st, const double* trs, int p) {
  return status_halted(st) || trs_skip(trs, p);
}

// L_ii^{-1} by rows, right-looking: thread t keeps row t/4, columns
// 16*(t%4) .. +15, of X (initially I) in registers. At step k row k is
// final once divided by L_kk; its owners publish it to LDS (two alternating
// buffers, one barrier per step) and every row below subtracts L_ik times
// it. 256 threads per diagonal block. The block, the thread's pivot
// reciprocal and the status are requested together (one memory round trip).
__global__ __launch_bounds__(256) void k_trtri_diag(const double* __restrict__ L,
                                                    const double* __restrict__ rdiag, int64_t d,
                                                    double* Linv, const DeviceStatus* st,
                                                    const double* __restrict__ trs) {
  __shared__ double Ls[kNb][kNb + 1];
  __shared__ double R[2][kNb];
  __shared__ int skip;
  const int p = blockIdx.y, tid = threadIdx.x;
  const int64_t jb = (int64_t)blockIdx.x * kNb;
  const int nb = (int)min((int64_t)kNb, d - jb);
  const double* Lp = L + (int64_t)p * d * d;
  const int i = tid >> 2, seg = tid & 3, c0 = 16 * seg;
  const double ri = i < nb ? rdiag[(int64_t)p * d + jb + i] : 0.0;
  if (tid == 0) skip = inv_skip(st, trs, p) ? 1 : 0;
  stage_lower64(Ls, Lp, d, jb, nb);
  double x[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = (c0 + q == i) ? 1.0 : 0.0;
  __syncthreads();
  if (skip) return;
  for (int k = 0; k < nb; ++k) {
    double* Rk = R[k & 1];
    if (i == k) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        x[q] *= ri;
        Rk[c0 + q] = x[q];
      }
    }
    __syncthreads();
    if (i > k && i < nb) {
      const double lik = Ls[i][k];
#pragma unroll
      for (int q = 0; q < 16; ++q) x[q] = fma(-lik, Rk[c0 + q], x[q]);
    }
  }
  double* Op = Linv + (int64_t)p * d * d;
  if (i < nb) {
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (c0 + q < nb) Op[(jb + i) * d + jb + c0 + q] = x[q];
  }
}

// Block tiles of the inverse stages: 64 x 64 doubles in LDS, one padding
// column against bank conflicts.
typedef double Tile64[kNb][kNb + 1];

// A pair of 64 x 64 blocks in flight: every thread holds 16 + 16 entries.
// load64x2 requests the blocks at (ra, ca) of the d x d matrix MA and at
// (rb, cb) of MB (entries at or beyond d read as zero, coalesced rows);
// store64x2 writes them to LDS. Splitting the two lets a kernel fetch the
// next pair while the MFMAs run on the current one. 256 threads.
struct Pair64 {
  double a[16], b[16];
};

__device__ __forceinline__ void load64x2(Pair64& v, const double* __restrict__ MA, int64_t ra,
                                         int64_t ca, const double* __restrict__ MB, int64_t rb,
                                         int64_t cb, int64_t d) {
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q, rr = e >> 6, cc = e & 63;
    v.a[q] = (ra + rr < d && ca + cc < d) ? MA[(ra + rr) * d + ca + cc] : 0.0;
    v.b[q] = (rb + rr < d && cb + cc < d) ? MB[(rb + rr) * d + cb + cc] : 0.0;
  }
}

__device__ __forceinline__ void store64x2(const Pair64& v, Tile64& TA, Tile64& TB) {
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    TA[e >> 6][e & 63] = v.a[q];
    TB[e >> 6][e & 63] = v.b[q];
  }
}

// acc += op(A) B for 64 x 64 tiles in LDS, op(A) = A or A^T, on a 256-thread
// workgroup: wave w owns the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 tiles
// of 16 x 16 (f64 MFMA 16x16x4).
template <bool TRANS_A>
__device__ __forceinline__ void tile_mma64(f64x4 (&acc)[2][2], const Tile64& A,
                                           const Tile64& B) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, kk = lane >> 4;
  const int r0 = 32 * (wv >> 1), c0 = 32 * (wv & 1);
#pragma unroll 4
  for (int k0 = 0; k0 < kNb; k0 += 4) {
    double av[2], bv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      av[t] = TRANS_A ? A[k0 + kk][r0 + 16 * t + r] : A[r0 + 16 * t + r][k0 + kk];
      bv[t] = B[k0 + kk][c0 + 16 * t + r];
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
  }
}

// Calls f(row, col, value) for every element a wave holds in acc.
template <typename F>
__device__ __forceinline__ void tile_store64(const f64x4 (&acc)[2][2], F f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r0 = 32 * (wv >> 1), c0 = 32 * (wv & 1);
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int reg = 0; reg < 4; ++reg)
        f(r0 + 16 * ti + 4 * reg + (lane >> 4), c0 + 16 * tj + (lane & 15), acc[ti][tj][reg]);
}

// One merge stage (segment size h blocks) of the triangular inverse. Block
// (x, y) of the grid is output tile (i, j) = (x / h, x % h) of pair y, whose
// segments start at a0 = 2 h y (A) and c0 = a0 + h (C, hc <= h blocks).
// PHASE 0: T_ij = sum_{k=j}^{h-1} L_{c0+i, a0+k} Linv_{a0+k, a0+j} -> Tb;
// PHASE 1: Linv_{c0+i, a0+j} = -sum_{k=0}^{i} Linv_{c0+i, c0+k} T_kj.
// Each operand pair is requested while the previous products are summed only
// through the LDS staging; the register footprint stays small enough for a
// workgroup to fit on a CU beside the bucket gather's waves.
template <int PHASE>
__global__ __launch_bounds__(256, 3) void k_trtri_merge(const double* __restrict__ L, double* Linv,
                                                        double* Tb, int64_t d, int32_t nblk,
                                                        int32_t h, const DeviceStatus* st,
                                                        const double* __restrict__ trs) {
  __shared__ Tile64 As, Bs;
  __shared__ int skip;
  const int p = blockIdx.z;
  const int i = (int)blockIdx.x / h, j = (int)blockIdx.x % h;
  const int a0 = 2 * h * (int)blockIdx.y, c0 = a0 + h;
  const int hc = min(h, nblk - c0);
  if (i >= hc) return;  // uniform per workgroup
  const int64_t off = (int64_t)p * d * d;
  const double* Lp = L + off;
  double* Xp = Linv + off;
  double* Tp = Tb + off;
  const int kbeg = PHASE == 0 ? j : 0, kend = PHASE == 0 ? h : i + 1;
  f64x4 acc[2][2] = {};
  for (int k = kbeg; k < kend; ++k) {
    Pair64 nx;
    if (PHASE == 0)
      load64x2(nx, Lp, (int64_t)(c0 + i) * kNb, (int64_t)(a0 + k) * kNb, Xp,
               (int64_t)(a0 + k) * kNb, (int64_t)(a0 + j) * kNb, d);
    else
      load64x2(nx, Xp, (int64_t)(c0 + i) * kNb, (int64_t)(c0 + k) * kNb, Tp,
               (int64_t)(c0 + k) * kNb, (int64_t)(a0 + j) * kNb, d);
    if (k == kbeg && threadIdx.x == 0) skip = inv_skip(st, trs, p) ? 1 : 0;
    if (k > kbeg) __syncthreads();  // the previous MFMAs are done with As, Bs
    store64x2(nx, As, Bs);
    __syncthreads();
    if (skip) return;
    tile_mma64<false>(acc, As, Bs);
  }
  const int64_t r0 = (int64_t)(c0 + i) * kNb, q0 = (int64_t)(a0 + j) * kNb;
  double* out = PHASE == 0 ? Tp : Xp;
  tile_store64(acc, [&](int rr, int cc, double v) {
    const int64_t row = r0 + rr, col = q0 + cc;
    if (row < d && col < d) out[row * d + col] = PHASE == 0 ? v : -v;
  });
}

// H^{-1} block (I, J), I >= J, per workgroup; the first operand pair is
// requested together with the status, later pairs one at a time (a small
// register footprint, so a workgroup fits beside the bucket gather's waves).
__global__ __launch_bounds__(256, 3) void k_lauum(const double* __restrict__ Linv, double* Hinv,
                                               int64_t d, int32_t nblk, const DeviceStatus* st,
                                               const double* __restrict__ trs) {
  __shared__ Tile64 As, Bs;
  __shared__ int skip;
  const int p = blockIdx.y;
  const int64_t t = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  const int64_t J = t - I * (I + 1) / 2;
  const int64_t Ib = I * kNb, Jb = J * kNb;
  const double* Xp = Linv + (int64_t)p * d * d;
  double* Hp = Hinv + (int64_t)p * d * d;
  const int64_t kend = (int64_t)nblk * kNb;
  f64x4 acc[2][2] = {};
  for (int64_t kb = Ib; kb < kend; kb += kNb) {  // sum_k Linv_kI^T Linv_kJ
    Pair64 nx;
    load64x2(nx, Xp, kb, Ib, Xp, kb, Jb, d);
    if (kb == Ib && threadIdx.x == 0) skip = inv_skip(st, trs, p) ? 1 : 0;
    if (kb > Ib) __syncthreads();  // the previous MFMAs are done with As, Bs
    store64x2(nx, As, Bs);
    __syncthreads();
    if (skip) return;
    tile_mma64<true>(acc, As, Bs);
  }
  tile_store64(acc, [&](int rr, int cc, double v) {
    const int64_t row = Ib + rr, col = Jb + cc;
    if (row < d && col < d) {
      Hp[row * d + col] = v;
      if (I != J) Hp[col * d + row] = v;
    }
  });
}

hipError_t launch_chol_inverse(const double* L, const double* rdiag, int64_t d, int32_t batch,
                               double* Hinv, double* Linv, DeviceStatus* status, hipStream_t st,
                               const double* trs) {
  const int32_t nblk = (int32_t)((d + kNb - 1) / kNb);
  hipLaunchKernelGGL(k_trtri_diag, dim3(nblk, batch), dim3(256), 0, st, L, rdiag, d, Linv, status,
                     trs);
  for (int32_t h = 1; h < nblk; h *= 2) {
    const dim3 grid((unsigned)(h * h), (unsigned)((nblk + 2 * h - 1) / (2 * h)), batch);
    hipLaunchKernelGGL(k_trtri_merge<0>, grid, dim3(256), 0, st, L, Linv, Hinv, d, nblk, h,
                       status, trs);
    hipLaunchKernelGGL(k_trtri_merge<1>, grid, dim3(256), 0, st, L, Linv, Hinv, d, nblk, h,
                       status, trs);
  }
  const unsigned ntri = (unsigned)(nblk * (nblk + 1) / 2);
  hipLaunchKernelGGL(k_lauum, dim3(ntri, batch), dim3(256), 0, st, Linv, Hinv, d, nblk, status,
                     trs);
  return hipGetLastError();
}

// x_out = x + Hinv g per problem, one wavefront per row of Hinv (a symmetric
// matrix, so row i is column i). A second kernel records sqrt(dx^T g) and
// checks finiteness. Skips (x_out = x) on a recorded failure.
__global__ __launch_bounds__(256) void k_inv_apply(const double* __restrict__ Hinv, int64_t d,
                                                   const double* __restrict__ g,
                                                   const double* x, double* x_out, double* dx,
                                                   const DeviceStatus* st,
                                                   const DeviceStatus* gate, int32_t gate_iter) {
  const int p = blockIdx.y;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= d) return;
  const bool skip = status_halted(st) || (gate && status_failed_by(gate, gate_iter));
  const double* hr = Hinv + ((int64_t)p * d + i) * d;
  const double* gp = g + (int64_t)p * d;
  const double s = row_dot<false>(hr, gp, d, lane);
  if (lane == 0) {
    const int64_t k = (int64_t)p * d + i;
    dx[k] = skip ? 0.0 : s;
    x_out[k] = skip ? x[k] : x[k] + s;
  }
}

__global__ __launch_bounds__(256) void k_inv_finish(int64_t d, int32_t batch, const double* g,
                                                    const double* dx, const double* x_out,
                                                    DeviceStatus* st) {
  __shared__ double red[256];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (status_halted(st)) return;  // uniform: no update was applied
  if (tid == 0) bad = 0;
  __syncthreads();
  double part = 0.0;
  for (int64_t k = tid; k < (int64_t)batch * d; k += 256) {
    if (k < d) part = fma(dx[k], g[k], part);
    if (!isfinite(x_out[k])) bad = 1;
  }
  red[tid] = part;
  __syncthreads();
  for (int stride = 128; stride > 0; stride >>= 1) {
    if (tid < stride) red[tid] += red[tid + stride];
    __syncthreads();
  }
  if (tid == 0) {
    if (bad) status_fail(st, 7 /* IHS_ERR_NONFINITE */, -1, 0);
    st->last_step = sqrt(fmax(red[0], 0.0));
  }
}

hipError_t launch_inv_apply(const double* Hinv, int64_t d, int32_t batch, const double* g,
                            const double* x, double* x_out, double* dx, DeviceStatus* status,
                            hipStream_t st, const DeviceStatus* gate, int32_t gate_iter) {
  hipLaunchKernelGGL(k_inv_apply, dim3((unsigned)((d + 3) / 4), batch), dim3(256), 0, st, Hinv, d,
                     g, x, x_out, dx, status, gate, gate_iter);
  hipLaunchKernelGGL(k_inv_finish, dim3(1), dim3(256), 0, st, d, batch, g, dx, x_out, status);
  return hipGetLastError();
}

__global__ void k_recip_diag(const double* L, int64_t d, int32_t batch, double* rdiag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)batch * d) return;
  const int64_t p = i / d, j = i - p * d;
  rdiag[i] = 1.0 / L[p * d * d + j * d + j];
}

hipError_t launch_recip_diag(const double* L, int64_t d, int32_t batch, double* rdiag,
                             hipStream_t st) {
  const int64_t n = (int64_t)batch * d;
  hipLaunchKernelGGL(k_recip_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, L, d,
                     batch, rdiag);
  return hipGetLastError();
}

// Reciprocal pivots inside the Cholesky scratch (after the side buffers).
double* chol_rdiag(double* scratch, int32_t batch) { return scratch + (int64_t)batch * kNb * kNb; }

// ---------------------------------------------------------------------------
// Recurrences of conjugate gradients preconditioned by a fixed Hessian sketch
// (one 256-thread workgroup per problem; every dot product is summed in a
// fixed order, strided per-thread partials and then a tree). pm holds -p, so
// that the natural-order gradient pass with b = 0 and x = pm returns
// q = A^T A p. rho[p] carries r^T z between iterations.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_dot256(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int stride = 128; stride > 0; stride >>= 1) {
    if (tid < stride) red[tid] += red[tid + stride];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// rho = r^T z, pm = -z.
__global__ __launch_bounds__(256) void k_pcg_begin(const double* __restrict__ r,
                                                   const double* __restrict__ z, double* pm,
                                                   double* rho, int64_t d,
                                                   const DeviceStatus* st) {
  __shared__ double red[256];
  __shared__ int skip;
  const int p = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) skip = status_halted(st) ? 1 : 0;
  __syncthreads();
  if (skip) return;
  const double* rp = r + (int64_t)p * d;
  const double* zp = z + (int64_t)p * d;
  double part = 0.0;
  for (int64_t i = tid; i < d; i += 256) {
    part = fma(rp[i], zp[i], part);
    pm[(int64_t)p * d + i] = -zp[i];
  }
  const double rz = block_dot256(part, red);
  if (tid == 0) rho[p] = rz;
}

// alpha = rho / p^T q, x += alpha p, r -= alpha q. A non-positive curvature
// p^T q (A^T A not positive definite) is recorded as IHS_ERR_NOT_PD, a
// non-finite one as IHS_ERR_NONFINITE; a zero rho (r = 0: the solution is
// reached) leaves x and r as they are.
__global__ __launch_bounds__(256) void k_pcg_x(const double* __restrict__ pm,
                                               const double* __restrict__ q,
                                               const double* __restrict__ rho, double* x,
                                               double* r, int64_t d, DeviceStatus* st,
                                               int32_t iter) {
  __shared__ double red[256];
  __shared__ int skip;
  const int p = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) skip = status_halted(st) ? 1 : 0;
  __syncthreads();
  if (skip) return;
  const double* pp = pm + (int64_t)p * d;
  const double* qp = q + (int64_t)p * d;
  double part = 0.0;
  for (int64_t i = tid; i < d; i += 256) part = fma(-pp[i], qp[i], part);
  const double pq = block_dot256(part, red);
  const double rz = rho[p];
  if (rz == 0.0) return;
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (tid == 0)
      status_fail(st, isfinite(pq) ? 5 /* IHS_ERR_NOT_PD */ : 7 /* IHS_ERR_NONFINITE */, iter, p);
    return;
  }
  const double alpha = rz / pq;
  for (int64_t i = tid; i < d; i += 256) {
    const int64_t k = (int64_t)p * d + i;
    x[k] = fma(-alpha, pp[i], x[k]);
    r[k] = fma(-alpha, qp[i], r[k]);
  }
}

// rho' = r^T z, pm = -z + (rho' / rho) pm, rho = rho'.
__global__ __launch_bounds__(256) void k_pcg_p(const double* __restrict__ r,
                                               const double* __restrict__ z, double* pm,
                                               double* rho, int64_t d, const DeviceStatus* st) {
  __shared__ double red[256];
  __shared__ int skip;
  const int p = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) skip = status_halted(st) ? 1 : 0;
  __syncthreads();
  if (skip) return;
  const double* rp = r + (int64_t)p * d;
  const double* zp = z + (int64_t)p * d;
  double part = 0.0;
  for (int64_t i = tid; i < d; i += 256) part = fma(rp[i], zp[i], part);
  const double rz_old = rho[p];
  const double rz = block_dot256(part, red);
  const double beta = rz_old > 0.0 ? rz / rz_old : 0.0;
  for (int64_t i = tid; i < d; i += 256) {
    const int64_t k = (int64_t)p * d + i;
    pm[k] = fma(beta, pm[k], -zp[i]);
  }
  if (tid == 0) rho[p] = rz;
}

hipError_t launch_pcg_begin(const double* r, const double* z, double* pm, double* rho, int64_t d,
                            int32_t batch, const DeviceStatus* status, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_begin, dim3(batch), dim3(256), 0, st, r, z, pm, rho, d, status);
  return hipGetLastError();
}

hipError_t launch_pcg_x(const double* pm, const double* q, const double* rho, double* x,
                        double* r, int64_t d, int32_t batch, DeviceStatus* status, int32_t iter,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_x, dim3(batch), dim3(256), 0, st, pm, q, rho, x, r, d, status, iter);
  return hipGetLastError();
}

hipError_t launch_pcg_p(const double* r, const double* z, double* pm, double* rho, int64_t d,
                        int32_t batch, const DeviceStatus* status, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_p, dim3(batch), dim3(256), 0, st, r, z, pm, rho, d, status);
  return hipGetLastError();
}

// Per-problem scratch of the QP kernels: the 64 x 64 diagonal-block side
// buffer of the blocked Cholesky plus vectors.
size_t qp_work_doubles(int64_t d, int32_t constraint) {
  // ball steps add c, the unconstrained minimiser, two Newton vectors, a
  // spare vector and the shift state; the l2 step also H^{-1}, L^{-1} and the
  // series vectors;
  // the wide unconstrained step H^{-1}, L^{-1} and its dx
  size_t n = (size_t)(kNb * kNb + 9 * d + 64);
  if (constraint == 0 && d >= kQpInverseMinD) n += (size_t)(2 * d * d + d);
  if (constraint != 0) n += (size_t)(5 * d + 8);
  if (constraint == 2)
    n += (size_t)(2 * d * d + (kL2SeriesTerms + 1) * d);
  return n;
}

hipError_t launch_qp_step(const QpArgs& a, hipStream_t st) {
  if (a.constraint != 0) return launch_qp_constrained(a, st);
  hipError_t e = launch_cholesky(a.H, a.L, a.d, a.batch, a.status, a.iter, 0.0,
                                 a.work, st);
  if (e != hipSuccess) return e;
  double* rdiag = chol_rdiag(a.work, a.batch);
  if (a.d < kQpInverseMinD)
    return launch_chol_solve_update(a.L, rdiag, a.d, a.batch, a.g, a.x, a.x_out, a.status, st);
  double* hinv = a.work + (int64_t)a.batch * (kNb * kNb + 9 * a.d + 64);
  double* linv = hinv + (int64_t)a.batch * a.d * a.d;
  double* dx = linv + (int64_t)a.batch * a.d * a.d;
  if ((e = launch_chol_inverse(a.L, rdiag, a.d, a.batch, hinv, linv, a.status, st)) != hipSuccess)
    return e;
  return launch_inv_apply(hinv, a.d, a.batch, a.g, a.x, a.x_out, dx, a.status, st, nullptr, 0);
}


// ---------------------------------------------------------------------------
// The outer loop's tolerance stop (Thm 2.2: the error contracts by a constant
// factor per step, so the prediction-norm length of a step bounds the error
// within a constant factor). After step t, with dx = x^{t+1} - x^t per
// problem, q_p = dx^T H_t dx, or dx^T g when the step solved H_t dx = g
// (H == nullptr; equal to it up to rounding). When no failure is recorded and
// every sqrt(q_p) <= tol, the step test sets `done` and `iters` = t + 1; the
// update kernels of later steps then keep x, and the passes return at once.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_step_rows(const double* __restrict__ H, int64_t d,
                                                   const double* __restrict__ xprev,
                                                   const double* __restrict__ x, double* q) {
  const int p = blockIdx.y;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= d) return;
  const double* xp = x + (int64_t)p * d;
  const double* xo = xprev + (int64_t)p * d;
  // (H dx)_i from the row of H and dx formed lane by lane, columns in order
  const double* hr = H + ((int64_t)p * d + i) * d;
  double s = 0.0;
  for (int64_t k0 = 0; k0 < d; k0 += 64) {
    const int64_t k = k0 + lane;
    const double dk = k < d ? xp[k] - xo[k] : 0.0;
    const double h = k < d ? hr[k] : 0.0;
    s = fma(h, dk, s);
  }
  s = wave_sum(s);
  if (lane == 0) q[(int64_t)p * d + i] = s * (xp[i] - xo[i]);
}

__global__ __launch_bounds__(256) void k_step_test(const double* __restrict__ q,
                                                   const double* __restrict__ g,
                                                   const double* __restrict__ xprev,
                                                   const double* __restrict__ x, int64_t d,
                                                   int32_t batch, double tol, DeviceStatus* st,
                                                   int32_t iter) {
  __shared__ double red[256];
  __shared__ int over;
  const int tid = threadIdx.x;
  if (status_halted(st)) return;  // uniform: failures and an earlier stop keep their record
  if (tid == 0) over = 0;
  __syncthreads();
  double q0 = 0.0;
  for (int32_t p = 0; p < batch; ++p) {
    double part = 0.0;
    for (int64_t i = tid; i < d; i += 256) {
      const int64_t k = (int64_t)p * d + i;
      part += g != nullptr ? (x[k] - xprev[k]) * g[k] : q[k];
    }
    red[tid] = part;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
      if (tid < stride) red[tid] += red[tid + stride];
      __syncthreads();
    }
    const double qp = red[0];
    if (tid == 0) {
      if (p == 0) q0 = qp;
      if (!(sqrt(fmax(qp, 0.0)) <= tol)) over = 1;
    }
    __syncthreads();
  }
  if (tid == 0) {
    st->last_step = sqrt(fmax(q0, 0.0));
    if (!over) {
      st->iters = iter + 1;
      __hip_atomic_store(&st->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

hipError_t launch_step_test(const double* H, const double* g, const double* xprev,
                            const double* x, int64_t d, int32_t batch, double tol, double* q,
                            DeviceStatus* status, int32_t iter, hipStream_t st) {
  if (H != nullptr)
    hipLaunchKernelGGL(k_step_rows, dim3((unsigned)((d + 3) / 4), batch), dim3(256), 0, st, H, d,
                       xprev, x, q);
  hipLaunchKernelGGL(k_step_test, dim3(1), dim3(256), 0, st, q, H != nullptr ? nullptr : g,
                     xprev, x, d, batch, tol, status, iter);
  return hipGetLastError();
}

}  // namespace ihs
