// Sparse-embedding kernels: hash, bucket sort, and the bucket gather that
// forms S A (Sec. 2, CountSketch / SJLT and their streaming application),
// fused with the residual, objective and gradient pass of Eq.(2).
//
// Design (gfx950):
//  * The hash is a pure function of (seed, iteration, row, block, problem)
//    (Philox4x64-10), so no random state is stored.
//  * Rows are sorted by sketch row with a stable counting sort: a per-tile
//    LDS histogram, a three-level exclusive scan, and a scatter that ranks
//    equal keys inside a wavefront with ballots. Integer atomics in LDS only.
//  * Each sketch row (bucket) is owned by one wavefront, which streams its
//    input rows in ascending order as contiguous 16-byte-per-lane loads and
//    keeps the accumulators in registers. No floating-point atomics: every
//    sum runs in the sequential order of the definition, so S A is bitwise
//    reproducible and equal to a sequential evaluation.
#include <algorithm>

#include "kernels.hpp"

namespace ihs {

__device__ __forceinline__ int find_by_tile(const ProbInfo* probs, int batch, int tile) {
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_by_chunk(const ProbInfo* probs, int batch, int c) {
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].chunk0 <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_by_seg(const ProbInfo* probs, int batch, int sgi) {
  int lo = 0, hi = batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].seg0 <= sgi) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Problem table upload through kernel arguments (no host buffer must outlive
// the call, and the copy is safe under stream capture).
// ---------------------------------------------------------------------------
__global__ void k_write_probs(ProbChunk c, ProbInfo* dst) {
  const int i = threadIdx.x;
  if (i < c.count) dst[c.first + i] = c.p[i];
}

hipError_t launch_write_probs(const ProbInfo* host, int32_t batch, ProbInfo* dst,
                              hipStream_t st) {
  for (int32_t f = 0; f < batch; f += kProbChunk) {
    ProbChunk c{};
    c.first = f;
    c.count = std::min<int32_t>(kProbChunk, batch - f);
    for (int32_t i = 0; i < c.count; ++i) c.p[i] = host[f + i];
    hipLaunchKernelGGL(k_write_probs, dim3(1), dim3(kProbChunk), 0, st, c, dst);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hash of one problem's rows, for inspection: bucket[i*s+k], sign[i*s+k].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sketch_hash(int64_t n, int32_t problem, int32_t s,
                                                     int64_t m_blk, uint64_t seed,
                                                     uint64_t iter, int32_t* bucket,
                                                     int8_t* sign) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < (s + 1) / 2; ++q) {
    const U64x4 w = philox4x64_10((uint64_t)i, (uint64_t)q, (uint64_t)problem, 0ull, seed, iter);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = 2 * q + h;
      if (k < s) {
        const uint32_t lb = range_reduce(w.w[2 * h], (uint64_t)m_blk);
        bucket[i * s + k] = (int32_t)(k * m_blk + lb);
        sign[i * s + k] = (w.w[2 * h + 1] >> 63) ? (int8_t)-1 : (int8_t)1;
      }
    }
  }
}

hipError_t launch_sketch_hash(const SketchPlan& p, int64_t n, int32_t problem,
                              int32_t* bucket, int8_t* sign, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_sketch_hash, dim3((unsigned)blocks), dim3(256), 0, st, n, problem,
                     p.s, p.m_blk, p.seed, p.iter, bucket, sign);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sort step 1: hash every (row, block) of a tile, store its key, and count
// keys per sketch row in LDS.
// ---------------------------------------------------------------------------
// Tiles are visited grid-stride by a capped grid, so the sort never takes
// more than a small share of the CUs beside a running pass over A.
__global__ __launch_bounds__(256) void k_hash_count(SketchPlan P) {
  extern __shared__ int32_t cnt[];
  for (int tile = blockIdx.x; tile < P.total_tiles; tile += gridDim.x) {
  const int p = find_by_tile(P.probs, P.batch, tile);
  const ProbInfo pi = P.probs[p];
  const int64_t lr0 = (int64_t)(tile - pi.tile0) * P.tile_rows;
  const int64_t nr = min((int64_t)P.tile_rows, pi.rows - lr0);
  for (int64_t b = threadIdx.x; b < P.m; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  const int npairs = (P.s + 1) / 2;
  for (int64_t i = threadIdx.x; i < nr; i += blockDim.x) {
    const int64_t lrow = lr0 + i;
    const int64_t grow = pi.row0 + lrow;
    for (int q = 0; q < npairs; ++q) {
      const U64x4 w = philox4x64_10((uint64_t)lrow, (uint64_t)q, (uint64_t)p, 0ull, P.seed,
                                    P.iter);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * q + h;
        if (k < P.s) {
          const uint32_t bkt = (uint32_t)(k * P.m_blk) + range_reduce(w.w[2 * h], (uint64_t)P.m_blk);
          const uint32_t neg = (uint32_t)(w.w[2 * h + 1] >> 63);
          P.keys[grow * P.s + k] = bkt | (neg << 31);
          atomicAdd(&cnt[bkt], 1);
        }
      }
    }
  }
  __syncthreads();
  int32_t* out = P.tile_count + (int64_t)tile * P.m;
  for (int64_t b = threadIdx.x; b < P.m; b += blockDim.x) out[b] = cnt[b];
  __syncthreads();  // the LDS histogram is reused by the next tile
  }
}

// The scan steps walk a column of counts (one sketch row, many tiles or
// chunks); each thread requests kScanBatch entries at once, so a column costs
// a round trip per kScanBatch entries rather than per entry.
constexpr int kScanBatch = 16;

// Sort step 2a: per (chunk of tiles, sketch row) totals.
__global__ __launch_bounds__(256) void k_scan_chunks(SketchPlan P) {
  const int c = blockIdx.x;
  const int64_t b = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (b >= P.m) return;
  const int p = find_by_chunk(P.probs, P.batch, c);
  const ProbInfo pi = P.probs[p];
  const int t0 = pi.tile0 + (c - pi.chunk0) * P.tiles_per_chunk;
  const int t1 = min(t0 + P.tiles_per_chunk, pi.tile0 + pi.ntiles);
  int32_t sum = 0;
  for (int t = t0; t < t1; t += kScanBatch) {
    int32_t v[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u)
      v[u] = t + u < t1 ? P.tile_count[(int64_t)(t + u) * P.m + b] : 0;
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) sum += v[u];
  }
  P.chunk_part[(int64_t)c * P.m + b] = sum;
}

// Sort step 2b: per sketch row, exclusive scan over the problem's chunks (in
// place); the row's total goes to bucket_start, which step 2b' turns into the
// exclusive scan over sketch rows.
__global__ __launch_bounds__(256) void k_scan_rows(SketchPlan P) {
  const int p = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= P.m) return;
  const ProbInfo pi = P.probs[p];
  int32_t run = 0;
  const int c1 = pi.chunk0 + pi.nchunks;
  for (int c = pi.chunk0; c < c1; c += kScanBatch) {
    int32_t v[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u)
      v[u] = c + u < c1 ? P.chunk_part[(int64_t)(c + u) * P.m + b] : 0;
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) {
      if (c + u < c1) P.chunk_part[(int64_t)(c + u) * P.m + b] = run;
      run += v[u];
    }
  }
  P.bucket_start[(int64_t)p * P.m + b] = run;
}

// Sort step 2b': one workgroup per problem turns the sketch-row totals into
// segment starts (exclusive scan, offset by the problem's first entry).
__global__ __launch_bounds__(1024) void k_scan_totals(SketchPlan P) {
  __shared__ int32_t wsum[16];
  const int p = blockIdx.x;
  const ProbInfo pi = P.probs[p];
  const int tid = threadIdx.x;
  int32_t* tot = P.bucket_start + (int64_t)p * P.m;
  const int64_t per = (P.m + 1023) / 1024;
  const int64_t lo = min((int64_t)tid * per, P.m), hi = min(lo + per, P.m);
  int32_t s = 0;
  for (int64_t b = lo; b < hi; ++b) s += tot[b];
  const int lane = tid & 63, wv = tid >> 6;
  int32_t incl = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (tid == 0) {
    int32_t run = 0;
    for (int w = 0; w < 16; ++w) {
      const int32_t v = wsum[w];
      wsum[w] = run;
      run += v;
    }
  }
  __syncthreads();
  int32_t base = (int32_t)(pi.row0 * P.s) + wsum[wv] + incl - s;
  for (int64_t b = lo; b < hi; ++b) {
    const int32_t v = tot[b];
    tot[b] = base;
    base += v;
  }
  if (p == P.batch - 1 && tid == 0) P.bucket_start[(int64_t)P.batch * P.m] = (int32_t)P.entries;
}

// Sort step 2c: absolute start of every (tile, sketch row) block.
__global__ __launch_bounds__(256) void k_scan_tiles(SketchPlan P) {
  const int c = blockIdx.x;
  const int64_t b = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (b >= P.m) return;
  const int p = find_by_chunk(P.probs, P.batch, c);
  const ProbInfo pi = P.probs[p];
  const int t0 = pi.tile0 + (c - pi.chunk0) * P.tiles_per_chunk;
  const int t1 = min(t0 + P.tiles_per_chunk, pi.tile0 + pi.ntiles);
  int32_t run = P.bucket_start[(int64_t)p * P.m + b] + P.chunk_part[(int64_t)c * P.m + b];
  for (int t = t0; t < t1; t += kScanBatch) {
    int32_t v[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u)
      v[u] = t + u < t1 ? P.tile_count[(int64_t)(t + u) * P.m + b] : 0;
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) {
      if (t + u < t1) P.tile_count[(int64_t)(t + u) * P.m + b] = run;
      run += v[u];
    }
  }
}

// Sort step 3: stable scatter. The tile's rows are taken 256 at a time in
// ascending order, one block of the SJLT at a time (blocks own disjoint
// sketch rows, so their order does not matter). Every wavefront ranks its
// lanes among equal keys with one ballot per key bit; then the four
// wavefronts take turns to claim positions from the LDS cursors. The keys of
// the next step are requested before the turns of the current one, so the
// turns never wait for memory.
// Workgroups are dispatched to the XCDs round-robin; the scatter hands each
// XCD a contiguous run of tiles, so consecutive entries of a sketch row's list
// are written through one L2, which assembles whole lines before they go out.
constexpr int kXcds = 8;

__global__ __launch_bounds__(256) void k_scatter(SketchPlan P) {
  extern __shared__ int32_t pos[];
  const int wv = threadIdx.x >> 6;
  const uint64_t lt = lanemask_lt();
  const int G = gridDim.x, q = G / kXcds, r = G % kXcds;
  const int x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
  const int first = x * q + min(x, r) + j;  // a bijection of [0, G)
  for (int tile = first; tile < P.total_tiles; tile += G) {
    const int p = find_by_tile(P.probs, P.batch, tile);
    const ProbInfo pi = P.probs[p];
    const int64_t lr0 = (int64_t)(tile - pi.tile0) * P.tile_rows;
    const int64_t nr = min((int64_t)P.tile_rows, pi.rows - lr0);
    const int64_t row0 = pi.row0 + lr0;
    const int64_t nsteps = ((nr + 255) / 256) * P.s;
    auto key_at = [&](int64_t step) -> uint32_t {
      const int64_t i = (step / P.s) * 256 + threadIdx.x;
      return i < nr ? P.keys[(row0 + i) * P.s + (int)(step % P.s)] : 0u;
    };
    uint32_t kv_next = nsteps > 0 ? key_at(0) : 0u;
    const int32_t* start = P.tile_count + (int64_t)tile * P.m;
    for (int64_t b = threadIdx.x; b < P.m; b += blockDim.x) pos[b] = start[b];
    __syncthreads();
    for (int64_t step = 0; step < nsteps; ++step) {
      const uint32_t kv = kv_next;
      if (step + 1 < nsteps) kv_next = key_at(step + 1);
      const int64_t i = (step / P.s) * 256 + threadIdx.x;
      const bool valid = i < nr;
      const uint32_t bkt = kv & 0x7FFFFFFFu;
      uint64_t peers = __ballot(valid);
      for (int bit = 0; bit < P.bucket_bits; ++bit) {
        const bool on = (bkt >> bit) & 1u;
        const uint64_t bb = __ballot(on);
        peers &= on ? bb : ~bb;
      }
      const int rank = __popcll(peers & lt);
      for (int w = 0; w < 4; ++w) {
        if (wv == w && valid) {
          const int32_t p0 = pos[bkt];
          P.perm[p0 + rank] = (uint32_t)(row0 + i) | (kv & 0x80000000u);
          if (rank == 0) pos[bkt] = p0 + __popcll(peers);
        }
        __syncthreads();
      }
    }
    __syncthreads();  // pos is reloaded for the next tile
  }
}

// Sort step 4 (dense gather with two sketch rows per wavefront): the list
// lengths vary from sketch row to sketch row, and a wavefront that streams two
// long lists finishes well after the others. Within every block the rows are
// ranked by (length descending, index ascending), and rank r goes to position
// 2r for r < ceil(m_blk/2), else to 2(m_blk-1-r)+1: each wavefront then takes
// one long and one short list. Each sketch row keeps its own list and order,
// so S A is unchanged; the order is a function of the lengths alone.
// A 1024-thread workgroup stages its block's lengths in LDS once; each of its
// sixteen wavefronts then ranks one sketch row against them.
constexpr int kPairThreads = 1024;
constexpr int kPairPerGroup = kPairThreads / 64;

__global__ __launch_bounds__(kPairThreads) void k_pair_order(SketchPlan P) {
  extern __shared__ int32_t len[];
  const int p = blockIdx.z, blk = blockIdx.y;
  const int64_t mb = P.m_blk;
  const int32_t* bs = P.bucket_start + (int64_t)p * P.m + (int64_t)blk * mb;
  // every thread requests 8 list extents before it stores their lengths
  for (int64_t j0 = 0; j0 < mb; j0 += 8 * kPairThreads) {
    int32_t lo[8], hi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t j = j0 + u * kPairThreads + threadIdx.x;
      lo[u] = j < mb ? bs[j] : 0;
      hi[u] = j < mb ? bs[j + 1] : 0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t j = j0 + u * kPairThreads + threadIdx.x;
      if (j < mb) len[j] = hi[u] - lo[u];
    }
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = (int64_t)blockIdx.x * kPairPerGroup + wv;
  if (r0 >= mb) return;  // no barriers below
  const int32_t mine = len[r0];
  int32_t cnt = 0;
#pragma unroll 8
  for (int64_t j = lane; j < mb; j += 64) {
    const int32_t v = len[j];
    cnt += (v > mine || (v == mine && j < r0)) ? 1 : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if (lane == 0) {
    const int64_t half = (mb + 1) / 2;
    const int64_t pos = cnt < half ? 2 * (int64_t)cnt : 2 * (mb - 1 - cnt) + 1;
    P.border[(int64_t)p * P.m + (int64_t)blk * mb + pos] = (int32_t)((int64_t)blk * mb + r0);
  }
}

constexpr int32_t kSortGrid = 2048;  // workgroup cap of the tile-parallel sort kernels

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_sort(const SketchPlan& P, hipStream_t st, hipEvent_t after_hash) {
  const unsigned gy = (unsigned)((P.m + 255) / 256);
  if (P.total_tiles == 0) {
    // every problem is empty: all segments start (and end) at 0
    const int64_t nb = (int64_t)P.batch * P.m + 1;
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st,
                       P.bucket_start, nb);
    if (after_hash != nullptr) {
      const hipError_t e = hipEventRecord(after_hash, st);
      if (e != hipSuccess) return e;
    }
  } else {
    const size_t lds_m = (size_t)P.m * sizeof(int32_t);
    const unsigned tiles_grid = (unsigned)std::min<int32_t>(P.total_tiles, kSortGrid);
    hipLaunchKernelGGL(k_hash_count, dim3(tiles_grid), dim3(256), lds_m, st, P);
    if (after_hash != nullptr) {
      const hipError_t e = hipEventRecord(after_hash, st);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_chunks, dim3(P.total_chunks, gy), dim3(256), 0, st, P);
    hipLaunchKernelGGL(k_scan_rows, dim3(gy, P.batch), dim3(256), 0, st, P);
    hipLaunchKernelGGL(k_scan_totals, dim3(P.batch), dim3(1024), 0, st, P);
    hipLaunchKernelGGL(k_scan_tiles, dim3(P.total_chunks, gy), dim3(256), 0, st, P);
    hipLaunchKernelGGL(k_scatter, dim3(tiles_grid), dim3(256), lds_m, st, P);
  }
  if (P.border != nullptr)
    hipLaunchKernelGGL(k_pair_order,
                       dim3((unsigned)((P.m_blk + kPairPerGroup - 1) / kPairPerGroup), P.s, P.batch),
                       dim3(kPairThreads), (size_t)P.m_blk * sizeof(int32_t), st, P);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense bucket gather, optionally fused with r = b - A x, g = A^T r, f.
// Lane l owns columns c*64*VEC + l*VEC + v (c < NCH, v < VEC).
// ---------------------------------------------------------------------------
// VEC consecutive elements of a row in one load, kept in the row's own
// type until use (so float rows take half the registers).
template <typename TA, int VEC>
struct VecLoad {
  static __device__ __forceinline__ void ld(const TA* p, TA* o) {
    if constexpr (VEC == 1) {
      o[0] = *p;
    } else if constexpr (sizeof(TA) == 8 && VEC == 2) {
      const double2 v = *reinterpret_cast<const double2*>(p);
      o[0] = v.x;
      o[1] = v.y;
    } else if constexpr (sizeof(TA) == 4 && VEC == 2) {
      const float2 v = *reinterpret_cast<const float2*>(p);
      o[0] = v.x;
      o[1] = v.y;
    } else {
      static_assert(sizeof(TA) == 4 && VEC == 4, "16-byte loads of floats");
      const float4 v = *reinterpret_cast<const float4*>(p);
      o[0] = v.x;
      o[1] = v.y;
      o[2] = v.z;
      o[3] = v.w;
    }
  }
};

__device__ __forceinline__ void store_sa(void* SA, int32_t dt, int64_t idx, double v) {
  if (dt == 0) {
    static_cast<double*>(SA)[idx] = v;
  } else if (dt == 1) {
    static_cast<float*>(SA)[idx] = (float)v;
  } else {
    static_cast<uint16_t*>(SA)[idx] = f64_to_bf16_bits(v);
  }
}

// Sum of U per-lane partial vectors across the wavefront with a transposing
// butterfly: each exchange step halves the number of live values, so U row
// sums cost log2(U) + (6 - log2(U)) exchanges of decreasing width instead of
// 6 U. Afterwards lanes with bits (32, 16, ...) equal to the row index bits
// hold that row's total; row_lane<U>(u) names one such lane. Fixed order.
template <int U>
__device__ __forceinline__ double multi_row_sum(const double (&v)[U], int lane) {
  double cur[U];
#pragma unroll
  for (int i = 0; i < U; ++i) cur[i] = v[i];
  int off = 32;
#pragma unroll
  for (int n = U; n > 1; n >>= 1) {
    const bool hi = (lane & off) != 0;
    const int h = n / 2;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const double send = hi ? cur[i] : cur[h + i];
      const double keep = hi ? cur[h + i] : cur[i];
      cur[i] = keep + __shfl_xor(send, off, 64);
    }
    off >>= 1;
  }
  double s = cur[0];
#pragma unroll
  for (; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

template <int U>
__device__ __forceinline__ int row_lane(int u) {
  // row u's bits, most significant first, select lanes 32, 16, ...
  int lane = 0, off = 32;
#pragma unroll
  for (int bit = U / 2; bit > 0; bit >>= 1, off >>= 1)
    if (u & bit) lane += off;
  return lane;
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// IDENT: natural row order (no sketch): wavefront w takes rows
// [row0 + seg*seg_rows, ...) of its problem, and only the gradient is formed.
// Otherwise the grid is (ceil(ceil(m/BPW)/4), batch): wavefront w of problem
// blockIdx.y owns positions [w*BPW, w*BPW + BPW) (the sketch rows that
// P.border names for them when it is set, else the same rows) and streams
// them one after the other, so each sketch row is still summed in ascending
// input-row order by one lane per column. Owning two sketch rows halves the
// number of resident wavefronts, which leaves room on every CU for the
// overlapped work of the next step. Each wavefront of block 0 writes one
// gradient partial.
template <typename TA, int VEC, int NCH, int U, int BPW, bool GRAD, bool IDENT>
__global__ __launch_bounds__(256, (BPW > 1 ? 3 : (NCH <= 4 ? 4 : 2))) void k_gather(
    SketchPlan P, GatherArgs G, int32_t total_seg, int32_t seg_rows) {
  // waves are independent (no workgroup barriers), so each may leave here
  if (G.halt != nullptr && status_word(G.halt) != 0) return;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t d = G.d;
  constexpr int SPAN = 64 * VEC;
  int p;
  int64_t wid, gslot, nown;
  bool active;
  if (IDENT) {
    wid = (int64_t)blockIdx.x * 4 + wv;
    active = wid < total_seg;
    p = active ? find_by_seg(P.probs, P.batch, (int)wid) : 0;
    gslot = wid;
    nown = 1;
  } else {
    p = blockIdx.y;
    wid = (int64_t)blockIdx.x * 4 + wv;
    const int64_t b0 = wid * BPW;
    active = b0 < P.m;
    nown = active ? min((int64_t)BPW, P.m - b0) : 0;
    gslot = (int64_t)p * ((P.m_blk + BPW - 1) / BPW) + wid;
  }
  const bool any_grad = GRAD && active && (IDENT || wid * BPW < P.m_blk);
  const TA* __restrict__ A = static_cast<const TA*>(G.A);

  double xr[NCH][VEC];
  double ga[NCH][VEC];
  double fa = 0.0;
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      ga[c][v] = 0.0;
      xr[c][v] = 0.0;
    }
  if (any_grad) {
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int64_t col = (int64_t)c * SPAN + lane * VEC + v;
        if (col < d) xr[c][v] = G.x[(int64_t)p * d + col];
      }
  }

  for (int64_t own = 0; own < nown; ++own) {
    int64_t bl, bg, beg, end;
    if (IDENT) {
      const ProbInfo pi = P.probs[p];
      bl = 0;
      bg = wid;
      beg = pi.row0 + (wid - pi.seg0) * (int64_t)seg_rows;
      end = min(beg + seg_rows, pi.row0 + pi.rows);
    } else {
      bl = wid * BPW + own;
      if (BPW > 1 && P.border != nullptr) bl = P.border[(int64_t)p * P.m + bl];
      bg = (int64_t)p * P.m + bl;
      beg = P.bucket_start[bg];
      end = P.bucket_start[bg + 1];
    }
    const bool grad = GRAD && (IDENT || bl < P.m_blk);  // block 0 visits every row once
    double acc[NCH][VEC];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[c][v] = 0.0;

    uint32_t pe_next = 0u;
    if (beg + lane < end) pe_next = IDENT ? (uint32_t)(beg + lane) : P.perm[beg + lane];
    for (int64_t base = beg; base < end; base += 64) {
      const int cnt = (int)min((int64_t)64, end - base);
      const uint32_t pe = pe_next;
      if (base + 64 + lane < end)  // next batch's row ids, one batch ahead
        pe_next = IDENT ? (uint32_t)(base + 64 + lane) : P.perm[base + 64 + lane];
      double bv = 0.0;
      if (grad && lane < cnt) bv = G.b ? G.b[pe & 0x7FFFFFFFu] : 0.0;
      for (int j = 0; j < cnt; j += U) {
        TA val[U][NCH][VEC];
        uint32_t ent[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int jj = min(j + u, cnt - 1);
          ent[u] = readlane_u32(pe, jj);
          const uint32_t row = ent[u] & 0x7FFFFFFFu;
          const TA* rp = A + (int64_t)row * G.ld;
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const int64_t col = (int64_t)c * SPAN + lane * VEC;
            if (col < d) {
              VecLoad<TA, VEC>::ld(rp + col, val[u][c]);
            } else {
#pragma unroll
              for (int v = 0; v < VEC; ++v) val[u][c][v] = TA(0);
            }
          }
        }
        if (grad) {
          double dot[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < NCH; ++c)
#pragma unroll
              for (int v = 0; v < VEC; ++v) s = fma((double)val[u][c][v], xr[c][v], s);
            dot[u] = s;
          }
          const double red = multi_row_sum<U>(dot, lane);
          if constexpr (sizeof(TA) == 4) {
            // convert the float rows again below rather than keep their
            // float64 copies live across the reduction (fewer registers)
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
              for (int c = 0; c < NCH; ++c)
#pragma unroll
                for (int v = 0; v < VEC; ++v) asm volatile("" : "+v"(val[u][c][v]));
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (j + u < cnt) {
              const double ri = readlane_f64(bv, j + u) - readlane_f64(red, row_lane<U>(u));
              fa = fma(ri, ri, fa);
#pragma unroll
              for (int c = 0; c < NCH; ++c)
#pragma unroll
                for (int v = 0; v < VEC; ++v)
                  ga[c][v] = fma(ri, (double)val[u][c][v], ga[c][v]);
              if (G.r_out != nullptr && lane == 0) G.r_out[ent[u] & 0x7FFFFFFFu] = ri;
            }
          }
        }
        if (!IDENT) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (j + u < cnt) {
              const bool neg = (ent[u] >> 31) != 0;
#pragma unroll
              for (int c = 0; c < NCH; ++c)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                  const double a = (double)val[u][c][v];
                  acc[c][v] = neg ? (acc[c][v] - a) : (acc[c][v] + a);
                }
            }
          }
        }
      }
    }
    if (!IDENT) {
      const int64_t orow = bg * G.ld_sa;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int64_t col = (int64_t)c * SPAN + lane * VEC + v;
          if (col < d) store_sa(G.SA, G.sa_dtype, orow + col, acc[c][v] * G.scale);
        }
    }
  }
  if (any_grad) {  // one partial per wavefront
    double* gp = G.gpart + gslot * d;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int64_t col = (int64_t)c * SPAN + lane * VEC + v;
        if (col < d) gp[col] = ga[c][v];
      }
    if (lane == 0) G.fpart[gslot] = fa;
  }
}

// Sketch rows per wavefront of the dense gather.
int32_t gather_rows_per_wave(int64_t m, int32_t batch, int64_t d) {
  return ((int64_t)batch * m >= 2048 && d > 64 && d <= 768) ? 2 : 1;
}

template <typename TA, int VEC, int NCH, bool GRAD, bool IDENT>
static hipError_t gather_inst(const SketchPlan& P, const GatherArgs& G, int32_t total_seg,
                              int32_t seg_rows, hipStream_t st) {
  // NE: chunks of 16 bytes per lane that a row occupies once converted
  constexpr int NE = VEC == 4 ? 2 * NCH : NCH;
  constexpr int UF = 1;
  if (IDENT) {
    // rows in flight per wavefront: enough with 16 wavefronts per CU, while the
    // register budget keeps 4 wavefronts per SIMD
    constexpr int U = std::min(8, UF * (NE == 1 ? 8 : (NE == 2 ? 4 : 2)));
    const unsigned blocks = (unsigned)((total_seg + 3) / 4);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_gather<TA, VEC, NCH, U, 1, GRAD, IDENT>), dim3(blocks), dim3(256), 0,
                       st, P, G, total_seg, seg_rows);
  } else if (gather_rows_per_wave(P.m, P.batch, G.d) == 2) {
    // half the wavefronts; about eight 16-byte loads per lane in flight, U rows
    // of NCH (measured in one process on the same sorted rows at 2^22 x 512
    // float64: two rows of four loads 2.86 ms against four rows 2.91; at
    // 2^20 x 256 four rows of two loads and two rows are equal; float32 rows
    // of two loads keep four rows in flight)
    constexpr int U = std::min(8, UF * (NE == 1 ? 8 : (NCH <= 2 ? 4 : 2)));
    const int64_t waves = (P.m + 1) / 2;
    hipLaunchKernelGGL((k_gather<TA, VEC, NCH, U, 2, GRAD, IDENT>),
                       dim3((unsigned)((waves + 3) / 4), P.batch), dim3(256), 0, st, P, G,
                       total_seg, seg_rows);
  } else {
    constexpr int U = std::min(8, UF * (NE == 1 ? 8 : (NE == 2 ? 4 : 2)));
    hipLaunchKernelGGL((k_gather<TA, VEC, NCH, U, 1, GRAD, IDENT>),
                       dim3((unsigned)((P.m + 3) / 4), P.batch), dim3(256), 0, st, P, G,
                       total_seg, seg_rows);
  }
  return hipGetLastError();
}

template <typename TA, int VEC, bool GRAD, bool IDENT>
static hipError_t gather_nch(const SketchPlan& P, const GatherArgs& G, int32_t ts, int32_t sr,
                             hipStream_t st) {
  const int64_t span = 64 * VEC;
  const int64_t nch = (G.d + span - 1) / span;
  // at most 1024 columns, i.e. 8 values per lane and row at VEC = 2
  switch (nch) {
    case 1: return gather_inst<TA, VEC, 1, GRAD, IDENT>(P, G, ts, sr, st);
    case 2: return gather_inst<TA, VEC, 2, GRAD, IDENT>(P, G, ts, sr, st);
    case 3: return gather_inst<TA, VEC, 3, GRAD, IDENT>(P, G, ts, sr, st);
    case 4: return gather_inst<TA, VEC, 4, GRAD, IDENT>(P, G, ts, sr, st);
    default: break;
  }
  if constexpr (VEC <= 2) {
    switch (nch) {
      case 5: return gather_inst<TA, VEC, 5, GRAD, IDENT>(P, G, ts, sr, st);
      case 6: return gather_inst<TA, VEC, 6, GRAD, IDENT>(P, G, ts, sr, st);
      case 7: return gather_inst<TA, VEC, 7, GRAD, IDENT>(P, G, ts, sr, st);
      case 8: return gather_inst<TA, VEC, 8, GRAD, IDENT>(P, G, ts, sr, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

// 16 bytes per lane per load when rows allow it: pairs of doubles, quads of
// floats; otherwise pairs of floats or single elements.
template <typename TA, bool GRAD, bool IDENT>
static hipError_t gather_vec(const SketchPlan& P, const GatherArgs& G, int32_t ts, int32_t sr,
                             hipStream_t st) {
  if constexpr (sizeof(TA) == 4) {
    const bool v4 = (G.d % 4 == 0) && (G.ld % 4 == 0) &&
                    ((reinterpret_cast<uintptr_t>(G.A) % 16) == 0) && G.d > 128;
    if (v4) return gather_nch<TA, 4, GRAD, IDENT>(P, G, ts, sr, st);
  }
  const bool v2 = (G.d % 2 == 0) && (G.ld % 2 == 0) &&
                  ((reinterpret_cast<uintptr_t>(G.A) % (2 * sizeof(TA))) == 0) && G.d > 64;
  if (v2) return gather_nch<TA, 2, GRAD, IDENT>(P, G, ts, sr, st);
  if (G.d > 512) return hipErrorInvalidValue;
  return gather_nch<TA, 1, GRAD, IDENT>(P, G, ts, sr, st);
}

hipError_t launch_sketch_gather(const SketchPlan& P, const GatherArgs& G, hipStream_t st) {
  const bool grad = G.b != nullptr;
  if (G.a_dtype == 0)
    return grad ? gather_vec<double, true, false>(P, G, 0, 0, st)
                : gather_vec<double, false, false>(P, G, 0, 0, st);
  return grad ? gather_vec<float, true, false>(P, G, 0, 0, st)
              : gather_vec<float, false, false>(P, G, 0, 0, st);
}

hipError_t launch_gradient_rows(const ProbInfo* probs, int32_t batch, int32_t total_seg,
                                int32_t seg_rows, const void* A, int32_t a_dtype, int64_t ld,
                                int64_t d, const double* b, const double* x, double* gpart,
                                double* fpart, double* r_out, hipStream_t st) {
  SketchPlan P{};
  P.probs = probs;
  P.batch = batch;
  P.s = 1;
  P.m = 1;
  P.m_blk = 1;
  GatherArgs G{};
  G.A = A;
  G.a_dtype = a_dtype;
  G.ld = ld;
  G.d = d;
  G.scale = 1.0;
  G.b = b;
  G.x = x;
  G.gpart = gpart;
  G.fpart = fpart;
  G.r_out = r_out;
  if (a_dtype == 0) return gather_vec<double, true, true>(P, G, total_seg, seg_rows, st);
  return gather_vec<float, true, true>(P, G, total_seg, seg_rows, st);
}

// ---------------------------------------------------------------------------
// CSR gradient rows in natural order (the gradient pass without a sketch;
// k_gather_csr_bucket below is the sketch's gather). One wavefront per
// segment of rows keeps a dense gradient row in LDS. Nonzeros are staged 64 at a time in
// (row, column) order; lanes holding the same column are ranked with ballots
// and applied round by round, so each column still sums in ascending row
// order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gradient_rows_csr(SketchPlan P, CsrGatherArgs G,
                                                           int32_t col_bits, int32_t total_seg,
                                                           int32_t seg_rows) {
  extern __shared__ double smem[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t d = G.d;
  double* gac = smem + (int64_t)wv * d;
  __shared__ int32_t st_col[4][64];
  __shared__ double st_rv[4][64];
  const int64_t bg = (int64_t)blockIdx.x * 4 + wv;
  if (bg >= (int64_t)total_seg) return;  // no workgroup barriers below
  if (G.halt != nullptr && status_word(G.halt) != 0) return;
  const int p = find_by_seg(P.probs, P.batch, (int)bg);
  const ProbInfo pi = P.probs[p];
  const int64_t beg = pi.row0 + (bg - pi.seg0) * (int64_t)seg_rows;
  const int64_t end = min(beg + seg_rows, pi.row0 + pi.rows);
  for (int64_t c = lane; c < d; c += 64) gac[c] = 0.0;
  const uint64_t lt = lanemask_lt();
  double fa = 0.0;
  for (int64_t base = beg; base < end; base += 64) {
    const bool rv_ok = base + lane < end;
    const int64_t row = base + lane;
    int32_t rs = 0, re = 0;
    if (rv_ok) {
      rs = G.row_ptr[row];
      re = G.row_ptr[row + 1];
    }
    double ri = 0.0;
    if (rv_ok) {
      double dot = 0.0;
      for (int32_t q = rs; q < re; ++q) dot = fma(G.values[q], G.x[(int64_t)p * d + G.col_idx[q]], dot);
      ri = G.b[row] - dot;
      fa = fma(ri, ri, fa);
      if (G.r_out != nullptr) G.r_out[row] = ri;
    }
    // flattened positions of this batch's nonzeros
    const int len = re - rs;
    int incl = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    const int excl = incl - len;
    const int total = __shfl(incl, 63, 64);
    for (int w0 = 0; w0 < total; w0 += 64) {
      // stage the nonzeros whose flattened index falls in [w0, w0 + 64)
      for (int q = max(excl, w0); q < min(excl + len, w0 + 64); ++q) {
        const int32_t src = rs + (q - excl);
        st_col[wv][q - w0] = G.col_idx[src];
        st_rv[wv][q - w0] = ri * G.values[src];
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const bool ok = (w0 + lane) < total;
      const int32_t col = ok ? st_col[wv][lane] : 0;
      const double rvv = ok ? st_rv[wv][lane] : 0.0;
      uint64_t peers = __ballot(ok);
      for (int bit = 0; bit < col_bits; ++bit) {
        const bool on = (col >> bit) & 1;
        const uint64_t bb = __ballot(on);
        peers &= on ? bb : ~bb;
      }
      const int rank = __popcll(peers & lt);
      for (int r = 0; __ballot(ok && rank >= r) != 0ull; ++r) {
        if (ok && rank == r) gac[col] = gac[col] + rvv;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
  double* gp = G.gpart + bg * d;
  for (int64_t c = lane; c < d; c += 64) gp[c] = gac[c];
  const double fs = wave_sum(fa);
  if (lane == 0) G.fpart[bg] = fs;
}

// ---------------------------------------------------------------------------
// CSR bucket gather. One wavefront per sketch row keeps a dense row of S A
// (and of the gradient partial) in LDS and walks the sketch row's sorted rows
// 64 at a time. The walk is software-pipelined: the sorted-row entries are
// requested two batches ahead and the rows' extents (and b) one batch ahead,
// so a batch waits only for its own nonzeros. Nonzeros are staged 64 at a
// time in (row, column) order; lanes holding the same column are ranked with
// ballots and applied round by round, so each (sketch row, column) still sums
// in ascending row order.
// ---------------------------------------------------------------------------
template <bool GRAD>
__global__ __launch_bounds__(256) void k_gather_csr_bucket(SketchPlan P, CsrGatherArgs G,
                                                           int32_t col_bits) {
  extern __shared__ double smem[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t d = G.d;
  double* acc = smem + (int64_t)wv * (GRAD ? 2 : 1) * d;
  double* gac = acc + d;
  __shared__ int32_t st_col[4][64];
  __shared__ double st_val[4][64];
  __shared__ double st_rv[4][64];
  const int64_t nbk = (int64_t)P.batch * P.m;
  const int64_t bg = (int64_t)blockIdx.x * 4 + wv;
  if (bg >= nbk) return;  // no workgroup barriers below: waves are independent
  if (G.halt != nullptr && status_word(G.halt) != 0) return;
  const int p = (int)(bg / P.m);
  const int64_t bl = bg - (int64_t)p * P.m;
  const int64_t beg = P.bucket_start[bg], end = P.bucket_start[bg + 1];
  const int64_t gslot = (int64_t)p * P.m_blk + bl;
  const bool grad = GRAD && (bl < P.m_blk);
  for (int64_t c = lane; c < d; c += 64) {
    acc[c] = 0.0;
    if (GRAD) gac[c] = 0.0;
  }
  const uint64_t lt = lanemask_lt();
  const double* xp = G.x + (int64_t)p * d;
  auto perm_at = [&](int64_t base) -> uint32_t {
    return base + lane < end ? P.perm[base + lane] : 0u;
  };
  // the current batch's entry and extent, the next batch's entry
  uint32_t pe = perm_at(beg), pe_n = perm_at(beg + 64);
  int32_t rs = 0, re = 0;
  double bi = 0.0;
  if (beg + lane < end) {
    const uint32_t row = pe & 0x7FFFFFFFu;
    rs = G.row_ptr[row];
    re = G.row_ptr[row + 1];
    if (grad) bi = G.b[row];
  }
  double fa = 0.0;
  for (int64_t base = beg; base < end; base += 64) {
    const bool rv_ok = base + lane < end;
    // requests for the next two batches
    const uint32_t pe_nn = perm_at(base + 128);
    int32_t rs_n = 0, re_n = 0;
    double bi_n = 0.0;
    if (base + 64 + lane < end) {
      const uint32_t row_n = pe_n & 0x7FFFFFFFu;
      rs_n = G.row_ptr[row_n];
      re_n = G.row_ptr[row_n + 1];
      if (grad) bi_n = G.b[row_n];
    }
    const uint32_t row = pe & 0x7FFFFFFFu;
    const double sg = (pe >> 31) ? -1.0 : 1.0;
    double ri = 0.0;
    if (grad && rv_ok) {
      double dot = 0.0;
      for (int32_t q = rs; q < re; ++q) dot = fma(G.values[q], xp[G.col_idx[q]], dot);
      ri = bi - dot;
      fa = fma(ri, ri, fa);
      if (G.r_out != nullptr) G.r_out[row] = ri;
    }
    // flattened positions of this batch's nonzeros
    const int len = re - rs;
    int incl = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    const int excl = incl - len;
    const int total = __shfl(incl, 63, 64);
    for (int w0 = 0; w0 < total; w0 += 64) {
      // stage the nonzeros whose flattened index falls in [w0, w0 + 64)
      for (int q = max(excl, w0); q < min(excl + len, w0 + 64); ++q) {
        const int32_t src = rs + (q - excl);
        st_col[wv][q - w0] = G.col_idx[src];
        const double v = G.values[src];
        st_val[wv][q - w0] = sg * v;
        st_rv[wv][q - w0] = ri * v;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const bool ok = (w0 + lane) < total;
      const int32_t col = ok ? st_col[wv][lane] : 0;
      const double v = ok ? st_val[wv][lane] : 0.0;
      const double rvv = ok ? st_rv[wv][lane] : 0.0;
      uint64_t peers = __ballot(ok);
      for (int bit = 0; bit < col_bits; ++bit) {
        const bool on = (col >> bit) & 1;
        const uint64_t bb = __ballot(on);
        peers &= on ? bb : ~bb;
      }
      const int rank = __popcll(peers & lt);
      for (int r = 0; __ballot(ok && rank >= r) != 0ull; ++r) {
        if (ok && rank == r) {
          acc[col] = acc[col] + v;
          if (grad) gac[col] = gac[col] + rvv;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    pe = pe_n;
    pe_n = pe_nn;
    rs = rs_n;
    re = re_n;
    bi = bi_n;
  }
  const int64_t orow = bg * G.ld_sa;
  for (int64_t c = lane; c < d; c += 64) store_sa(G.SA, G.sa_dtype, orow + c, acc[c] * G.scale);
  if (grad) {
    double* gp = G.gpart + gslot * d;
    for (int64_t c = lane; c < d; c += 64) gp[c] = gac[c];
    const double fs = wave_sum(fa);
    if (lane == 0) G.fpart[gslot] = fs;
  }
}

static int32_t bits_for(int64_t d) {
  int32_t bits = 0;
  while ((1ll << bits) < d) ++bits;
  return bits;
}

hipError_t launch_sketch_gather_csr(const SketchPlan& P, const CsrGatherArgs& G,
                                    hipStream_t st) {
  const int64_t nbk = (int64_t)P.batch * P.m;
  const unsigned blocks = (unsigned)((nbk + 3) / 4);
  const bool grad = G.b != nullptr;
  const size_t lds = (size_t)4 * (grad ? 2 : 1) * G.d * sizeof(double);
  if (grad)
    hipLaunchKernelGGL(k_gather_csr_bucket<true>, dim3(blocks), dim3(256), lds, st, P, G,
                       bits_for(G.d));
  else
    hipLaunchKernelGGL(k_gather_csr_bucket<false>, dim3(blocks), dim3(256), lds, st, P, G,
                       bits_for(G.d));
  return hipGetLastError();
}

hipError_t launch_gradient_rows_csr(const ProbInfo* probs, int32_t batch, int32_t total_seg,
                                    int32_t seg_rows, const int32_t* row_ptr,
                                    const int32_t* col_idx, const double* values, int64_t d,
                                    const double* b, const double* x, double* gpart,
                                    double* fpart, double* r_out, hipStream_t st) {
  if (total_seg == 0) return hipSuccess;
  SketchPlan P{};
  P.probs = probs;
  P.batch = batch;
  P.s = 1;
  P.m = 1;
  P.m_blk = 1;
  CsrGatherArgs G{};
  G.row_ptr = row_ptr;
  G.col_idx = col_idx;
  G.values = values;
  G.d = d;
  G.scale = 1.0;
  G.b = b;
  G.x = x;
  G.gpart = gpart;
  G.fpart = fpart;
  G.r_out = r_out;
  const size_t lds = (size_t)4 * d * sizeof(double);
  hipLaunchKernelGGL(k_gradient_rows_csr, dim3((unsigned)((total_seg + 3) / 4)), dim3(256), lds,
                     st, P, G, bits_for(d), total_seg, seg_rows);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint S^T G over the rows of up to kAdjointBatch problems in one launch:
// row i of problem p re-derives its s (bucket, sign) pairs from the hash and
// receives the sum over blocks, ascending from +0.0, of sign * (c_s * G row).
// Each wave takes 64 consecutive rows; lane l hashes row l of the group, so a
// Philox block is computed once per (row, block pair) rather than once per
// lane. The keys and each row's problem go through LDS; the wave then walks
// its rows kAdjU at a time, lanes over columns, so that every lane has kAdjU
// independent G loads in flight before its stores.
// ---------------------------------------------------------------------------
constexpr int kAdjU = 8;

__global__ __launch_bounds__(256) void k_adjoint(AdjointBatch ab, int32_t s, int64_t m,
                                                 int64_t m_blk, uint64_t seed, uint64_t iter,
                                                 const double* __restrict__ Gm, int64_t ld_g,
                                                 int64_t d, double* __restrict__ out,
                                                 int64_t ld_out, double scale) {
  __shared__ int64_t off[kAdjointBatch + 1];
  __shared__ uint32_t keys[4][16][64];  // [wave][block][row of the group]
  __shared__ int32_t prob[4][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i <= kAdjointBatch; ++i) off[i] = ab.off[i];
  }
  __syncthreads();
  const int count = ab.count;
  const int64_t row0 = off[0], row_end = off[count];
  const int64_t groups = (row_end - row0 + 63) / 64;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t gi = (int64_t)blockIdx.x * 4 + wv; gi < groups; gi += waves) {
    const int64_t base = row0 + gi * 64;
    const int64_t row = base + lane;
    // problem of this lane's row: the last p with off[p] <= row
    int lo = 0, hi = count;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= row) lo = mid;
      else hi = mid;
    }
    const uint64_t local = (uint64_t)(row - off[lo]);
    if (row < row_end) {
      for (int q = 0; q < (s + 1) / 2; ++q) {
        const U64x4 w = philox4x64_10(local, (uint64_t)q, (uint64_t)(ab.first + lo), 0ull,
                                      seed, iter);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = 2 * q + h;
          if (k < s)
            keys[wv][k][lane] =
                ((uint32_t)(k * m_blk) + range_reduce(w.w[2 * h], (uint64_t)m_blk)) |
                ((uint32_t)(w.w[2 * h + 1] >> 63) << 31);
        }
      }
    }
    prob[wv][lane] = lo;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int nr = (int)((row_end - base) < 64 ? (row_end - base) : 64);
    for (int r0 = 0; r0 < nr; r0 += kAdjU) {
      int64_t gbase[kAdjU];
#pragma unroll
      for (int j = 0; j < kAdjU; ++j) gbase[j] = (int64_t)prob[wv][r0 + j < 64 ? r0 + j : 63] * m;
      for (int64_t c = lane; c < d; c += 64) {
        double acc[kAdjU];
#pragma unroll
        for (int j = 0; j < kAdjU; ++j) acc[j] = 0.0;
        for (int k = 0; k < s; ++k) {
          double t[kAdjU];
#pragma unroll
          for (int j = 0; j < kAdjU; ++j) {
            const uint32_t key = keys[wv][k][r0 + j < 64 ? r0 + j : 63];
            t[j] = (r0 + j < nr) ? Gm[(gbase[j] + (int64_t)(key & 0x7FFFFFFFu)) * ld_g + c] : 0.0;
          }
#pragma unroll
          for (int j = 0; j < kAdjU; ++j) {
            const uint32_t key = keys[wv][k][r0 + j < 64 ? r0 + j : 63];
            const double v = s > 1 ? t[j] * scale : t[j];
            acc[j] = (key >> 31) ? (acc[j] - v) : (acc[j] + v);
          }
        }
#pragma unroll
        for (int j = 0; j < kAdjU; ++j)
          if (r0 + j < nr) out[(base + r0 + j) * ld_out + c] = acc[j];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

hipError_t launch_sketch_adjoint(const AdjointBatch& ab, int32_t s, int64_t m, uint64_t seed,
                                 uint64_t iter, const double* G, int64_t ld_g, int64_t d,
                                 double* out, int64_t ld_out, hipStream_t st) {
  if (ab.count < 1 || ab.count > kAdjointBatch || s < 1 || s > 16) return hipErrorInvalidValue;
  const int64_t rows = ab.off[ab.count] - ab.off[0];
  if (rows == 0) return hipSuccess;
  const double scale = 1.0 / sqrt((double)s);
  const int64_t groups = (rows + 63) / 64;
  const unsigned blocks = (unsigned)std::min<int64_t>((groups + 3) / 4, 16384);
  hipLaunchKernelGGL(k_adjoint, dim3(blocks), dim3(256), 0, st, ab, s, m, m / s, seed, iter, G,
                     ld_g, d, out, ld_out, scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dL/db = A lambda and dL/dA = r lambda^T - (A lambda) x^T, r = b - A x, for
// the rows of up to kAdjointBatch problems in one launch (global row indices;
// each row finds its problem in the offsets staged in LDS). One wavefront
// per row.
// ---------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(256) void k_solution_grads(AdjointBatch ab, int64_t d,
                                                        const TA* __restrict__ A, int64_t ld,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ lam,
                                                        double* dl_db, double* dl_da,
                                                        int64_t ld_da) {
  __shared__ int64_t off[kAdjointBatch + 1];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i <= kAdjointBatch; ++i) off[i] = ab.off[i];
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int count = ab.count;
  const int64_t row_end = off[count];
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t row = off[0] + (int64_t)blockIdx.x * 4 + wv; row < row_end; row += waves) {
    int lo = 0, hi = count;  // the last problem whose rows start at or before `row`
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= row) lo = mid;
      else hi = mid;
    }
    const int64_t pq = (int64_t)ab.first + lo;
    const double* xp = x + pq * d;
    const double* lp = lam + pq * d;
    const TA* ar = A + row * ld;
    double sl = 0.0, sx = 0.0;
    for (int64_t c = lane; c < d; c += 64) {
      const double a = (double)ar[c];
      sl = fma(a, lp[c], sl);
      sx = fma(a, xp[c], sx);
    }
    sl = wave_sum(sl);
    sx = wave_sum(sx);
    const double r = b[row] - sx;
    if (dl_db != nullptr && lane == 0) dl_db[row] = sl;
    if (dl_da != nullptr)
      for (int64_t c = lane; c < d; c += 64) dl_da[row * ld_da + c] = r * lp[c] - sl * xp[c];
  }
}

hipError_t launch_solution_grads(const AdjointBatch& ab, int64_t d, const void* A, bool a_f32,
                                 int64_t ld, const double* b, const double* x,
                                 const double* lambda, double* dl_db, double* dl_da,
                                 int64_t ld_da, hipStream_t st) {
  if (ab.count < 1 || ab.count > kAdjointBatch) return hipErrorInvalidValue;
  const int64_t rows = ab.off[ab.count] - ab.off[0];
  if (rows == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((rows + 3) / 4, 65536);
  if (a_f32)
    hipLaunchKernelGGL(k_solution_grads<float>, dim3(blocks), dim3(256), 0, st, ab, d,
                       static_cast<const float*>(A), ld, b, x, lambda, dl_db, dl_da, ld_da);
  else
    hipLaunchKernelGGL(k_solution_grads<double>, dim3(blocks), dim3(256), 0, st, ab, d,
                       static_cast<const double*>(A), ld, b, x, lambda, dl_db, dl_da, ld_da);
  return hipGetLastError();
}

}  // namespace ihs
