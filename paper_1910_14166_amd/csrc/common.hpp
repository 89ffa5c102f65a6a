// Device helpers shared by the libihs kernels (gfx950, wave64).
#pragma once

#include <cstddef>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ihs {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128 products
// with the key advanced by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct U64x4 {
  uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
  const uint64_t kMul1 = 0xCA5A826395121157ull;
  const uint64_t kInc0 = 0x9E3779B97F4A7C15ull;
  const uint64_t kInc1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kInc0;
      k1 += kInc1;
    }
    const uint64_t lo_a = kMul0 * c0, hi_a = __umul64hi(kMul0, c0);
    const uint64_t lo_b = kMul1 * c2, hi_b = __umul64hi(kMul1, c2);
    const uint64_t n0 = hi_b ^ c1 ^ k0;
    const uint64_t n2 = hi_a ^ c3 ^ k1;
    c0 = n0;
    c1 = lo_b;
    c2 = n2;
    c3 = lo_a;
  }
  U64x4 out;
  out.w[0] = c0;
  out.w[1] = c1;
  out.w[2] = c2;
  out.w[3] = c3;
  return out;
}

// Sketch row within a block of `m_blk` rows: floor(w * m_blk / 2^64).
__device__ __forceinline__ uint32_t range_reduce(uint64_t w, uint64_t m_blk) {
  return (uint32_t)__umul64hi(w, m_blk);
}

// ---------------------------------------------------------------------------
// Rounding float64 -> bfloat16 (nearest, ties to even) in one step.
// Returns the bfloat16 bit pattern. Normal-range values; NaN stays NaN.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f64_to_bf16_bits(double v) {
  uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t exp_all = 0x7FF0000000000000ull;
  if ((u & exp_all) == exp_all) {  // Inf or NaN
    float f = (float)v;
    uint32_t fb = __float_as_uint(f);
    if ((u & 0x000FFFFFFFFFFFFFull) != 0) fb |= 0x00400000u;  // keep NaN quiet
    return (uint16_t)(fb >> 16);
  }
  const int drop = 52 - 7;
  const uint64_t lsb = (u >> drop) & 1ull;
  u += ((1ull << (drop - 1)) - 1ull) + lsb;
  u &= ~((1ull << drop) - 1ull);
  const float f = (float)__longlong_as_double((long long)u);  // exact
  return (uint16_t)(__float_as_uint(f) >> 16);
}

__device__ __forceinline__ double bf16_bits_to_f64(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Device status block written by kernels that can fail numerically.
struct DeviceStatus {
  int32_t code;          // ihs_status, 0 while healthy
  int32_t failed_iter;
  int32_t failed_problem;
  int32_t done;          // early-stop flag of the outer loop
  int32_t iters;         // steps whose update was applied
  int32_t claim;         // first failure wins the claim, then publishes
  int32_t unpolished;    // l1 QPs that ended on a converged first-order iterate
                         // which the KKT polish did not certify
  int32_t pad;
  double objective;      // 1/2 ||A x - b||^2 of problem 0 at the last pass
  double last_step;      // sqrt(dx^T H dx) of problem 0 at the last step
};

static_assert(sizeof(DeviceStatus) == 48 && offsetof(DeviceStatus, done) == 12,
              "the host reads code .. done as four leading words");

// The first failing thread claims the record, writes where it failed, and
// only then publishes the code, so a reader that sees a non-zero code (from
// any stream) also sees the step and problem it belongs to.
__device__ __forceinline__ void status_fail(DeviceStatus* st, int code, int iter,
                                            int problem) {
  if (atomicCAS(&st->claim, 0, 1) == 0) {
    st->failed_iter = iter;
    st->failed_problem = problem;
    __threadfence();
    atomicExch(&st->code, code);
  }
}

// Status words are read at device (agent) scope: every writer is a kernel on
// this GPU. A system-scope acquire would invalidate the L2 for every reading
// wavefront, which in the d x d row kernels (one wavefront per row) cost more
// than the products themselves.
__device__ __forceinline__ int status_word(const int32_t* w) {
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True when `st` records any failure or the tolerance stop of the outer loop
// (`done`): the update kernels then leave x as it is. Only the words
// themselves are read, so no ordering is needed.
__device__ __forceinline__ bool status_halted(const DeviceStatus* st) {
  return status_word(&st->code) != 0 || status_word(&st->done) != 0;
}

// True when `st` records a failure at or before step `iter` (iter < 0: any).
__device__ __forceinline__ bool status_failed_by(const DeviceStatus* st, int iter) {
  // acquire: the step recorded before the code was published is visible
  const int code = __hip_atomic_load(&st->code, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  if (code == 0) return false;
  if (iter < 0) return true;
  const int fi = status_word(&st->failed_iter);
  return fi <= iter;
}

}  // namespace ihs
