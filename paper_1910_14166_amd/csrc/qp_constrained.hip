// The step of Eq.(2) over the l1 and l2 balls of Eq.(1):
//     minimise 1/2 x^T H x - c^T x  over C,   c = H x^t + g,
// solved to optimality at every outer step (the experiments of Sec. 3 solve
// each sketched subproblem exactly).
//
// Both start from the unconstrained minimiser x^t + H^{-1} g (the regular
// Cholesky kernels) and return it when it already lies in the ball.
//
// l1 ball ||x||_1 <= tau (one 1024-thread workgroup per problem, d <= 1024):
//   accelerated projected gradient (FISTA) with step 1/L, L from power steps
//   raised by backtracking, momentum restart by the gradient-mapping test of
//   O'Donoghue and Candes (2015), and the exact finite projection of
//   Michelot (1986). Once the support and signs stop changing (and at the
//   end), a KKT polish solves the face exactly,
//       H_SS x_S + mu sigma = c_S,   sigma^T x_S = tau,
//   (a Cholesky factor of H_SS in LDS when it fits, conjugate gradients on
//   the two right-hand sides otherwise) and is accepted when it keeps the
//   signs, has mu >= 0 and leaves every off-support |c_j - (H x)_j| <= mu
//   (to 1e-9 max(1, |c|_inf)). An accepted KKT point is the minimiser, which
//   ends the iteration.
// l1 penalty lambda ||x||_1 added to the objective (the penalised LASSO of
// the experiments of Sec. 3): the same kernel with the soft threshold by
// lambda / L as the proximal map in place of the projection, and the polish
// with mu fixed at lambda (H_SS x_S = c_S - lambda sigma); a rejected
// polish of the warm start's face is followed by a few primal-dual
// active-set corrections before FISTA. An empty support is the answer when
// every |c_j| <= lambda. No unconstrained solve first.
// l2 ball ||x||_2 <= r:
//   Newton's method on phi(mu) = 1/||x(mu)|| - 1/r, x(mu) = (H + mu I)^{-1} c
//   (More and Sorensen, 1983). 1/||x(mu)|| is concave and increasing, so from
//   mu = 0 the iterates rise monotonically to the root when H is positive
//   definite; phi'(mu) needs x^T (H + mu I)^{-1} x, one more solve with the
//   same factor. The shifts live on the device and each Newton step
//   re-factors H + mu I with per-problem shifts.
#include <algorithm>
#include <vector>

#include "kernels.hpp"
#include "rowdot.hpp"

namespace ihs {

constexpr int kQpThreads = 1024;
constexpr int kQpWaves = kQpThreads / 64;
constexpr int kPolishMax = 256;   // largest support the KKT polish takes on
constexpr int kPolishEvery = 4;   // unchanged iterations before a polish attempt
constexpr int kActiveSetSteps = 4;  // penalty: active-set corrections of a rejected face
constexpr int kPowerSteps = 8;    // power steps for the first Lipschitz estimate
constexpr size_t kQpLdsBytes = 61440;

constexpr int kRed = 8;  // values one fused block reduction carries

constexpr int kColChunk = 256;  // columns per pass of the symmetric product
constexpr int kRowsPer = 2;     // rows whose loads a wavefront issues together

struct ColPartials {
  double v[kQpWaves][kColChunk];
};

struct BlockShared {
  ColPartials part;
  double red[kQpWaves];
  double redv[kQpWaves][kRed];
  int flag[4];
  int wave_count[kQpWaves];
};

// Block-wide sum (resp. max) of one double per thread; every thread gets it.
__device__ __forceinline__ double block_sum(double v, BlockShared& sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh.red[wv] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kQpWaves; ++w) s += sh.red[w];
  return s;
}

__device__ __forceinline__ double block_max(double v, BlockShared& sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) sh.red[wv] = v;
  __syncthreads();
  double s = sh.red[0];
#pragma unroll
  for (int w = 1; w < kQpWaves; ++w) s = fmax(s, sh.red[w]);
  return s;
}

// Fused block reduction: the first NS entries of v are summed, the next NM
// maximised; one barrier pair for all of them. Results replace v.
template <int NS, int NM>
__device__ __forceinline__ void block_reduce(double (&v)[NS + NM], BlockShared& sh) {
  static_assert(NS + NM <= kRed, "too many values");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NS + NM; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v[q], off, 64);
      v[q] = q < NS ? v[q] + o : fmax(v[q], o);
    }
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NS + NM; ++q) sh.redv[wv][q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS + NM; ++q) {
    double s = sh.redv[0][q];
    for (int w = 1; w < kQpWaves; ++w) s = q < NS ? s + sh.redv[w][q] : fmax(s, sh.redv[w][q]);
    v[q] = s;
  }
}

// out = H v for the symmetric H, v and out in LDS, formed by columns:
// (H v)_j = sum_i v_i H[i][j]. Each lane of wavefront w accumulates four
// columns of a 256-column chunk over the row pairs 2w, 2w + 1, 2w + 32,
// 2w + 33, ..., kRowsPer rows' loads at a time (rows read coalesced, no
// cross-lane reduction); the 16 wavefronts' partial sums are then added
// through LDS in a fixed order. (Two rows at a time measured 6% faster than
// four at d = 256, one row the same as two, eight rows 60% slower: the
// kernel's registers are full.)
// Ends with a barrier.
template <int NV>
__device__ __forceinline__ void sym_products(const double* __restrict__ H, int64_t d,
                                             const double* const (&v)[NV], double* const (&out)[NV],
                                             ColPartials& part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // Even d and H 16-byte aligned: every row is 16-byte aligned, and lane l
  // takes the column pairs 2l, 2l + 1 and 128 + 2l, 129 + 2l of the chunk
  // (16-byte loads; 15% faster products at d = 256). Otherwise columns
  // l + 64q. Each column's sum runs over the rows in the same order either way.
  const bool pairs = (d & 1) == 0 && (reinterpret_cast<uintptr_t>(H) & 15) == 0;
  auto col = [&](int q) { return pairs ? 2 * lane + 128 * (q >> 1) + (q & 1) : lane + 64 * q; };
  for (int64_t c0 = 0; c0 < d; c0 += kColChunk) {
    double acc[NV][4];
#pragma unroll
    for (int n = 0; n < NV; ++n)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[n][q] = 0.0;
    for (int64_t i0 = (int64_t)wv * kRowsPer; i0 < d; i0 += kQpWaves * kRowsPer) {
      double h[kRowsPer][4];
#pragma unroll
      for (int r = 0; r < kRowsPer; ++r) {
        const int64_t i = i0 + r < d ? i0 + r : d - 1;
        const double* hr = H + i * d + c0;
        if (pairs) {
#pragma unroll
          for (int q2 = 0; q2 < 2; ++q2) {
            const int64_t j = 2 * lane + 128 * q2;
            double2 t = make_double2(0.0, 0.0);
            if (c0 + j < d) t = *reinterpret_cast<const double2*>(hr + j);
            h[r][2 * q2] = t.x;
            h[r][2 * q2 + 1] = t.y;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t j = lane + 64 * q;
            h[r][q] = (c0 + j < d) ? hr[j] : 0.0;
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kRowsPer; ++r)
#pragma unroll
        for (int n = 0; n < NV; ++n) {
          const double vi = i0 + r < d ? v[n][i0 + r] : 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[n][q] = fma(h[r][q], vi, acc[n][q]);
        }
    }
#pragma unroll
    for (int n = 0; n < NV; ++n) {
#pragma unroll
      for (int q = 0; q < 4; ++q) part.v[wv][col(q)] = acc[n][q];
      __syncthreads();
      if (threadIdx.x < kColChunk && c0 + threadIdx.x < d) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kQpWaves; ++w) s += part.v[w][threadIdx.x];
        out[n][c0 + threadIdx.x] = s;
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ void block_rows(const double* __restrict__ H, int64_t d,
                                           const double* v, double* out, BlockShared& sh) {
  const double* const vs[1] = {v};
  double* const os[1] = {out};
  sym_products<1>(H, d, vs, os, sh.part);
}

// Euclidean projection onto {||x||_1 <= tau}, thread i < d holding v_i: when
// ||v||_1 > tau, x_i = sign(v_i) max(|v_i| - theta, 0) with theta from
// Michelot's finite iteration theta = (sum of |v_i| over the active set - tau)
// / |active set|, the active set shrinking to {|v_i| > theta}; it only
// shrinks, so an unchanged count means it is stable.
__device__ double project_l1(double vi, int64_t d, double tau, BlockShared& sh) {
  const int tid = threadIdx.x;
  const double a = tid < d ? fabs(vi) : 0.0;
  bool act = tid < d;
  double r[2] = {act ? 1.0 : 0.0, a};
  block_reduce<2, 0>(r, sh);
  if (r[1] <= tau) return vi;
  double theta = (r[1] - tau) / r[0];
  for (int64_t it = 0; it <= d; ++it) {
    const bool nact = act && a > theta;
    double q[2] = {nact ? 1.0 : 0.0, nact ? a : 0.0};
    block_reduce<2, 0>(q, sh);
    act = nact;
    if (q[0] == r[0]) break;
    r[0] = q[0];
    r[1] = q[1];
    theta = (r[1] - tau) / r[0];
  }
  return (tid < d && a > theta) ? copysign(a - theta, vi) : 0.0;
}

// Outcomes of a KKT polish on a face (support and signs).
constexpr int kPolishAccepted = 0;  // the candidate meets the KKT conditions
constexpr int kPolishRejected = 1;  // a candidate was formed but fails them
constexpr int kPolishNone = 2;      // no candidate (factorisation or solve failed)

// Common end of the polish variants: thread i holds the candidate xs (on the
// support, signs sg) and the multiplier mu. The candidate is accepted when it
// keeps the signs, mu >= 0, and every off-support |c_j - (H x)_j| <= mu (to
// 1e-9 max(1, |c|_inf)). Unless the result is kPolishNone, *xi receives the
// candidate, *gi = c_i - (H x)_i and *mu_out = mu, for an active-set update.
// buf, hbuf: d doubles of LDS.
__device__ int polish_finish(const double* __restrict__ H, int64_t d, double ci, bool on,
                             double sg, double xs, double mu, double* buf, double* hbuf,
                             double cscale, double* xi, double* gi, double* mu_out,
                             BlockShared& sh) {
  const int tid = threadIdx.x;
  if (!(mu >= 0.0) || !isfinite(mu)) return kPolishNone;  // the same value in every thread
  const bool bad = on && (!(copysign(1.0, xs) == sg) || xs == 0.0 || !isfinite(xs));
  if (tid < d) buf[tid] = on ? xs : 0.0;
  __syncthreads();
  block_rows(H, d, buf, hbuf, sh);
  const double g = tid < d ? ci - hbuf[tid] : 0.0;
  double r[2] = {bad ? 1.0 : 0.0, (tid < d && !on) ? fabs(g) - mu : -1.0};
  block_reduce<0, 2>(r, sh);
  *xi = on ? xs : 0.0;
  *gi = g;
  *mu_out = mu;
  return (r[0] == 0.0 && r[1] <= 1e-9 * cscale) ? kPolishAccepted : kPolishRejected;
}

// Cholesky factor of the n x n symmetric positive definite matrix M (row
// major, LDS or global; lower triangle, in place, one column per round).
// False, in every thread, when a pivot is not positive. Ends with a barrier.
__device__ bool lds_cholesky(double* M, int n, BlockShared& sh) {
  const int tid = threadIdx.x;
  if (tid == 0) sh.flag[2] = 1;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double piv = M[j * n + j];
    if (!(piv > 0.0) || !isfinite(piv)) {  // the same value in every thread
      if (tid == 0) sh.flag[2] = 0;
      break;
    }
    const double ljj = sqrt(piv);
    for (int i = j + 1 + tid; i < n; i += kQpThreads) M[i * n + j] /= ljj;
    __syncthreads();
    if (tid == 0) M[j * n + j] = ljj;
    const int rem = n - j - 1;
    for (int e = tid; e < rem * rem; e += kQpThreads) {
      const int i = j + 1 + e / rem, k = j + 1 + (e - (e / rem) * rem);
      if (k <= i) M[i * n + k] = fma(-M[i * n + j], M[k * n + j], M[i * n + k]);
    }
    __syncthreads();
  }
  __syncthreads();
  const bool ok = sh.flag[2] != 0;
  __syncthreads();
  return ok;
}

// z = (L L^T)^{-1} z for the factor L left in M by lds_cholesky (z: n
// doubles of LDS): a forward then a backward sweep. Ends with a barrier.
__device__ void lds_chol_solve(const double* M, int n, double* z) {
  const int tid = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    const double zj = z[j] / M[j * n + j];
    for (int i = j + 1 + tid; i < n; i += kQpThreads) z[i] = fma(-M[i * n + j], zj, z[i]);
    __syncthreads();
    if (tid == 0) z[j] = zj;
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double zj = z[j] / M[j * n + j];
    for (int i = tid; i < j; i += kQpThreads) z[i] = fma(-M[j * n + i], zj, z[i]);
    __syncthreads();
    if (tid == 0) z[j] = zj;
  }
  __syncthreads();
}

// KKT polish on the support of x (thread i holds x_i in *xi). M: ns*ns
// doubles (LDS or global), u, w: kPolishMax doubles, idx: kPolishMax ints,
// cand, hc: d doubles of LDS. Ball (penalty false): mu from sigma^T x_S = tau;
// penalty: mu = tau = lambda. On success returns true with the polished x_i.
__device__ __attribute__((noinline)) int l1_polish(const double* __restrict__ H, int64_t d,
                                                   double ci, double tau, bool penalty,
                                                   double* xi, double* gi, double* mu_out,
                                                   double* M, double* u, double* w, int* idx,
                                                   double* cand, double* hc, double cscale,
                                                   BlockShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool on = tid < d && *xi != 0.0;
  // ascending support indices by wave ballots
  const uint64_t bal = __ballot(on);
  if (lane == 0) sh.wave_count[wv] = __popcll(bal);
  __syncthreads();
  int base = 0, ns = 0;
  for (int k = 0; k < kQpWaves; ++k) {
    if (k < wv) base += sh.wave_count[k];
    ns += sh.wave_count[k];
  }
  if (ns == 0) {  // x = 0: optimal for the penalty when every |c_j| <= lambda
    if (!penalty) return kPolishNone;
    return polish_finish(H, d, ci, false, 0.0, 0.0, tau, cand, hc, cscale, xi, gi, mu_out, sh);
  }
  if (ns > kPolishMax) return kPolishNone;
  const int slot = on ? base + __popcll(bal & lanemask_lt()) : -1;
  if (on) idx[slot] = tid;
  __syncthreads();
  for (int e = tid; e < ns * ns; e += kQpThreads) {
    const int a = e / ns, b = e - (e / ns) * ns;
    M[e] = H[(int64_t)idx[a] * d + idx[b]];
  }
  if (!lds_cholesky(M, ns, sh)) return kPolishNone;
  // u = H_SS^{-1} c_S and w = H_SS^{-1} sigma: forward then backward sweep
  for (int a = tid; a < ns; a += kQpThreads) u[a] = w[a] = 0.0;
  __syncthreads();
  const double sg = on ? copysign(1.0, *xi) : 0.0;
  if (on) {
    u[slot] = ci;
    w[slot] = sg;
  }
  __syncthreads();
  for (int j = 0; j < ns; ++j) {
    const double r = 1.0 / M[j * ns + j];
    const double uj = u[j] * r, wj = w[j] * r;
    for (int i = j + 1 + tid; i < ns; i += kQpThreads) {
      const double lij = M[i * ns + j];
      u[i] = fma(-lij, uj, u[i]);
      w[i] = fma(-lij, wj, w[i]);
    }
    __syncthreads();
    if (tid == 0) {
      u[j] = uj;
      w[j] = wj;
    }
  }
  __syncthreads();
  for (int j = ns - 1; j >= 0; --j) {
    const double r = 1.0 / M[j * ns + j];
    const double uj = u[j] * r, wj = w[j] * r;
    for (int i = tid; i < j; i += kQpThreads) {
      const double lji = M[j * ns + i];
      u[i] = fma(-lji, uj, u[i]);
      w[i] = fma(-lji, wj, w[i]);
    }
    __syncthreads();
    if (tid == 0) {
      u[j] = uj;
      w[j] = wj;
    }
  }
  __syncthreads();
  const double SU = block_sum(on ? sg * u[slot] : 0.0, sh);
  const double SW = block_sum(on ? sg * w[slot] : 0.0, sh);
  const double mu = penalty ? tau : (SU - tau) / SW;
  const double xs = on ? u[slot] - mu * w[slot] : 0.0;
  return polish_finish(H, d, ci, on, sg, xs, mu, cand, hc, cscale, xi, gi, mu_out, sh);
}

// KKT polish for a support too large to factor in LDS: the reduced systems
// are solved by conjugate gradients instead of a Cholesky factor, with no
// ns x ns storage. Ball: u = H_SS^{-1} c_S and w = H_SS^{-1} sigma_S from 0,
// both right-hand sides advancing through the same sweeps over H; then
// mu = (sigma^T u - tau) / sigma^T w and x_S = u - mu w. Penalty: x_S =
// H_SS^{-1} (c_S - lambda sigma_S) from the current x_S. Each recurrence
// stops once its residual is 1e-15 of its right-hand side (or after max_cg
// sweeps). Acceptance as in l1_polish. pa, pb, qa, qb: d doubles of LDS.
__device__ int l1_polish_cg(const double* __restrict__ H, int64_t d, double ci, double tau,
                            bool penalty, double* xi, double* gi, double* mu_out, double* pa,
                            double* pb, double* qa, double* qb, double cscale, int max_cg,
                            BlockShared& sh) {
  const int tid = threadIdx.x;
  const bool on = tid < d && *xi != 0.0;
  const double sg = on ? copysign(1.0, *xi) : 0.0;
  const double fa = on ? (penalty ? ci - tau * sg : ci) : 0.0;
  const double fb = (on && !penalty) ? sg : 0.0;
  double a = (penalty && on) ? *xi : 0.0, b = 0.0;
  double ra = fa, rb = fb;
  if (penalty) {  // residual of the warm start
    if (tid < d) pa[tid] = a;
    __syncthreads();
    block_rows(H, d, pa, qa, sh);
    ra = on ? fa - qa[tid] : 0.0;
  }
  double n0[4] = {ra * ra, rb * rb, fa * fa, fb * fb};
  block_reduce<4, 0>(n0, sh);
  double rra = n0[0], rrb = n0[1];
  const double tola = 1e-30 * n0[2], tolb = 1e-30 * n0[3];
  double qA = ra, qB = rb;  // search directions
  for (int k = 0; k < max_cg && (rra > tola || rrb > tolb); ++k) {
    if (tid < d) {
      pa[tid] = qA;
      pb[tid] = qB;
    }
    __syncthreads();
    {
      const double* const vs[2] = {pa, pb};
      double* const os[2] = {qa, qb};
      sym_products<2>(H, d, vs, os, sh.part);
    }
    const double ha = on ? qa[tid] : 0.0, hb = on ? qb[tid] : 0.0;
    double cv[2] = {qA * ha, qB * hb};
    block_reduce<2, 0>(cv, sh);
    const double al_a = (rra > tola && cv[0] > 0.0) ? rra / cv[0] : 0.0;
    const double al_b = (rrb > tolb && cv[1] > 0.0) ? rrb / cv[1] : 0.0;
    a = fma(al_a, qA, a);
    b = fma(al_b, qB, b);
    ra = fma(-al_a, ha, ra);
    rb = fma(-al_b, hb, rb);
    double nn[2] = {ra * ra, rb * rb};
    block_reduce<2, 0>(nn, sh);
    if (!(cv[0] > 0.0) && rra > tola) break;  // H_SS not positive definite
    if (!(cv[1] > 0.0) && rrb > tolb) break;
    const double be_a = rra > 0.0 ? nn[0] / rra : 0.0;
    const double be_b = rrb > 0.0 ? nn[1] / rrb : 0.0;
    qA = ra + be_a * qA;
    qB = rb + be_b * qB;
    rra = nn[0];
    rrb = nn[1];
  }
  if (rra > tola || rrb > tolb || !isfinite(rra) || !isfinite(rrb)) return kPolishNone;
  double mu = tau;
  if (!penalty) {
    double sw[2] = {sg * a, sg * b};
    block_reduce<2, 0>(sw, sh);
    mu = (sw[0] - tau) / sw[1];
  }
  const double xs = on ? (penalty ? a : a - mu * b) : 0.0;
  return polish_finish(H, d, ci, on, sg, xs, mu, pa, qa, cscale, xi, gi, mu_out, sh);
}

// y_S = (H_SS)^{-1} f_S through G = H^{-1}, thread i holding f_i (zero off
// the support S): with N the complement of S, the inverse of the block H_SS
// is the Schur complement G_SS - G_SN G_NN^{-1} G_NS of G_NN in G, so
// y_S = (G f)_S - (G z)_S with z = G_NN^{-1} (G f)_N. M holds the factor of
// G_NN (lds_cholesky), slot the thread's position in N (-1 on S), z nn
// doubles of LDS, vec and hv d doubles of LDS. Zero off S.
__device__ double inv_face_solve(const double* __restrict__ G, int64_t d, double f, bool on,
                                 int slot, int nn, const double* M, double* z, double* vec,
                                 double* hv, BlockShared& sh) {
  const int tid = threadIdx.x;
  if (tid < d) vec[tid] = f;
  __syncthreads();
  block_rows(G, d, vec, hv, sh);
  const double y = tid < d ? hv[tid] : 0.0;
  if (nn == 0) return on ? y : 0.0;
  if (slot >= 0) z[slot] = y;
  __syncthreads();
  lds_chol_solve(M, nn, z);
  if (tid < d) vec[tid] = slot >= 0 ? z[slot] : 0.0;
  __syncthreads();
  block_rows(G, d, vec, hv, sh);
  return on ? y - hv[tid] : 0.0;
}

// KKT polish through the explicit inverse G = H^{-1}, for a support whose
// complement N is the smaller set: each face solve is two products with G
// and a solve with the |N| x |N| block G_NN (inv_face_solve), followed by one
// step of iterative refinement whose residual is formed with H itself. Ball:
// u = H_SS^{-1} c_S and w = H_SS^{-1} sigma_S, mu = (sigma^T u - tau) /
// sigma^T w, x_S = u - mu w; penalty: x_S = H_SS^{-1} (c_S - lambda sigma_S).
// Acceptance as in l1_polish. M: nn*nn doubles, z: kPolishMax doubles, idx:
// kPolishMax ints, vec, hv, cand: d doubles, all LDS.
__device__ __attribute__((noinline)) int l1_polish_inverse(
    const double* __restrict__ H, const double* __restrict__ G, int64_t d, double ci, double tau,
    bool penalty, double* xi, double* gi, double* mu_out, double* M, double* z, int* idx,
    double* vec, double* hv, double* cand, double cscale, BlockShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool on = tid < d && *xi != 0.0;
  const bool off = tid < d && !on;
  // ascending complement indices by wave ballots
  const uint64_t bal = __ballot(off);
  if (lane == 0) sh.wave_count[wv] = __popcll(bal);
  __syncthreads();
  int base = 0, nn = 0;
  for (int k = 0; k < kQpWaves; ++k) {
    if (k < wv) base += sh.wave_count[k];
    nn += sh.wave_count[k];
  }
  __syncthreads();
  if (nn > kPolishMax) return kPolishNone;
  const int slot = off ? base + __popcll(bal & lanemask_lt()) : -1;
  if (off) idx[slot] = tid;
  __syncthreads();
  for (int e = tid; e < nn * nn; e += kQpThreads) {
    const int a = e / nn, b = e - (e / nn) * nn;
    M[e] = G[(int64_t)idx[a] * d + idx[b]];
  }
  __syncthreads();
  if (!lds_cholesky(M, nn, sh)) return kPolishNone;
  const double sg = on ? copysign(1.0, *xi) : 0.0;
  // one face solve and one refinement step: y += H_SS^{-1} (f - H_SS y)_S
  auto solve = [&](double f) {
    double y = inv_face_solve(G, d, f, on, slot, nn, M, z, vec, hv, sh);
    if (tid < d) vec[tid] = y;
    __syncthreads();
    block_rows(H, d, vec, hv, sh);
    const double r = on ? f - hv[tid] : 0.0;
    return y + inv_face_solve(G, d, r, on, slot, nn, M, z, vec, hv, sh);
  };
  double xs, mu;
  if (penalty) {
    mu = tau;
    xs = solve(on ? ci - tau * sg : 0.0);
  } else {
    const double u = solve(on ? ci : 0.0);
    const double w = solve(sg);
    double sw[2] = {sg * u, sg * w};
    block_reduce<2, 0>(sw, sh);
    mu = (sw[0] - tau) / sw[1];
    xs = on ? u - mu * w : 0.0;
  }
  return polish_finish(H, d, ci, on, sg, xs, mu, cand, hv, cscale, xi, gi, mu_out, sh);
}

// The polish on the face of *xi (its support and signs): through G = H^{-1}
// (nullable) when the complement of the support is the smaller set and its
// block of G fits in LDS; otherwise factored in LDS when the support is small
// enough, by conjugate gradients beyond (kPolishNone instead unless allow_cg).
struct PolishLds {
  double* vec;
  double* cand;
  double* hv;
  double* u;
  double* w;
  double* M;
  int* idx;
  int32_t mcap;  // doubles of M
};

__device__ int polish_face(const double* __restrict__ H, const double* __restrict__ G, int64_t d,
                           double ci, double tau, bool penalty, double* xi, double* gi,
                           double* mu_out, const PolishLds& L, double cscale, bool allow_cg,
                           BlockShared& sh) {
  double nz[1] = {*xi != 0.0 ? 1.0 : 0.0};
  block_reduce<1, 0>(nz, sh);
  const int64_t nsz = (int64_t)nz[0], ncz = d - nsz;
  if (G != nullptr && ncz < nsz && ncz <= kPolishMax && ncz * ncz <= L.mcap)
    return l1_polish_inverse(H, G, d, ci, tau, penalty, xi, gi, mu_out, L.M, L.u, L.idx, L.vec,
                             L.hv, L.cand, cscale, sh);
  if (nsz * nsz <= L.mcap)
    return l1_polish(H, d, ci, tau, penalty, xi, gi, mu_out, L.M, L.u, L.w, L.idx, L.cand, L.hv,
                     cscale, sh);
  if (!allow_cg) return kPolishNone;
  return l1_polish_cg(H, d, ci, tau, penalty, xi, gi, mu_out, L.vec, L.cand, L.hv, L.M, cscale,
                      (int)(2 * nsz + 40), sh);
}

// One workgroup per problem. xunc: the unconstrained minimiser. Ginv_all
// (nullable): H^{-1} per problem for the polish, unused when gst records a
// failure at or before this step (gst nullable). The polish factors H_SS in
// LDS when it fits and runs conjugate gradients otherwise.
//
// The Lipschitz constant L of the gradient starts at 1.05 x the Rayleigh
// quotient of kPowerSteps power steps and is raised by backtracking (Beck and
// Teboulle, 2009): for this quadratic the sufficient-decrease test reads
// (x+ - y)^T H (x+ - y) <= L ||x+ - y||^2. The kernel forms H x+ once per
// iteration and gets H y by linearity, y = x+ + beta (x+ - x).
__global__ __launch_bounds__(kQpThreads) void k_qp_l1(
    const double* __restrict__ Hall, const double* __restrict__ call,
    const double* __restrict__ xunc_all, const double* x0_all, double* xout_all,
    const double* __restrict__ Ginv_all, const DeviceStatus* gst, int64_t d, double tau,
    int32_t penalty, int32_t max_iter, double tol, int32_t lds_mcap, DeviceStatus* st,
    int32_t iter) {
  extern __shared__ double lds[];
  double* vec = lds;            // d: the vector being multiplied
  double* cand = vec + d;       // d: polish candidate
  double* hv = cand + d;        // d: products
  double* u = hv + d;           // kPolishMax
  double* w = u + kPolishMax;   // kPolishMax
  double* Mlds = w + kPolishMax;
  __shared__ int idx[kPolishMax];
  __shared__ BlockShared sh;
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid == 0) {
    sh.flag[0] = status_halted(st) ? 1 : 0;
    sh.flag[1] = (Ginv_all != nullptr && (gst == nullptr || !status_failed_by(gst, iter))) ? 1 : 0;
  }
  __syncthreads();
  const double* H = Hall + (int64_t)p * d * d;
  const double* G = sh.flag[1] != 0 ? Ginv_all + (int64_t)p * d * d : nullptr;
  double* xout = xout_all + (int64_t)p * d;
  const double x0 = tid < d ? x0_all[(int64_t)p * d + tid] : 0.0;
  if (sh.flag[0] != 0) {  // an earlier failure or the tolerance stop: keep x^t
    if (tid < d) xout[tid] = x0;
    return;
  }
  const double ci = tid < d ? call[(int64_t)p * d + tid] : 0.0;
  const double xu = (!penalty && tid < d) ? xunc_all[(int64_t)p * d + tid] : 0.0;
  double r0[2] = {fabs(xu), 0.0};
  r0[1] = fabs(ci);
  block_reduce<1, 1>(r0, sh);
  if (!penalty && r0[0] <= tau) {  // the ball is inactive
    if (tid < d) xout[tid] = xu;
    return;
  }
  if (penalty && r0[1] <= tau) {  // 0 satisfies the optimality conditions
    if (tid < d) xout[tid] = 0.0;
    return;
  }
  const double cscale = fmax(1.0, r0[1]);
  // The warm start: x^t for the penalty, its projection for the ball. Across
  // IHS steps the support and signs of the solution rarely change once the
  // iterates settle, so the KKT polish is tried on the warm start's face
  // first; an accepted polish is the minimiser and needs no Lipschitz
  // estimate and no iteration. For the penalty a rejected face is followed by
  // up to kActiveSetSteps primal-dual active-set corrections (the semismooth
  // Newton method for this problem): with g = c - H x of the last candidate,
  // the next face keeps j where the coordinate-wise minimiser of the
  // objective, soft(x_j + g_j / H_jj, lambda / H_jj), is non-zero, with its
  // sign, i.e. |H_jj x_j + g_j| > lambda. They stop when the face repeats.
  // (For the ball the same corrections were measured: the faces of its early
  // steps differ too much for them to settle.) For the ball the one other
  // face tried is that of the projected unconstrained minimiser. FISTA then
  // starts from the warm start. One call site of the polish keeps the
  // kernel's registers for FISTA.
  const PolishLds pl{vec, cand, hv, u, w, Mlds, idx, lds_mcap};
  const double xw = penalty ? x0 : project_l1(x0, d, tau, sh);
  {
    const double hjj = (penalty && tid < d) ? H[(int64_t)tid * d + tid] : 0.0;
    double xp = xw, gp = 0.0, mup = 0.0;
    double face = (tid < d && xw != 0.0) ? copysign(1.0, xw) : 0.0;
    for (int k = 0;; ++k) {  // every exit below follows block-wide values
      // the ball's second face is a guess: not worth conjugate gradients
      const int res = polish_face(H, G, d, ci, tau, penalty != 0, &xp, &gp, &mup, pl, cscale,
                                  penalty != 0 || k == 0, sh);
      if (res == kPolishAccepted) {
        if (tid < d) xout[tid] = xp;
        return;
      }
      if (!penalty) {
        if (k > 0) break;
        xp = project_l1(xu, d, tau, sh);
        continue;
      }
      if (res != kPolishRejected || k == kActiveSetSteps) break;
      const double v = fma(hjj, xp, gp);
      const double next = (tid < d && fabs(v) > tau) ? copysign(1.0, v) : 0.0;
      double moved[1] = {next != face ? 1.0 : 0.0};
      block_reduce<0, 1>(moved, sh);
      if (moved[0] == 0.0) break;
      face = next;
      xp = next;  // polish_face reads the face from the signs of xp
    }
  }
  // power steps for the initial Lipschitz estimate
  double pv = tid < d ? 1.0 + 0.25 * (double)((tid * 7) % 5) : 0.0;
  double rq = 0.0;
  for (int k = 0; k < kPowerSteps; ++k) {
    if (tid < d) vec[tid] = pv;
    __syncthreads();
    block_rows(H, d, vec, hv, sh);
    const double hp = tid < d ? hv[tid] : 0.0;
    double q[3] = {pv * hp, hp * hp, pv * pv};
    block_reduce<3, 0>(q, sh);
    rq = q[0] / q[2];
    pv = hp / sqrt(fmax(q[1], 1e-300));
  }
  double Lip = 1.05 * rq;
  // FISTA from the warm start; thread i keeps x_i, (Hx)_i, y_i, (Hy)_i
  double xi = xw;
  if (tid < d) vec[tid] = xi;
  __syncthreads();
  block_rows(H, d, vec, hv, sh);
  double hxi = tid < d ? hv[tid] : 0.0;
  double yi = xi, hyi = hxi;
  double tk = 1.0;
  double sig_prev = -1.0;
  int stable = 0;
  bool done = false;
  bool polished = false;
  for (int it = 0; it < max_iter && !done; ++it) {
    const double vi = tid < d ? yi - (hyi - ci) / Lip : 0.0;
    const double xn = penalty ? copysign(fmax(fabs(vi) - tau / Lip, 0.0), vi)
                              : project_l1(vi, d, tau, sh);
    if (tid < d) vec[tid] = xn;
    __syncthreads();
    block_rows(H, d, vec, hv, sh);
    const double hxn = tid < d ? hv[tid] : 0.0;
    const double e = xn - yi;
    // sums: curvature, |e|^2, restart test, support signature, support size;
    // maxima: step, |x|
    double red[7] = {e * (hxn - hyi), e * e, (yi - xn) * (xn - xi),
                     xn != 0.0 ? (xn > 0.0 ? 1.0 : -1.0) * (double)(tid + 1) : 0.0,
                     xn != 0.0 ? 1.0 : 0.0, fabs(xn - xi), fabs(xn)};
    block_reduce<5, 2>(red, sh);
    if (red[0] > Lip * red[1] * (1.0 + 1e-12)) {  // L too small: back off
      Lip = 1.25 * fmax(Lip, red[0] / red[1]);
      continue;
    }
    double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
    double beta = (tk - 1.0) / tn;
    if (red[2] > 0.0) {  // the momentum points uphill: restart it
      tn = 1.0;
      beta = 0.0;
    }
    yi = xn + beta * (xn - xi);
    hyi = hxn + beta * (hxn - hxi);
    xi = xn;
    hxi = hxn;
    tk = tn;
    const bool conv = red[5] <= tol * fmax(1.0, red[6]);
    const double sig = red[3] + 4096.0 * red[4];
    stable = (sig == sig_prev) ? stable + 1 : 0;
    sig_prev = sig;
    // polish when the support has settled, and at convergence
    if (conv || stable == kPolishEvery) {
      stable = 0;
      double xp = xi, gp = 0.0, mup = 0.0;
      if (polish_face(H, G, d, ci, tau, penalty != 0, &xp, &gp, &mup, pl, cscale, true, sh) ==
          kPolishAccepted) {
        xi = xp;
        done = true;
        polished = true;
      } else if (conv) {
        done = true;  // converged iterate; the polish did not apply
      }
    }
  }
  if (!done) {  // uniform: `done` follows block-wide values only
    if (tid < d) xout[tid] = x0;  // keep x^t
    if (tid == 0) status_fail(st, 6 /* IHS_ERR_NOT_CONVERGED */, iter, p);
    return;
  }
  // counted, so that callers can tell a certified minimiser from an iterate
  // that is only as accurate as the first-order method's stopping test
  if (tid == 0 && !polished) atomicAdd(&st->unpolished, 1);
  if (tid < d) xout[tid] = xi;
}

// out = x + H^{-1} g per problem, one wavefront per row: the unconstrained
// step as the wide unconstrained QP forms it. Keeps x after a failure.
__global__ __launch_bounds__(256) void k_apply_inverse(const double* __restrict__ Hinv, int64_t d,
                                                       const double* __restrict__ g,
                                                       const double* __restrict__ x, double* out,
                                                       const DeviceStatus* st) {
  const int p = blockIdx.y;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= d) return;
  const int64_t e = (int64_t)p * d + i;
  if (status_halted(st)) {
    if (lane == 0) out[e] = x[e];
    return;
  }
  const double s = row_dot<false>(Hinv + e * d, g + (int64_t)p * d, d, lane);
  if (lane == 0) out[e] = x[e] + s;
}

// c = H x + g per problem (one wavefront per row).
__global__ __launch_bounds__(256) void k_form_c(const double* __restrict__ H, int64_t d,
                                                const double* __restrict__ x,
                                                const double* __restrict__ g, double* c) {
  const int p = blockIdx.y;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= d) return;
  const double* hr = H + ((int64_t)p * d + i) * d;
  const double* xp = x + (int64_t)p * d;
  const double s = row_dot<false>(hr, xp, d, lane);
  if (lane == 0) c[(int64_t)p * d + i] = s + g[(int64_t)p * d + i];
}

__global__ void k_fill_zero(double* v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = 0.0;
}

// ---------------------------------------------------------------------------
// The shifted-inverse series of the l2 step. With R = (H + mu0 I)^{-1} held
// and beta >= ||R||, every shift mu with |t| < 1, t = -(mu - mu0) beta, has
// (H + mu I)^{-1} = R sum_j (t R / beta)^j. The series is cut after J + 1
// terms where its tail is provably below kSeriesTail of the first term (see
// series_reaches): first at J = kSeriesFirst, which covers the small shift
// changes of later steps, then, for the problems that need it, at
// J = kSeriesTerms.
constexpr int32_t kSeriesTerms = kL2SeriesTerms;
constexpr int32_t kSeriesFirst = 8;
constexpr double kSeriesTail = 1e-17;

// l2 ball. State per problem: trs[4p] = mu, trs[4p+1] = phase
// (0 iterating, 1 one last Newton step, 2 done), trs[4p+2] = the shift mu0
// of the held inverse (H + mu0 I)^{-1}, trs[4p+3] = a bound on its 2-norm
// (infinite while no inverse is held).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block256_sum(double v, double* red) {
  const int tid = threadIdx.x;
  v = wave_sum(v);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Start of a warm step that holds the inverse of H + mu0 I formed ahead (on
// another stream, at the shift mu0 of a snapshot `pre`): the shift starts
// from the previous step's root, the inverse's shift and norm bound become
// the held state, and v = g - mu0 x^t (as k_trs_rhs). A failure recorded
// while forming the inverse (pre_st) leaves an infinite bound, so the step
// factors H + mu I itself as it would without it. One thread per entry of v.
__global__ void k_trs_begin_held(double* trs, const double* __restrict__ pre,
                                 const DeviceStatus* pre_st, const double* __restrict__ g,
                                 const double* __restrict__ x, int64_t d, int32_t batch,
                                 double* v) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)batch * d) return;
  const int p = (int)(e / d);
  const double mu0 = pre[4 * p + 2];
  v[e] = fma(-mu0, x[e], g[e]);
  if (e - (int64_t)p * d == 0) {
    const bool bad = pre_st != nullptr && status_failed_by(pre_st, -1);
    trs[4 * p] = fmax(trs[4 * p], 0.0);
    trs[4 * p + 1] = 0.0;
    trs[4 * p + 2] = mu0;
    trs[4 * p + 3] = bad ? INFINITY : pre[4 * p + 3];
  }
}

// The shift state as the next step's side work will see it: mu of each
// problem, phase 0 (so the factorisation and inverse kernels run for it).
__global__ void k_trs_snapshot(const double* trs, double* snap, int32_t batch, int32_t cold) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= batch) return;
  snap[4 * p] = cold ? 0.0 : fmax(trs[4 * p], 0.0);
  snap[4 * p + 1] = 0.0;
  snap[4 * p + 2] = 0.0;
  snap[4 * p + 3] = INFINITY;
}

// Start of a step: phase 0; the shift starts from the previous step's root
// when `warm` (the same problems, with nearby H and c), else from 0.
__global__ void k_trs_init(double* trs, int32_t batch, int32_t warm) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= batch) return;
  trs[4 * p] = warm ? fmax(trs[4 * p], 0.0) : 0.0;
  trs[4 * p + 1] = 0.0;
  trs[4 * p + 2] = 0.0;
  trs[4 * p + 3] = INFINITY;
}

// The unconstrained minimiser inside the ball is the answer.
__global__ __launch_bounds__(256) void k_trs_inside(const double* __restrict__ xunc, int64_t d,
                                                    double r, double* trs, double* xout,
                                                    const DeviceStatus* st) {
  __shared__ double red[4];
  __shared__ int skip;
  const int p = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) skip = status_halted(st) ? 1 : 0;
  __syncthreads();
  if (skip) return;
  const double* xp = xunc + (int64_t)p * d;
  double sx = 0.0;
  for (int64_t i = tid; i < d; i += 256) sx = fma(xp[i], xp[i], sx);
  if (sqrt(block256_sum(sx, red)) > r) return;
  for (int64_t i = tid; i < d; i += 256) xout[(int64_t)p * d + i] = xp[i];
  if (tid == 0) trs[4 * p + 1] = 2.0;
}

// v = g - mu0 x^t per problem (mu0 the shift of the held inverse): with it
// x(mu0) = x^t + (H + mu0 I)^{-1} v, the same point as (H + mu0 I)^{-1}
// (H x^t + g) without forming H x^t.
__global__ void k_trs_rhs(const double* __restrict__ g, const double* __restrict__ x,
                          const double* __restrict__ trs, int64_t d, int32_t batch, double* v) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)batch * d) return;
  const int p = (int)(e / d);
  v[e] = fma(-trs[4 * p + 2], x[e], g[e]);
}

// out = base + M v per problem (M symmetric, one wavefront per row; base
// nullable), for problems still iterating.
__global__ __launch_bounds__(256) void k_trs_symv(const double* __restrict__ M, int64_t d,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ base, double* out,
                                                  const double* __restrict__ trs,
                                                  const DeviceStatus* st) {
  const int p = blockIdx.y;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= d) return;
  const double* mr = M + ((int64_t)p * d + i) * d;
  const double* vp = v + (int64_t)p * d;
  const double s = row_dot<false>(mr, vp, d, lane);  // issued before the state is read
  if (trs[4 * p + 1] >= 2.0 || status_halted(st)) return;
  if (lane == 0) out[(int64_t)p * d + i] = base ? base[(int64_t)p * d + i] + s : s;
}

// y_next = (R / beta) v per problem (one wavefront per row; beta = the norm
// bound trs[4p + 3], base nullable: out = base + R v unscaled), for problems
// still iterating. The scaling keeps the series vectors y_j = (R / beta)^j y_0
// at or below the size of y_0 however small or large ||R|| is. LATE: the
// problem has usually finished already, so its state is read first and the
// row only when needed; otherwise the row's loads go out first.
template <bool LATE>
__global__ __launch_bounds__(256) void k_trs_krylov(const double* __restrict__ R, int64_t d,
                                                    const double* __restrict__ v,
                                                    const double* __restrict__ base,
                                                    double* out, const double* __restrict__ trs,
                                                    const DeviceStatus* st) {
  const int p = blockIdx.y;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= d) return;
  if (LATE && (trs[4 * p + 1] >= 2.0 || status_halted(st))) return;
  const double s = row_dot<false>(R + ((int64_t)p * d + i) * d, v + (int64_t)p * d, d, lane);
  if (!LATE && (trs[4 * p + 1] >= 2.0 || status_halted(st))) return;
  if (lane == 0) {
    const int64_t e = (int64_t)p * d + i;
    out[e] = base ? base[e] + s : s / trs[4 * p + 3];
  }
}

// Whether the series cut after y_J reaches the shift with coefficient t: the
// tail sum_{k > J} t^k y_k has norm at most
// |t|^(J+1) ||y_J|| / (1 - |t|), since ||R / beta|| <= 1 makes every later
// vector no longer than y_J; it must stay below kSeriesTail ||y_0||. The
// measured ||y_J|| = sqrt(M_2J) is far below ||y_0|| when beta overstates
// ||R||, which widens the reach to what the spectrum allows. Infinite or NaN
// t (no inverse held) is never reached.
__device__ __forceinline__ bool series_reaches(double t, double m0, double m2j, int32_t J) {
  const double a = fabs(t);
  if (!(a < 1.0)) return false;
  double pw = a;
  for (int j = 0; j < J; ++j) pw *= a;
  return pw * sqrt(m2j) <= kSeriesTail * (1.0 - a) * sqrt(m0);
}

// One round's series step for one problem (one workgroup of 256 per
// problem), for the problems still iterating:
//  1. the moments M_s = y_0^T (R / beta)^s y_0, s = 0 .. 2J, from the series
//     vectors: M_2j = y_j^T y_j and M_2j+1 = y_j^T y_j+1 (R is symmetric),
//     each summed strided over the threads, then over the wavefronts in a
//     fixed order;
//  2. the Newton iteration of k_trs_update on the series, in one thread:
//     with t = -(mu - mu0) beta, x(mu) = sum_j t^j y_j, so ||x(mu)||^2 =
//     sum_s (s + 1) M_s t^s and x^T (H + mu I)^{-1} x = -(1/2) d||x||^2/dmu
//     = (beta / 2) sum_s s (s + 1) M_s t^(s-1). A shift the series does not
//     reach is left in trs[4p] for a new factorisation (or a longer series);
//  3. for an accepted shift, x_out = sum_j t^j y_j; the problem finishes
//     (phase 2).
template <int J>
__global__ __launch_bounds__(256) void k_trs_series_solve(const double* __restrict__ Y, int64_t d,
                                                          int32_t batch, double r, double tol,
                                                          int32_t max_steps, double* trs,
                                                          double* xout, const DeviceStatus* st) {
  constexpr int NM = 2 * J + 1;
  __shared__ double part[4][NM];
  __shared__ double M[NM];
  __shared__ int skip;
  __shared__ double t_acc;
  const int p = blockIdx.x, tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  if (tid == 0) skip = (status_halted(st) || trs[4 * p + 1] >= 2.0) ? 1 : 0;
  __syncthreads();
  if (skip) return;
  double acc[NM];
#pragma unroll
  for (int q = 0; q < NM; ++q) acc[q] = 0.0;
  for (int64_t i = tid; i < d; i += 256) {
    double y[J + 1];
#pragma unroll
    for (int j = 0; j <= J; ++j) y[j] = Y[((int64_t)j * batch + p) * d + i];
#pragma unroll
    for (int j = 0; j <= J; ++j) {
      acc[2 * j] = fma(y[j], y[j], acc[2 * j]);
      if (j < J) acc[2 * j + 1] = fma(y[j], y[j + 1], acc[2 * j + 1]);
    }
  }
#pragma unroll
  for (int q = 0; q < NM; ++q) {
    const double w = wave_sum(acc[q]);
    if (lane == 0) part[wv][q] = w;
  }
  __syncthreads();
  if (tid < NM) M[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
  __syncthreads();
  if (tid == 0) {
    const double mu0 = trs[4 * p + 2], beta = trs[4 * p + 3];
    double mu = trs[4 * p], phase = trs[4 * p + 1];
    bool accepted = false;
    // a warm start beyond the series' reach starts at mu0 instead (t = 0,
    // where the series is exact): the root may still lie within reach
    if (phase == 0.0 && !series_reaches(-(mu - mu0) * beta, M[0], M[2 * J], J) &&
        series_reaches(0.0, M[0], M[2 * J], J))
      mu = mu0;
    for (int32_t k = 0; k < max_steps; ++k) {
      const double t = -(mu - mu0) * beta;
      if (!series_reaches(t, M[0], M[2 * J], J)) break;
      double phi = 0.0, dq = 0.0;  // Horner, highest power first
      for (int sidx = 2 * J; sidx >= 0; --sidx) {
        phi = fma(phi, t, (sidx + 1) * M[sidx]);
        if (sidx >= 1) dq = fma(dq, t, 0.5 * sidx * (sidx + 1) * M[sidx]);
      }
      const double nx2 = phi, q = beta * dq, nx = sqrt(nx2);
      if (phase == 1.0 || (mu == 0.0 && nx <= r)) {
        accepted = true;
        break;
      }
      const double next = fmax(mu + (nx2 / q) * ((nx - r) / r), 0.0);
      if (fabs(nx - r) <= tol * r) phase = 1.0;
      mu = next;
    }
    trs[4 * p] = mu;
    trs[4 * p + 1] = accepted ? 2.0 : phase;
    skip = accepted ? 0 : 1;
    t_acc = -(mu - mu0) * beta;
  }
  __syncthreads();
  if (skip) return;
  const double t = t_acc;
  for (int64_t i = tid; i < d; i += 256) {
    double x = Y[((int64_t)J * batch + p) * d + i];
    for (int j = J - 1; j >= 0; --j) x = fma(x, t, Y[((int64_t)j * batch + p) * d + i]);
    xout[(int64_t)p * d + i] = x;
  }
}

// Given x = x(mu) and z = (H + mu I)^{-1} x, applies the Newton step
// mu <- max(mu + (||x||^2 / x^T z) (||x|| - r) / r, 0). When
// | ||x|| - r | <= tol r the problem takes that one more step (phase 1) and
// accepts the next x, which the quadratic rate puts at rounding level. From
// a warm start above the root, the first step lands below it (the tangent of
// a concave function lies above it) and the rest rise monotonically; at
// mu = 0 a point inside the ball is the unconstrained minimiser and is
// accepted as it is.
__global__ __launch_bounds__(256) void k_trs_update(const double* __restrict__ xk,
                                                    const double* __restrict__ zk, int64_t d,
                                                    double r, double tol, double* trs,
                                                    double* xout, const DeviceStatus* st) {
  __shared__ double red[4];
  __shared__ int skip;
  const int p = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) skip = (status_halted(st) || trs[4 * p + 1] >= 2.0) ? 1 : 0;
  __syncthreads();
  if (skip) return;
  const double* xp = xk + (int64_t)p * d;
  const double* zp = zk + (int64_t)p * d;
  double sx = 0.0, sq = 0.0;
  for (int64_t i = tid; i < d; i += 256) {
    sx = fma(xp[i], xp[i], sx);
    sq = fma(xp[i], zp[i], sq);
  }
  const double nx2 = block256_sum(sx, red);
  const double q = block256_sum(sq, red);
  const double nx = sqrt(nx2);
  // one last step taken, or the unconstrained minimiser (mu = 0) in the ball
  if (trs[4 * p + 1] == 1.0 || (trs[4 * p] == 0.0 && nx <= r)) {
    for (int64_t i = tid; i < d; i += 256) xout[(int64_t)p * d + i] = xp[i];
    if (tid == 0) trs[4 * p + 1] = 2.0;
    return;
  }
  if (tid == 0) {
    trs[4 * p] = fmax(trs[4 * p] + (nx2 / q) * ((nx - r) / r), 0.0);
    if (fabs(nx - r) <= tol * r) trs[4 * p + 1] = 1.0;
  }
}

// Row sums of |M| per problem (one wavefront per row), for the norm bound.
__global__ __launch_bounds__(256) void k_trs_abs_rows(const double* __restrict__ M, int64_t d,
                                                      const double* __restrict__ trs,
                                                      double* rows, const DeviceStatus* st) {
  const int p = blockIdx.y;
  if (trs[4 * p + 1] >= 2.0 || status_halted(st)) return;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= d) return;
  const double* mr = M + ((int64_t)p * d + i) * d;
  const double s = row_dot<true>(mr, nullptr, d, lane);
  if (lane == 0) rows[(int64_t)p * d + i] = s;
}

// Records the shift of the inverse just formed and a bound on its 2-norm: the
// largest absolute row sum (the infinity norm, which bounds the 2-norm of a
// symmetric matrix), and 1/mu0 when mu0 > 0 (H is positive semidefinite).
__global__ __launch_bounds__(256) void k_trs_inv_norm(const double* __restrict__ rows, int64_t d,
                                                      double* trs, const DeviceStatus* st) {
  __shared__ double red[4];
  const int p = blockIdx.x, tid = threadIdx.x;
  if (trs[4 * p + 1] >= 2.0 || status_halted(st)) return;
  double mx = 0.0;
  for (int64_t i = tid; i < d; i += 256) mx = fmax(mx, rows[(int64_t)p * d + i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = mx;
  __syncthreads();
  if (tid == 0) {
    const double mu0 = trs[4 * p];
    double nrm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (mu0 > 0.0) nrm = fmin(nrm, 1.0 / mu0);
    trs[4 * p + 2] = mu0;
    trs[4 * p + 3] = nrm;
  }
}

// Problems still iterating after the last Newton step keep x^t and report.
__global__ void k_trs_finish(const double* trs, int64_t d, const double* x, double* xout,
                             DeviceStatus* st, int32_t iter) {
  const int p = blockIdx.x;
  if (status_halted(st) || trs[4 * p + 1] >= 2.0) return;
  for (int64_t i = threadIdx.x; i < d; i += 256) xout[(int64_t)p * d + i] = x[(int64_t)p * d + i];
  if (threadIdx.x == 0) status_fail(st, 6 /* IHS_ERR_NOT_CONVERGED */, iter, p);
}

// Copies the status words that end the Newton loop (a failure, the outer
// loop's stop) behind the shift state, so one read brings both to the host.
__global__ void k_trs_status(const DeviceStatus* st, double* dst) {
  if (threadIdx.x == 0) dst[0] = (double)(status_word(&st->code) | status_word(&st->done));
}

// True when every problem has finished its Newton iteration, a failure is
// recorded or the outer loop has stopped; leaves the shift state in h.
// Synchronises the stream.
static bool trs_all_done(double* trs, const DeviceStatus* status, int32_t batch,
                         hipStream_t st, std::vector<double>& h) {
  h.assign((size_t)4 * batch + 1, 0.0);
  hipLaunchKernelGGL(k_trs_status, dim3(1), dim3(64), 0, st, status, trs + 4 * batch);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(h.data(), trs, h.size() * sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return false;
  if (h[(size_t)4 * batch] != 0.0) return true;
  for (int32_t p = 0; p < batch; ++p)
    if (h[(size_t)4 * p + 1] < 2.0) return false;
  return true;
}

hipError_t launch_qp_constrained(const QpArgs& a, hipStream_t st) {
  const int64_t d = a.d;
  const int32_t B = a.batch;
  if (d > kQpThreads) return hipErrorNotSupported;
  double* scratch = a.work;
  double* rdiag = chol_rdiag(scratch, B);
  // past the unconstrained step's scratch: c, x_unc, x(mu), z, a spare
  // vector, the shift state, then (l2) H^{-1} and the triangular inverse
  double* cbuf = a.work + (int64_t)B * (64 * 64 + 9 * d + 64);
  double* xunc = cbuf + (int64_t)B * d;
  double* xk = xunc + (int64_t)B * d;
  double* zk = xk + (int64_t)B * d;
  double* zero = zk + (int64_t)B * d;
  double* trs = zk + (int64_t)B * 2 * d;
  double* hinv = trs + (int64_t)B * 8;
  double* linv = hinv + (int64_t)B * d * d;
  hipError_t e;
  if (a.constraint == 1 || a.constraint == 3) {
    const bool penalty = a.constraint == 3;
    hipLaunchKernelGGL(k_form_c, dim3((unsigned)((d + 3) / 4), B), dim3(256), 0, st, a.H, d,
                       a.x, a.g, cbuf);
    if (!penalty && a.hinv_pre) {  // the unconstrained minimiser from a given inverse
      hipLaunchKernelGGL(k_apply_inverse, dim3((unsigned)((d + 3) / 4), B), dim3(256), 0, st,
                         a.hinv_pre, d, a.g, a.x, xunc, a.status);
    } else if (!penalty) {  // the unconstrained minimiser, the answer when the ball is inactive
      const double* rd = a.rdiag_pre;
      if (!rd) {
        if ((e = launch_cholesky(a.H, a.L, d, B, a.status, a.iter, 0.0, scratch, st)) !=
            hipSuccess)
          return e;
        rd = rdiag;
      }
      e = launch_chol_solve_update(a.L, rd, d, B, a.g, a.x, xunc, a.status, st);
      if (e != hipSuccess) return e;
    }
    const int32_t max_iter = a.max_inner > 0 ? a.max_inner : 5000;
    const double tol = a.tol > 0 ? a.tol : 1e-15;
    const size_t fixed = (size_t)(3 * d + 2 * kPolishMax) * sizeof(double);
    const int32_t lds_mcap = (int32_t)((kQpLdsBytes - fixed) / sizeof(double));
    hipLaunchKernelGGL(k_qp_l1, dim3(B), dim3(kQpThreads), kQpLdsBytes, st, a.H, cbuf, xunc,
                       a.x, a.x_out, a.hinv_pre, penalty ? a.pre_status : nullptr, d, a.radius,
                       penalty ? 1 : 0, max_iter, tol, lds_mcap, a.status, a.iter);
    return hipGetLastError();
  }
  // l2 ball. A cold start (mu = 0) first takes the unconstrained step
  // x^t + H^{-1} g, the answer when it lies in the ball, and the Newton step
  // from it; a warm start begins at the previous step's shift.
  const int32_t newton = a.max_inner > 0 ? a.max_inner : 30;
  const double tol = a.tol > 0 ? a.tol : 1e-10;
  const int64_t bd = (int64_t)B * d;
  const dim3 rows_grid((unsigned)((d + 3) / 4), B);
  const bool pre_held = a.warm && a.hinv_pre && a.trs_pre;  // an inverse formed ahead
  if (pre_held)
    hipLaunchKernelGGL(k_trs_begin_held, dim3((unsigned)((bd + 255) / 256)), dim3(256), 0, st,
                       trs, a.trs_pre, a.pre_status, a.g, a.x, d, B, cbuf);
  else
    hipLaunchKernelGGL(k_trs_init, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, trs, B,
                       a.warm);
  if (!a.warm) {
    if ((e = launch_cholesky(a.H, a.L, d, B, a.status, a.iter, 0.0, scratch, st)) != hipSuccess)
      return e;
    // the unconstrained step computed as the unconstrained QP computes it
    // (so an inactive ball returns that step bit for bit), then z
    const bool inv = d >= kQpInverseMinD;
    if (inv) {
      if ((e = launch_chol_inverse(a.L, rdiag, d, B, hinv, linv, a.status, st)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(k_trs_symv, rows_grid, dim3(256), 0, st, hinv, d, a.g, a.x, xunc, trs,
                         a.status);
    } else if ((e = launch_chol_solve_update(a.L, rdiag, d, B, a.g, a.x, xunc, a.status, st)) !=
               hipSuccess) {
      return e;
    }
    hipLaunchKernelGGL(k_trs_inside, dim3(B), dim3(256), 0, st, xunc, d, a.radius, trs, a.x_out,
                       a.status);
    if (inv) {
      hipLaunchKernelGGL(k_trs_symv, rows_grid, dim3(256), 0, st, hinv, d, xunc, nullptr, zk, trs,
                         a.status);
    } else {
      hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((bd + 255) / 256)), dim3(256), 0, st, zero,
                         bd);
      e = launch_chol_solve_update(a.L, rdiag, d, B, xunc, zero, zk, a.status, st);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_trs_update, dim3(B), dim3(256), 0, st, xunc, zk, d, a.radius, tol, trs,
                       a.x_out, a.status);
  }
  // The Newton iteration runs on the series of a held inverse R = (H + mu0
  // I)^{-1}: y_0 = x(mu0), y_j = (R / beta) y_j-1 and their moments give
  // ||x(mu)|| and its derivative at every shift the series reaches, so the
  // iteration itself needs no solve and no read-back. A round factors H + mu I
  // at the current shift (unless an inverse formed ahead is held), forms the
  // series and iterates; a shift beyond its reach starts the next round there.
  // The accepted x(mu) is formed from the series vectors.
  double* Y = linv + (int64_t)B * d * d;
  std::vector<double> h;
  bool held = pre_held;  // v = g - mu0 x^t is then formed already
  const double* R = pre_held ? a.hinv_pre : hinv;
  for (int32_t round = 0; round < newton; ++round) {
    if (!held) {
      if ((e = launch_cholesky(a.H, a.L, d, B, a.status, a.iter, 0.0, scratch, st, trs)) !=
          hipSuccess)
        return e;
      if ((e = launch_chol_inverse(a.L, rdiag, d, B, hinv, linv, a.status, st, trs)) !=
          hipSuccess)
        return e;
      hipLaunchKernelGGL(k_trs_abs_rows, rows_grid, dim3(256), 0, st, hinv, d, trs, zero,
                         a.status);
      hipLaunchKernelGGL(k_trs_inv_norm, dim3(B), dim3(256), 0, st, zero, d, trs, a.status);
      R = hinv;
      hipLaunchKernelGGL(k_trs_rhs, dim3((unsigned)((bd + 255) / 256)), dim3(256), 0, st, a.g,
                         a.x, trs, d, B, cbuf);
    }
    held = false;
    hipLaunchKernelGGL(k_trs_krylov<false>, rows_grid, dim3(256), 0, st, R, d, cbuf, a.x, Y,
                       trs, a.status);
    // the series to kSeriesFirst; then, only if some problem needs it, on to
    // kSeriesTerms (one read-back between: launches that would find every
    // problem finished still cost their dispatch)
    for (int32_t j = 1; j <= kSeriesFirst; ++j)
      hipLaunchKernelGGL(k_trs_krylov<false>, rows_grid, dim3(256), 0, st, R, d,
                         Y + (j - 1) * bd, nullptr, Y + j * bd, trs, a.status);
    hipLaunchKernelGGL(k_trs_series_solve<kSeriesFirst>, dim3(B), dim3(256), 0, st, Y, d, B,
                       a.radius, tol, newton, trs, a.x_out, a.status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (trs_all_done(trs, a.status, B, st, h)) break;
    for (int32_t j = kSeriesFirst + 1; j <= kSeriesTerms; ++j)
      hipLaunchKernelGGL(k_trs_krylov<true>, rows_grid, dim3(256), 0, st, R, d,
                         Y + (j - 1) * bd, nullptr, Y + j * bd, trs, a.status);
    hipLaunchKernelGGL(k_trs_series_solve<kSeriesTerms>, dim3(B), dim3(256), 0, st, Y, d, B,
                       a.radius, tol, newton, trs, a.x_out, a.status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (trs_all_done(trs, a.status, B, st, h)) break;
  }
  hipLaunchKernelGGL(k_trs_finish, dim3(B), dim3(256), 0, st, trs, d, a.x, a.x_out, a.status,
                     a.iter);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// The l2 step's factorisation ahead of time (overlapped schedule): while the
// caller's stream runs the steps before it, another stream factors H_k + mu I
// and inverts it, mu from a snapshot of the shift state taken on the caller's
// stream (the root of an earlier step). Step k then runs its Newton iteration
// on the series of that inverse for every shift the series reaches, and
// factors afresh only beyond.
// ---------------------------------------------------------------------------
static double* l2_trs(double* work, int64_t d, int32_t B) {
  // past the unconstrained step's scratch: c, x_unc, x(mu), z, a spare, then
  // the shift state (as laid out in launch_qp_constrained)
  return work + (int64_t)B * (64 * 64 + 9 * d + 64) + (int64_t)B * 5 * d;
}

hipError_t launch_l2_snapshot(double* work, int64_t d, int32_t batch, double* snap, int32_t cold,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_trs_snapshot, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st,
                     l2_trs(work, d, batch), snap, batch, cold);
  return hipGetLastError();
}

hipError_t launch_l2_prefactor(const double* H, int64_t d, int32_t batch, double* snap, double* L,
                               double* hinv, double* linv, double* scratch, double* rows,
                               DeviceStatus* status, int32_t iter, hipStream_t st) {
  hipError_t e;
  if ((e = launch_cholesky(H, L, d, batch, status, iter, 0.0, scratch, st, snap)) != hipSuccess)
    return e;
  if ((e = launch_chol_inverse(L, chol_rdiag(scratch, batch), d, batch, hinv, linv, status, st,
                               snap)) != hipSuccess)
    return e;
  const dim3 rows_grid((unsigned)((d + 3) / 4), batch);
  hipLaunchKernelGGL(k_trs_abs_rows, rows_grid, dim3(256), 0, st, hinv, d, snap, rows, status);
  hipLaunchKernelGGL(k_trs_inv_norm, dim3(batch), dim3(256), 0, st, rows, d, snap, status);
  return hipGetLastError();
}

}  // namespace ihs
