/*
 * ihs.h -- C ABI of libihs, an MI355X (gfx950) implementation of the
 * Iterative Hessian Sketch with sparse embeddings (Cormode and Dickens,
 * "Iterative Hessian Sketch in Input Sparsity Time").
 *
 * Problem (Eq.(1)):   x_OPT = argmin_{x in C} 1/2 ||A x - b||^2,
 *                     C = R^d, {||x||_1 <= radius} or {||x||_2 <= radius}.
 * Step (Eq.(2)):      x^{t+1} = argmin_{x in C} 1/2 ||S^{t+1} A (x - x^t)||^2
 *                                 - <A^T (b - A x^t), x - x^t>,
 *                     with a fresh sparse embedding S^{t+1} every step.
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" are HIP device memory owned by the caller; the
 *    library never allocates memory that outlives a call and never frees
 *    caller memory. Pointers marked "host" are ordinary host memory.
 *  - Dense matrices are row-major with a leading dimension in elements.
 *  - Work is enqueued on `stream` (0 = the null stream). Calls that say
 *    "synchronises" wait for the stream before returning; the others are
 *    asynchronous and report only argument and launch errors.
 *  - All argument checks run on the host before anything is enqueued; a
 *    failed check returns an error code and has no side effects.
 *  - `ws` is a caller-owned device workspace of at least the size returned by
 *    the matching *_workspace_size query. Two calls may run concurrently on
 *    different streams only with distinct workspaces.
 *  - Floating-point results are deterministic: no floating-point atomics are
 *    used, every reduction runs in a fixed order, and two runs with the same
 *    inputs are bitwise equal.
 */
#ifndef IHS_H
#define IHS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IHS_OK = 0,
  IHS_ERR_INVALID_ARG = 1,   /* null pointer, bad size, s not dividing m, ...  */
  IHS_ERR_UNSUPPORTED = 2,   /* valid but outside what the kernels implement   */
  IHS_ERR_WORKSPACE = 3,     /* ws_bytes below the queried size                */
  IHS_ERR_HIP = 4,           /* a HIP runtime call or kernel launch failed     */
  IHS_ERR_NOT_PD = 5,        /* non-positive Cholesky pivot: H not definite    */
  IHS_ERR_NOT_CONVERGED = 6, /* an inner QP iteration hit its cap, or a solve
                                with tol > 0 ran max_iter steps unconverged   */
  IHS_ERR_NONFINITE = 7      /* NaN or Inf in the objective or the iterate     */
} ihs_status;

typedef enum { IHS_F64 = 0, IHS_F32 = 1, IHS_BF16 = 2 } ihs_dtype;
/* The sparse embeddings (CountSketch, SJLT) and the two dense sketches of
 * Sec. 2 that the paper compares them with (SRHT, Gaussian). */
typedef enum {
  IHS_COUNTSKETCH = 0,
  IHS_SJLT = 1,
  IHS_SRHT = 2,
  IHS_GAUSSIAN = 3
} ihs_sketch_kind;
/* The set C of Eq.(1), or (IHS_L1_PENALTY) the weight lambda ||x||_1 added to
 * the objective over R^d: the penalised LASSO of the experiments of Sec. 3. */
typedef enum {
  IHS_UNCONSTRAINED = 0,
  IHS_L1_BALL = 1,
  IHS_L2_BALL = 2,
  IHS_L1_PENALTY = 3
} ihs_constraint;
typedef enum { IHS_DENSE = 0, IHS_CSR = 1 } ihs_format;
/* How ihs_solve iterates. IHS_METHOD_IHS: the Iterative Hessian Sketch,
 * Eq.(2) with a fresh sketch at every step (Sec. 1, Thm 2.2).
 * IHS_METHOD_FIXED_SKETCH_CG: the direction the conclusion names, fewer
 * passes over the data: one sketch S_0 is drawn once and its Hessian sketch
 * H_0 = (S_0 A)^T S_0 A preconditions conjugate gradients on the normal
 * equations A^T A x = A^T b (C = R^d only). */
typedef enum { IHS_METHOD_IHS = 0, IHS_METHOD_FIXED_SKETCH_CG = 1 } ihs_method;

/* The data matrix A (n x d). Dense: `values` (device) holds n rows of `ld`
 * elements, dtype F64 or F32. CSR: `row_ptr` (device, n+1), `col_idx`
 * (device, nnz, sorted and unique within each row, in [0, d)) and `values`
 * (device, nnz, F64). A ragged batch (`batch` > 1, dense or CSR) stacks the
 * rows of `batch` independent problems of the same width d (for CSR, row_ptr
 * and col_idx span all n rows); `row_offsets` is a HOST array of batch+1
 * increasing entries with row_offsets[0] = 0 and row_offsets[batch] = n.
 * batch = 1 ignores row_offsets. */
typedef struct {
  int32_t format;              /* ihs_format                                  */
  int32_t dtype;               /* ihs_dtype of values: IHS_F64 or IHS_F32     */
  int64_t n, d, ld;            /* rows, columns, leading dimension (dense)    */
  const void* values;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  int64_t nnz;
  int32_t batch;
  int32_t reserved;
  const int64_t* row_offsets;
} ihs_matrix;

/* A sparse embedding (Sec. 2). CountSketch: s = 1, each column of S holds one
 * +-1 at a uniformly chosen row. SJLT: s blocks of m/s rows stacked row-wise,
 * each an independent CountSketch, entries scaled by 1/sqrt(s) so that
 * E[S^T S] = I (App. A.1.1, Lemma A.7). The random choices are a pure function
 * of (seed, iter, row, block, problem) through Philox4x64-10:
 *   words = Philox4x64-10(counter = (row, block / 2, problem, 0),
 *                         key = (seed, iter))
 *   block k: sketch row = k*(m/s) + floor(words[2(k%2)] * (m/s) / 2^64),
 *            sign = -1 if bit 63 of words[2(k%2)+1] is set, else +1.
 * `row` counts from 0 within a problem. `m` is per problem.
 *
 * The dense sketches (s = 1, one problem: batch = 1), with their own counter
 * streams under the same key (counter word 3 names the stream):
 *  SRHT (Sec. 2): S = (1/sqrt(m)) P H D. D_i = -1 if bit 63 of word 1 of
 *   Philox(counter = (i, 0, 0, 1)) is set, else +1; H is the unnormalised
 *   Sylvester-Hadamard transform on N = 2^ceil(log2 n) rows (A padded with
 *   zero rows), applied as the radix-2 recursion (stages h = 1, 2, 4, ...,
 *   (y_i, y_{i+h}) -> (y_i + y_{i+h}, y_i - y_{i+h})); row k of P samples
 *   row floor(word 0 of Philox((k, 0, 0, 2)) * N / 2^64), independently
 *   (with replacement). The result is bitwise that of this definition.
 *  Gaussian (Sec. 2): S = G / sqrt(m), G[4q + j][i] (j = 0..3) from
 *   Philox((i, q, 0, 3)) by the Box-Muller method: for word pairs (0, 1) and
 *   (2, 3), u1 = ((w_a >> 11) + 1) 2^-53, u2 = (w_b >> 11) 2^-53,
 *   rho = sqrt(-2 ln u1), G = rho cos(2 pi u2) (j even) and rho sin(2 pi u2)
 *   (j odd). Summed in float64 on the matrix cores in a fixed order. */
typedef struct {
  int32_t kind;                /* ihs_sketch_kind                             */
  int32_t s;                   /* blocks; 1 for CountSketch                   */
  int64_t m;                   /* sketch rows per problem                     */
  uint64_t seed;
  uint64_t iter;               /* iteration word of the key                   */
} ihs_sketch;

/* Options of ihs_solve. Step t (0-based) of a solve uses the sketch keyed
 * (sketch.seed, sketch.iter + t). */
typedef struct {
  int32_t constraint;          /* ihs_constraint                              */
  int32_t max_iter;            /* number of IHS steps N >= 1                  */
  double radius;               /* ball radius (> 0 for ball constraints), or
                                  lambda >= 0 for IHS_L1_PENALTY               */
  ihs_sketch sketch;
  int32_t gram_in;             /* dtype SA is stored in for the Gram          */
  int32_t gram_acc;            /* dtype the Gram accumulates in (F64 or F32)  */
  int32_t qp_max_inner;        /* cap on inner QP iterations; 0 = default:
                                  l1 ball and penalty: accelerated (projected
                                  or proximal) gradient iterations (5000); l2
                                  ball: Newton steps on the shift (30)         */
  int32_t keep_factors;        /* store each step's Cholesky factor           */
  double qp_tol;               /* inner stopping tolerance; 0 = default:
                                  l1 ball and penalty: max |x_{k+1} - x_k| <= qp_tol
                                  max(1, |x|_inf) (1e-15; a KKT-certified
                                  polish usually ends the iteration first);
                                  l2 ball: | ||x|| - r | <= qp_tol r, then one
                                  more Newton step (1e-10)                     */
  double tol;                  /* stopping tolerance on the length of a step
                                  in the prediction norm (Def. A.1; Thm 2.2:
                                  the error contracts geometrically, so the
                                  step length tracks it): after step t the
                                  solve stops when no failure is recorded and
                                  every problem's sqrt(dx^T H_t dx),
                                  dx = x^{t+1} - x^t, is at most tol. The test
                                  runs on the device; the steps already queued
                                  behind it return at once and keep x, so the
                                  result is bitwise that of a solve with
                                  max_iter = rep->iters. 0: run max_iter
                                  steps. With tol > 0, reaching max_iter first
                                  returns IHS_ERR_NOT_CONVERGED (x holds x^N,
                                  failed_iter = -1). Rows of x_hist after
                                  rep->iters repeat the final iterate. Must be
                                  finite and >= 0; not with
                                  IHS_METHOD_FIXED_SKETCH_CG                  */
  int32_t schedule;            /* 0: overlap the next step's sort, Gram and
                                  (unconstrained and l1 ball) factorisation
                                  with the current pass over A on other
                                  streams (one extra sketch-only pass per
                                  solve); the constrained QP of the step then
                                  runs on the caller's stream from the Gram
                                  (and factor) formed beside the previous
                                  pass. From d = 89 on the factor is also
                                  inverted there, and the l1 penalty's step
                                  (whose H is otherwise not factored) gets
                                  the inverse too, for its KKT polish;
                                  1: strictly sequential steps;
                                  2: as 0 but two steps ahead, so the
                                  factorisation has two passes of time (for
                                  short passes, e.g. float32 data; two
                                  sketch-only passes per solve; constrained
                                  problems look one step ahead).
                                  All form bitwise identical sketches and
                                  factors; the iterates agree to rounding,
                                  since the fused pass adds up A^T r in the
                                  row order of the sketch it forms (S_{t+1} or
                                  S_{t+2} when overlapping, S_t otherwise).
                                  The dense sketch kinds always run
                                  sequential steps: the sketch, then a
                                  separate gradient pass.                     */
  int32_t method;              /* ihs_method. IHS_METHOD_FIXED_SKETCH_CG:
                                  max_iter conjugate-gradient iterations after
                                  one pass that forms S_0 A (key (sketch.seed,
                                  sketch.iter)) and A^T (b - A x^0); each
                                  iteration is one more pass over A. Requires
                                  C = R^d and factors = NULL; schedule is not
                                  read.                                        */
} ihs_options;

/* Filled by ihs_solve (host memory). */
typedef struct {
  int32_t iters;               /* steps actually taken (the tolerance stop's
                                  step count, or the step of a failure)        */
  int32_t status;              /* ihs_status of the device work               */
  int32_t failed_iter;         /* step at which a device error occurred, or -1 */
  int32_t failed_problem;      /* problem index of that error, or -1          */
  double objective;            /* 1/2 ||A x^{N-1} - b||^2 (problem 0), from the last
                                  pass (IHS_METHOD_FIXED_SKETCH_CG: at x^0)     */
  double last_step;            /* sqrt(dx^T H dx) of the last step (problem 0) */
  int32_t qp_unpolished;       /* l1-ball and l1-penalty QPs (over steps and
                                  problems) that ended on a converged
                                  first-order iterate the KKT polish did not
                                  certify; 0 when every QP solution is an
                                  exact KKT point                              */
  int32_t reserved;
} ihs_report;

const char* ihs_status_string(int32_t status);

/* The HIP runtime error behind the most recent IHS_ERR_HIP returned on the
 * calling thread: its name (hipGetErrorName), and its hipError_t value in
 * *code when code is not NULL ("hipSuccess" and 0 before any such failure).
 * Every entry point first clears an error that earlier, unrelated HIP calls
 * left pending on the thread, so IHS_ERR_HIP always names a failure of the
 * library's own launches or runtime calls. Host only. */
const char* ihs_last_hip_error(int32_t* code);

/* Bucket and sign of every (row, block) pair of one problem's sketch, exactly
 * as defined under ihs_sketch. bucket (device, n*s int32) receives the sketch
 * row in [0, m) of pair (i, k) at index i*s + k; sign (device, n*s int8)
 * receives +1 or -1. The dense sketch kinds have no hash
 * (IHS_ERR_UNSUPPORTED). Asynchronous. */
ihs_status ihs_sketch_hash(const ihs_sketch* sk, int64_t n, int32_t problem,
                           int32_t* bucket, int8_t* sign, hipStream_t stream);

/* Workspace bytes sufficient for ihs_sketch_apply, ihs_gradient and
 * ihs_solve on this matrix with these options (for ihs_sketch_apply and
 * ihs_gradient only opt->sketch is read). Host only, no launch. Returns 0 for
 * invalid arguments. */
size_t ihs_workspace_size(const ihs_matrix* A, const ihs_options* opt);

/* SA = S A (Sec. 2, "Time Complexity": one pass over the nonzeros of A for
 * the sparse embeddings; a fast Hadamard transform for the SRHT and a dense
 * product on the matrix cores for the Gaussian sketch, both on one problem
 * (batch = 1, else IHS_ERR_UNSUPPORTED), CSR data expanded to dense rows in
 * the workspace first).
 * SA (device) is (batch*m) x d row-major with leading dimension ld_sa >= d;
 * problem p fills rows [p*m, (p+1)*m). Each entry is the sum, in ascending
 * row order from +0.0, of sign * A[row][col] over the rows hashed to that
 * sketch row, accumulated in float64 and multiplied once by 1/sqrt(s) when
 * s > 1; sa_dtype F32 or BF16 stores that float64 value rounded to nearest
 * even once. The result is therefore bitwise reproducible and equal to a
 * sequential evaluation of the definition. Asynchronous. */
ihs_status ihs_sketch_apply(const ihs_sketch* sk, const ihs_matrix* A,
                            void* SA, int32_t sa_dtype, int64_t ld_sa,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of the device scratch array that ihs_sketch_apply_static uses in
 * place of a workspace (one array per GPU, held until the process ends). */
#define IHS_STATIC_SCRATCH_BYTES (64u << 20)

/* ihs_sketch_apply without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): the same SA, bit for bit, with the sort state (keys,
 * per-tile counts, scan partials, bucket starts and the row permutation) in
 * a file-scope device array of IHS_STATIC_SCRATCH_BYTES per GPU instead of
 * `ws`. It calls no hipMalloc, hipFree or other allocating routine; the
 * first call on a device looks the array's address up (hipGetSymbolAddress).
 * The caller still provides A and SA. A problem whose sort state exceeds the
 * array returns IHS_ERR_WORKSPACE before anything is enqueued (it fits
 * n*s <= 2^22 rows with m = 4096, e.g. the 2^22 x 512 matrix with a
 * CountSketch of 4096 rows). Every call on one GPU shares the array: calls
 * that overlap in time on one GPU (different streams or threads) race, and
 * must be ordered by the caller. Asynchronous. */
ihs_status ihs_sketch_apply_static(const ihs_sketch* sk, const ihs_matrix* A,
                                   void* SA, int32_t sa_dtype, int64_t ld_sa,
                                   hipStream_t stream);

/* out = S^T G (the adjoint of ihs_sketch_apply, used by its derivative).
 * G (device) is (batch*m) x d F64 with leading dimension ld_g; out (device)
 * is n x d F64 with leading dimension ld_out. Row i of problem p receives the
 * sum over blocks k, ascending from +0.0, of sign(i,k) * (c_s * G[p*m +
 * bucket(i,k)][:]), c_s = 1/sqrt(s) (the factor is skipped for s = 1).
 * row_offsets: HOST, batch+1 entries (NULL when batch = 1). s > 16 returns
 * IHS_ERR_UNSUPPORTED, and so do the dense sketch kinds. Asynchronous. */
ihs_status ihs_sketch_adjoint(const ihs_sketch* sk, int64_t n, int64_t d,
                              int32_t batch, const int64_t* row_offsets,
                              const double* G, int64_t ld_g,
                              double* out, int64_t ld_out, hipStream_t stream);

/* Workspace bytes for ihs_gram. Host only. */
size_t ihs_gram_workspace_size(int64_t m, int64_t d, int32_t batch,
                               int32_t in_dtype, int32_t acc_dtype);

/* H = (SA)^T (SA), the approximate Hessian of Eq.(2) (Sec. 1, T_QP), for each
 * of `batch` stacked m x d blocks of SA (device, dtype in_dtype, leading
 * dimension ld). H (device) receives batch full symmetric d x d float64
 * matrices, contiguous. in_dtype F64 requires acc_dtype F64 (FP64 matrix
 * cores); F32 inputs accumulate in F32 or F64; BF16 inputs accumulate in F32.
 * An F32 accumulation is widened to float64 when stored. Asynchronous. */
ihs_status ihs_gram(const void* SA, int32_t in_dtype, int64_t m, int64_t d,
                    int64_t ld, int32_t batch, int32_t acc_dtype, double* H,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/* Residual r = b - A x, the linear term g = A^T r of Eq.(2) and the objective
 * f = 1/2 ||r||^2 of Eq.(1), all float64. b (device, n), x (device,
 * batch x d), g (device, batch x d), r (device, n, nullable), f (device,
 * batch, nullable). ws from ihs_workspace_size. Asynchronous. */
ihs_status ihs_gradient(const ihs_matrix* A, const double* b, const double* x,
                        double* g, double* r, double* f,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for ihs_qp_step. Host only. */
size_t ihs_qp_workspace_size(int64_t d, int32_t batch, const ihs_options* opt);

/* One QP of Eq.(2) per problem: given H (device, batch x d x d symmetric
 * positive definite, float64), g (device, batch x d) and x^t (device,
 * batch x d), writes x^{t+1} (device, batch x d) = argmin over C of
 * 1/2 (x - x^t)^T H (x - x^t) - g^T (x - x^t), with C from Eq.(1): R^d, the
 * l1 ball or the l2 ball of radius opt->radius centred at 0 (d <= 1024 for
 * the balls); for IHS_L1_PENALTY, argmin over R^d of the same plus
 * opt->radius ||x||_1 (d <= 1024). Only opt->constraint, radius, qp_max_inner
 * and qp_tol are read.
 * x_out may alias x. Synchronises; returns IHS_ERR_NOT_PD when a
 * factorisation meets a non-positive pivot and IHS_ERR_NOT_CONVERGED when a
 * ball QP ends its iteration budget unsolved (x_out then holds x^t).
 * rep (host, nullable) receives status, failed_problem and qp_unpolished
 * (iters = 1; the other fields are 0). */
ihs_status ihs_qp_step(int64_t d, int32_t batch, const double* H,
                       const double* g, const double* x, double* x_out,
                       const ihs_options* opt, void* ws, size_t ws_bytes,
                       hipStream_t stream, ihs_report* rep);

/* The IHS loop (Eq.(2), Thm 2.2): from x^0 = x (device, batch x d; zeros for
 * the usual start) run opt->max_iter steps, writing x^N back to x.
 * x_hist (device, nullable) receives x^1 .. x^N as max_iter x batch x d.
 * factors (device, nullable, needs keep_factors = 1 and the unconstrained
 * case) receives each step's lower Cholesky factor of H, max_iter x batch x
 * d x d, for ihs_adjoint_solve. rep (host) receives the outcome.
 * Synchronises once, at the end. A device error stops further updates of x,
 * which keeps the last good iterate. */
ihs_status ihs_solve(const ihs_matrix* A, const double* b,
                     const ihs_options* opt, double* x, double* x_hist,
                     double* factors, ihs_report* rep,
                     void* ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint of the unconstrained solve (implicit differentiation of the normal
 * equations A^T A x = A^T b): lambda solves A^T A lambda = xbar through the
 * IHS-preconditioned iteration lambda <- lambda + (L_k L_k^T)^{-1}
 * (xbar - A^T A lambda), k = 0 .. n_factors-1, from lambda = 0, reusing the
 * forward's factors in the forward's order. xbar, lambda: device,
 * batch x d. factors: device, as written by ihs_solve. ws from
 * ihs_workspace_size. Asynchronous. */
ihs_status ihs_adjoint_solve(const ihs_matrix* A, const double* xbar,
                             const double* factors, int32_t n_factors,
                             double* lambda, void* ws, size_t ws_bytes,
                             hipStream_t stream);

/* Gradients of a loss L(x) through x = x_OPT(A, b), given lambda from
 * ihs_adjoint_solve: dL/db = A lambda (device, n) and
 * dL/dA = r lambda^T - (A lambda) x^T with r = b - A x (device, float64,
 * n x d, leading dimension ld_da; dense A, F64 or F32). Either output may be
 * NULL.
 * Asynchronous. */
ihs_status ihs_solution_grads(const ihs_matrix* A, const double* b,
                              const double* x, const double* lambda,
                              double* dl_db, double* dl_da, int64_t ld_da,
                              hipStream_t stream);

/* Kernel timing for measurement. While enabled, the library brackets every
 * launch of its sketch-apply pass (the bucket gather over A) with HIP events
 * on the launch stream. ihs_profile_read synchronises those events and
 * returns the number of such launches and their total duration in
 * milliseconds since the last enable. Host only; not thread-safe. */
void ihs_profile_enable(int32_t on);
ihs_status ihs_profile_read(int64_t* launches, double* total_ms);

/* The read ceiling a pass over A is measured against: reads the `bytes`
 * (rounded down to a multiple of 16) of the device buffer `buf` (16-byte
 * aligned) once per repetition, each of up to 8192 workgroups streaming one
 * contiguous chunk with eight 16-byte loads per lane in flight, and returns the average milliseconds per read from HIP events
 * on `stream` (after one untimed read). The buffer is not modified while it
 * holds finite values. Synchronises; host only otherwise. */
ihs_status ihs_profile_read_ceiling(const void* buf, int64_t bytes, int32_t reps,
                                    double* ms_per_read, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* IHS_H */
