// Internal launch interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace ihs {

// Row-range and sort-tile layout of one problem of a (possibly ragged) batch.
struct ProbInfo {
  int64_t row0;     // first global row
  int64_t rows;     // number of rows
  int32_t tile0;    // first sort tile
  int32_t ntiles;
  int32_t chunk0;   // first scan chunk
  int32_t nchunks;
  int32_t seg0;     // first row segment of the natural-order passes
  int32_t nseg;
};

// Up to kProbChunk table entries travel by value in one kernel argument.
constexpr int32_t kProbChunk = 48;
struct ProbChunk {
  int32_t first;
  int32_t count;
  ProbInfo p[kProbChunk];
};
hipError_t launch_write_probs(const ProbInfo* host, int32_t batch, ProbInfo* dst,
                              hipStream_t st);

// Everything the sort and gather kernels need about the sketch of one pass.
struct SketchPlan {
  const ProbInfo* probs;   // device, batch entries
  int32_t batch;
  int32_t s;               // blocks
  int64_t m;               // sketch rows per problem
  int64_t m_blk;           // m / s
  uint64_t seed;
  uint64_t iter;
  int32_t tile_rows;       // rows per sort tile
  int32_t tiles_per_chunk;
  int32_t total_tiles;
  int32_t total_chunks;
  int32_t bucket_bits;     // ceil(log2(m))
  int64_t entries;         // n * s
  // workspace arrays
  uint32_t* keys;          // entries: bucket | sign << 31, at row*s + k
  int32_t* tile_count;     // total_tiles * m
  int32_t* chunk_part;     // total_chunks * m
  int32_t* bucket_start;   // batch*m + 1
  uint32_t* perm;          // entries: global row | sign << 31, bucket-sorted
  // nullable, batch*m: border[p*m + j] is the sketch row that position j of
  // problem p stands for in the dense gather with two sketch rows per
  // wavefront (positions 2w, 2w+1 belong to wavefront w); null: position j is
  // sketch row j
  int32_t* border;
};

// Largest block length (m / s) for which the sort pairs long with short
// sketch rows (the ranking costs m_blk^2 comparisons per block).
constexpr int64_t kPairMaxBlock = 8192;

hipError_t launch_sketch_hash(const SketchPlan& p, int64_t n, int32_t problem,
                              int32_t* bucket, int8_t* sign, hipStream_t st);
// after_hash (nullable) is recorded on st once every key is hashed and counted.
hipError_t launch_sort(const SketchPlan& p, hipStream_t st, hipEvent_t after_hash = nullptr);

struct GatherArgs {
  const void* A;           // dense rows
  int32_t a_dtype;         // 0 f64, 1 f32
  int64_t ld;
  int64_t d;
  void* SA;                // (batch*m) x d, ld_sa
  int32_t sa_dtype;        // 0 f64, 1 f32, 2 bf16
  int64_t ld_sa;
  double scale;            // 1/sqrt(s) for s > 1, else 1
  // fused gradient (nullable b => no gradient)
  const double* b;
  const double* x;         // batch x d
  double* gpart;           // batch * m_blk * d
  double* fpart;           // batch * m_blk
  double* r_out;           // n, nullable
  const int32_t* halt;     // nullable: when it reads non-zero the pass is skipped
                           // (the outer loop's tolerance stop)
};
hipError_t launch_sketch_gather(const SketchPlan& p, const GatherArgs& g, hipStream_t st);
// Sketch rows owned by one wavefront of the dense gather (1 or 2).
int32_t gather_rows_per_wave(int64_t m, int32_t batch, int64_t d);

// CSR counterpart of the gather (values f64).
struct CsrGatherArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* values;
  int64_t d;
  void* SA;
  int32_t sa_dtype;
  int64_t ld_sa;
  double scale;
  const double* b;
  const double* x;
  double* gpart;           // batch * m_blk * d
  double* fpart;
  double* r_out;
  const int32_t* halt;     // as in GatherArgs
};
hipError_t launch_sketch_gather_csr(const SketchPlan& p, const CsrGatherArgs& g,
                                    hipStream_t st);

// The dense sketches of Sec. 2 (kind 2: SRHT, kind 3: Gaussian) for one
// problem: SA (m x d, ld_sa, sa_dtype) = S A with the scale applied once.
struct DenseSketchArgs {
  int32_t kind;
  const void* A;           // dense rows (a_dtype 0 f64, 1 f32, leading dim lda),
                           // or the CSR values (f64) when csr
  int32_t a_dtype;
  int64_t lda;
  bool csr;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  int64_t n, d, m;
  double scale;            // 1 / sqrt(m), formed on the host
  void* SA;
  int32_t sa_dtype;
  int64_t ld_sa;
  uint64_t seed, iter;
  int32_t problem;
  double* work;            // dense_sketch_workspace_bytes
};
size_t dense_sketch_workspace_bytes(int32_t kind, int64_t m, int64_t n, int64_t d, bool csr);
hipError_t launch_dense_sketch(const DenseSketchArgs& a, hipStream_t st);

// Reads `bytes` (a multiple of 16, 16-byte aligned) once: the read ceiling.
hipError_t launch_read_probe(const void* buf, int64_t bytes, double* sink, hipStream_t st);

// Natural-order gradient pass over dense rows: segments of seg_rows rows.
hipError_t launch_gradient_rows(const ProbInfo* probs, int32_t batch, int32_t total_seg,
                                int32_t seg_rows, const void* A, int32_t a_dtype,
                                int64_t ld, int64_t d, const double* b, const double* x,
                                double* gpart, double* fpart, double* r_out,
                                hipStream_t st);
hipError_t launch_gradient_rows_csr(const ProbInfo* probs, int32_t batch,
                                    int32_t total_seg, int32_t seg_rows,
                                    const int32_t* row_ptr, const int32_t* col_idx,
                                    const double* values, int64_t d, const double* b,
                                    const double* x, double* gpart, double* fpart,
                                    double* r_out, hipStream_t st);

// g[p][:] = sum over parts w (ascending, fixed tree) of gpart[p][w][:];
// parts_of(p) = nparts_fixed if > 0, else probs[p].nseg (natural-order passes).
// scratch: reduce_scratch_doubles(batch, d) doubles.
size_t reduce_scratch_doubles(int32_t batch, int64_t d);
hipError_t launch_reduce_partials(const double* gpart, const double* fpart,
                                  int32_t batch, int64_t parts_fixed,
                                  const ProbInfo* probs, int64_t d, double* g,
                                  double* f, DeviceStatus* status, int32_t iter,
                                  double* scratch, hipStream_t st);
hipError_t launch_recip_diag(const double* L, int64_t d, int32_t batch, double* rdiag,
                             hipStream_t st);

// Gram H = SA^T SA.
size_t gram_partials_bytes(int64_t m, int64_t d, int32_t batch, int32_t in_dtype,
                           int32_t acc_dtype);
// per_cu (1 .. 4): workgroups per CU the launch may fill; below 4 the Gram
// takes longer but leaves registers for kernels running beside it. The
// partials buffer sized by gram_partials_bytes serves every per_cu.
hipError_t launch_gram(const void* SA, int32_t in_dtype, int64_t m, int64_t d,
                       int64_t ld, int32_t batch, int32_t acc_dtype, double* H,
                       void* partials, hipStream_t st, int32_t per_cu = 4);

// QP step kernels.
struct QpArgs {
  int64_t d;
  int32_t batch;
  int32_t constraint;
  double radius;
  int32_t max_inner;
  double tol;
  const double* H;         // batch x d x d
  const double* g;         // batch x d
  const double* x;         // batch x d
  double* x_out;           // batch x d (may alias x)
  double* L;               // batch x d x d factor workspace / output
  double* work;            // batch x qp_work_doubles(d)
  DeviceStatus* status;
  int32_t iter;
  int32_t warm;            // l2 ball: start the shift from the previous step's root
  const double* rdiag_pre; // l1 ball (nullable): L already holds the factor of H and
                           // this its reciprocal pivots, so the step does not factor H
  const double* hinv_pre;  // l1 ball (nullable): H^{-1} formed elsewhere; the step
                           // then uses neither L nor rdiag_pre, and its polish
                           // uses it too. l1 penalty (nullable): H^{-1} for the
                           // polish only. l2 ball (with trs_pre, warm steps):
                           // (H + mu0 I)^{-1} formed ahead
  const double* trs_pre;   // l2 ball (nullable): the snapshot state of hinv_pre
                           // (mu0 and a norm bound at [4p + 2], [4p + 3])
  const DeviceStatus* pre_status;  // l2 ball, l1 penalty: failures while forming
                                   // hinv_pre (the penalty step then ignores it)
};
// The l2 step's inverse ahead of time: snapshot the shift state of the QP
// workspace `work` (cold: mu = 0), and factor and invert H + mu I at that
// snapshot into L / hinv (linv: d x d scratch; scratch: batch * (64*64 + d);
// rows: batch * d), its shift and norm bound into snap[4p + 2], snap[4p + 3].
hipError_t launch_l2_snapshot(double* work, int64_t d, int32_t batch, double* snap, int32_t cold,
                              hipStream_t st);
hipError_t launch_l2_prefactor(const double* H, int64_t d, int32_t batch, double* snap, double* L,
                               double* hinv, double* linv, double* scratch, double* rows,
                               DeviceStatus* status, int32_t iter, hipStream_t st);
// Terms of the shifted-inverse series the l2 step iterates on.
constexpr int32_t kL2SeriesTerms = 24;
size_t qp_work_doubles(int64_t d, int32_t constraint);
hipError_t launch_qp_step(const QpArgs& a, hipStream_t st);
// The l1-ball, l2-ball and l1-penalty steps (constraint 1, 2, 3); a.work holds
// qp_work_doubles(d, constraint) doubles per problem.
hipError_t launch_qp_constrained(const QpArgs& a, hipStream_t st);

// Cholesky alone (lower factor of each H into L) and the two triangular
// solves applied to a right-hand side: out = in + (L L^T)^{-1} v.
// scratch: batch * (64*64 + d) doubles: the diagonal-block side buffers of
// the blocked path, then the reciprocal pivots 1/L_jj (chol_rdiag).
// trs (nullable): per-problem shift and skip state of the l2-ball iteration
// (trs[4p] replaces `shift`; problems with trs[4p+1] >= 2 are left untouched).
hipError_t launch_cholesky(const double* H, double* L, int64_t d, int32_t batch,
                           DeviceStatus* status, int32_t iter, double shift, double* scratch,
                           hipStream_t st, const double* trs = nullptr);
double* chol_rdiag(double* scratch, int32_t batch);
// H^{-1} = L^{-T} L^{-1} (blocked triangular inverse, then the product).
// Linv: batch x d x d scratch. trs as for launch_cholesky (nullable).
hipError_t launch_chol_inverse(const double* L, const double* rdiag, int64_t d, int32_t batch,
                               double* Hinv, double* Linv, DeviceStatus* status, hipStream_t st,
                               const double* trs = nullptr);
// x_out = x + Hinv g (dx receives Hinv g); records sqrt(dx^T g) of problem 0.
hipError_t launch_inv_apply(const double* Hinv, int64_t d, int32_t batch, const double* g,
                            const double* x, double* x_out, double* dx, DeviceStatus* status,
                            hipStream_t st, const DeviceStatus* gate, int32_t gate_iter);
// Skips the update (out = base) when `status` records any failure or `gate`
// (nullable, another stream's record) a failure at or before step gate_iter.
hipError_t launch_chol_solve_update(const double* L, const double* rdiag, int64_t d,
                                    int32_t batch, const double* v, const double* base,
                                    double* out, DeviceStatus* status, hipStream_t st,
                                    const DeviceStatus* gate = nullptr,
                                    int32_t gate_iter = -1);

// The outer loop's tolerance stop after step `iter`: q_p = dx^T H dx per
// problem (H: batch x d x d, or nullptr to use dx^T g), dx = x - xprev; sets
// status->done and status->iters = iter + 1 when no failure is recorded and
// every sqrt(q_p) <= tol. q: batch x d scratch. Records sqrt(q_0) as
// status->last_step.
hipError_t launch_step_test(const double* H, const double* g, const double* xprev,
                            const double* x, int64_t d, int32_t batch, double tol, double* q,
                            DeviceStatus* status, int32_t iter, hipStream_t st);

// Conjugate gradients preconditioned by a fixed Hessian sketch (pm = -p):
// begin: rho = r^T z, pm = -z; x: alpha = rho / p^T q, x += alpha p,
// r -= alpha q; p: rho' = r^T z, pm = -z + (rho'/rho) pm, rho = rho'.
hipError_t launch_pcg_begin(const double* r, const double* z, double* pm, double* rho, int64_t d,
                            int32_t batch, const DeviceStatus* status, hipStream_t st);
hipError_t launch_pcg_x(const double* pm, const double* q, const double* rho, double* x,
                        double* r, int64_t d, int32_t batch, DeviceStatus* status, int32_t iter,
                        hipStream_t st);
hipError_t launch_pcg_p(const double* r, const double* z, double* pm, double* rho, int64_t d,
                        int32_t batch, const DeviceStatus* status, hipStream_t st);

// Adjoint and solution-gradient passes.
// S^T G for the nrows rows of one problem (G points at that problem's m rows).
// Rows [off[0], off[count]) of problems first .. first+count-1 (global row
// offsets; problem p's rows start at off[p - first]).
constexpr int kAdjointBatch = 64;
struct AdjointBatch {
  int64_t off[kAdjointBatch + 1];
  int32_t count;
  int32_t first;
};
// out = S^T G for those rows; G points at problem `first`'s m x d block.
hipError_t launch_sketch_adjoint(const AdjointBatch& ab, int32_t s, int64_t m, uint64_t seed,
                                 uint64_t iter, const double* G, int64_t ld_g, int64_t d,
                                 double* out, int64_t ld_out, hipStream_t st);
// dL/db and dL/dA for the rows of problems first .. first+count-1 (global
// row indices into A, b, dl_db, dl_da; x and lambda indexed by problem).
hipError_t launch_solution_grads(const AdjointBatch& ab, int64_t d, const void* A, bool a_f32,
                                 int64_t ld, const double* b, const double* x,
                                 const double* lambda, double* dl_db, double* dl_da,
                                 int64_t ld_da, hipStream_t st);

}  // namespace ihs
