// libihs C ABI: argument validation, workspace carving and the IHS loop.
// Declarations and their contracts live in include/ihs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/ihs.h"
#include "kernels.hpp"
#include "rowdot.hpp"

using namespace ihs;

namespace {

constexpr int64_t kMaxSketchRows = 16384;  // per problem: 64 KiB LDS histogram
constexpr int64_t kMaxDenseD = 1024;       // register-resident row slices
constexpr int64_t kMaxCsrD = 1024;         // LDS-resident bucket rows (64 KiB)
constexpr int32_t kSegRows = 512;          // rows per wavefront, natural-order passes
constexpr int32_t kTilesPerChunk = 32;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// The HIP error behind the most recent IHS_ERR_HIP returned on this thread.
thread_local int32_t t_last_hip_error = 0;

// True, and recorded for ihs_last_hip_error, when e reports a failure.
bool hip_failed(hipError_t e) {
  if (e == hipSuccess) return false;
  t_last_hip_error = (int32_t)e;
  return true;
}

ihs_status hip_status(hipError_t e) { return hip_failed(e) ? IHS_ERR_HIP : IHS_OK; }

// Drops an error that earlier HIP calls of the caller left pending on this
// thread, so that the checks after this library's own launches see only
// theirs. Called once argument checks pass, before the first launch.
void clear_stale_error() { (void)hipGetLastError(); }

// Bump allocator over the caller's workspace (or a size count when base is null).
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    used = align_up(used, 256);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

int64_t dtype_size(int32_t dt) { return dt == IHS_F64 ? 8 : (dt == IHS_F32 ? 4 : 2); }

// The Gaussian and SRHT sketches (dense S) against the sparse embeddings.
bool dense_kind(const ihs_sketch* sk) { return sk->kind == IHS_SRHT || sk->kind == IHS_GAUSSIAN; }

bool valid_sketch(const ihs_sketch* sk) {
  if (!sk) return false;
  if (sk->kind != IHS_COUNTSKETCH && sk->kind != IHS_SJLT && !dense_kind(sk)) return false;
  if (sk->m < 1 || sk->s < 1) return false;
  if (sk->kind != IHS_SJLT && sk->s != 1) return false;
  if (sk->m % sk->s != 0) return false;
  return true;
}

ihs_status check_sketch(const ihs_sketch* sk) {
  if (!valid_sketch(sk)) return IHS_ERR_INVALID_ARG;
  if (sk->m > kMaxSketchRows) return IHS_ERR_UNSUPPORTED;
  return IHS_OK;
}

// Problem table of a matrix (host copy).
struct Layout {
  std::vector<ProbInfo> probs;
  bool csr = false;
  int32_t batch = 1;
  int64_t n = 0, d = 0;
  int32_t tile_rows = 256;
  int32_t total_tiles = 0, total_chunks = 0, total_seg = 0;
};

ihs_status check_matrix(const ihs_matrix* A) {
  if (!A) return IHS_ERR_INVALID_ARG;
  if (A->n < 0 || A->d < 1 || A->batch < 1) return IHS_ERR_INVALID_ARG;
  if (A->n >= (int64_t(1) << 31)) return IHS_ERR_UNSUPPORTED;
  if (A->format == IHS_DENSE) {
    if (A->dtype != IHS_F64 && A->dtype != IHS_F32) return IHS_ERR_INVALID_ARG;
    if (A->ld < A->d) return IHS_ERR_INVALID_ARG;
    if (A->n > 0 && !A->values) return IHS_ERR_INVALID_ARG;
    if (A->d > kMaxDenseD) return IHS_ERR_UNSUPPORTED;
    // beyond 512 columns rows are read as aligned pairs
    if (A->d > 512 && (A->d % 2 != 0 || A->ld % 2 != 0 ||
                       reinterpret_cast<uintptr_t>(A->values) % (2 * (A->dtype == IHS_F64 ? 8 : 4)) != 0))
      return IHS_ERR_UNSUPPORTED;
  } else if (A->format == IHS_CSR) {
    if (A->dtype != IHS_F64) return IHS_ERR_INVALID_ARG;
    if (A->nnz < 0 || !A->row_ptr) return IHS_ERR_INVALID_ARG;
    if (A->nnz > 0 && (!A->col_idx || !A->values)) return IHS_ERR_INVALID_ARG;
    if (A->nnz >= (int64_t(1) << 31)) return IHS_ERR_UNSUPPORTED;
    if (A->d > kMaxCsrD) return IHS_ERR_UNSUPPORTED;
  } else {
    return IHS_ERR_INVALID_ARG;
  }
  if (A->batch > 1) {
    if (!A->row_offsets) return IHS_ERR_INVALID_ARG;
    if (A->row_offsets[0] != 0 || A->row_offsets[A->batch] != A->n) return IHS_ERR_INVALID_ARG;
    for (int32_t p = 0; p < A->batch; ++p)
      if (A->row_offsets[p + 1] < A->row_offsets[p]) return IHS_ERR_INVALID_ARG;
  }
  return IHS_OK;
}

Layout make_layout(const ihs_matrix* A, int64_t m_local) {
  Layout L;
  L.csr = A->format == IHS_CSR;
  L.batch = A->batch;
  L.n = A->n;
  L.d = A->d;
  int64_t tr = std::max<int64_t>(m_local, (A->n + 1023) / 1024);
  tr = std::max<int64_t>(256, align_up((size_t)tr, 256));
  L.tile_rows = (int32_t)std::min<int64_t>(tr, int64_t(1) << 20);
  L.probs.resize(A->batch);
  int32_t tile = 0, chunk = 0, seg = 0;
  for (int32_t p = 0; p < A->batch; ++p) {
    ProbInfo& q = L.probs[p];
    q.row0 = A->batch > 1 ? A->row_offsets[p] : 0;
    q.rows = A->batch > 1 ? A->row_offsets[p + 1] - A->row_offsets[p] : A->n;
    q.tile0 = tile;
    q.ntiles = (int32_t)((q.rows + L.tile_rows - 1) / L.tile_rows);
    q.chunk0 = chunk;
    q.nchunks = (q.ntiles + kTilesPerChunk - 1) / kTilesPerChunk;
    q.seg0 = seg;
    q.nseg = (int32_t)((q.rows + kSegRows - 1) / kSegRows);
    tile += q.ntiles;
    chunk += q.nchunks;
    seg += q.nseg;
  }
  L.total_tiles = tile;
  L.total_chunks = chunk;
  L.total_seg = seg;
  return L;
}

// Device arrays of one sketch pass (sort + gather + gradient partials).
struct PassBuffers {
  ProbInfo* probs = nullptr;
  DeviceStatus* status = nullptr;
  uint32_t* keys = nullptr;
  int32_t* tile_count = nullptr;
  int32_t* chunk_part = nullptr;
  int32_t* bucket_start = nullptr;
  uint32_t* perm = nullptr;
  int32_t* border = nullptr;  // pairing of long with short sketch rows (dense gather)
  double* gpart = nullptr;
  double* fpart = nullptr;
  double* g = nullptr;
  double* f = nullptr;
  double* bzero = nullptr;
  double* red = nullptr;   // two-level reduction scratch
  double* rdiag = nullptr; // batch x d reciprocal pivots (adjoint path)
  const int32_t* halt = nullptr;  // &status->done while a solve may stop early
  bool profile = true;            // false: never create timing events
};

void carve_pass(Carver& c, const Layout& L, const ihs_sketch* sk, PassBuffers& B) {
  const int64_t m = sk ? sk->m : 1;
  const int64_t s = sk ? sk->s : 1;
  const int64_t m_blk = m / s;
  const int64_t entries = L.n * s;
  B.probs = c.take<ProbInfo>(L.batch);
  B.status = c.take<DeviceStatus>(1);
  B.keys = c.take<uint32_t>((size_t)std::max<int64_t>(entries, 1));
  B.tile_count = c.take<int32_t>((size_t)std::max<int64_t>((int64_t)L.total_tiles * m, 1));
  B.chunk_part = c.take<int32_t>((size_t)std::max<int64_t>((int64_t)L.total_chunks * m, 1));
  B.bucket_start = c.take<int32_t>((size_t)(L.batch * m + 1));
  B.perm = c.take<uint32_t>((size_t)std::max<int64_t>(entries, 1));
  B.border = c.take<int32_t>((size_t)(L.batch * m));
  const int64_t parts = std::max<int64_t>((int64_t)L.batch * m_blk, L.total_seg);
  B.gpart = c.take<double>((size_t)std::max<int64_t>(parts * L.d, 1));
  B.fpart = c.take<double>((size_t)std::max<int64_t>(parts, 1));
  B.g = c.take<double>((size_t)(L.batch * L.d));
  B.f = c.take<double>((size_t)L.batch);
  B.bzero = c.take<double>((size_t)std::max<int64_t>(L.n, 1));
  B.red = c.take<double>(reduce_scratch_doubles(L.batch, L.d));
  B.rdiag = c.take<double>((size_t)(L.batch * L.d));
}

// The arrays a sketch-only pass (sort + gather, no gradient) uses, for the
// allocation-free entry point: the others of carve_pass stay null.
void carve_sketch_only(Carver& c, const Layout& L, const ihs_sketch* sk, PassBuffers& B) {
  const int64_t m = sk->m;
  const int64_t entries = L.n * sk->s;
  B.probs = c.take<ProbInfo>(L.batch);
  B.status = c.take<DeviceStatus>(1);
  B.keys = c.take<uint32_t>((size_t)std::max<int64_t>(entries, 1));
  B.tile_count = c.take<int32_t>((size_t)std::max<int64_t>((int64_t)L.total_tiles * m, 1));
  B.chunk_part = c.take<int32_t>((size_t)std::max<int64_t>((int64_t)L.total_chunks * m, 1));
  B.bucket_start = c.take<int32_t>((size_t)(L.batch * m + 1));
  B.perm = c.take<uint32_t>((size_t)std::max<int64_t>(entries, 1));
  B.border = c.take<int32_t>((size_t)(L.batch * m));
}

// ---- the allocation-free sketch apply ----
// One file-scope device array serves every call of ihs_sketch_apply_static
// on a GPU; each device holds its own copy, at its own address, found once per
// device with hipGetSymbolAddress. In host code `scratch` names a host-side
// stand-in, so only the looked-up addresses are ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[IHS_STATIC_SCRATCH_BYTES];

// The device address of `scratch` on the current device (nullptr when the
// lookup fails; the failure is recorded for ihs_last_hip_error).
void* static_scratch_address() {
  static std::mutex mu;
  static std::vector<void*> addr;
  int dev = 0;
  if (hip_failed(hipGetDevice(&dev))) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (addr.size() <= (size_t)dev) addr.resize((size_t)dev + 1, nullptr);
  if (!addr[(size_t)dev]) {
    void* p = nullptr;
    if (hip_failed(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)))) return nullptr;
    addr[(size_t)dev] = p;
  }
  return addr[(size_t)dev];
}

// Gradient partials written by one sketch pass: one per wavefront that owns
// sketch rows of block 0 (dense), one per sketch row of block 0 (CSR).
int64_t pass_parts(const ihs_matrix* A, const ihs_sketch* sk, int32_t batch) {
  const int64_t m_blk = sk->m / sk->s;
  if (A->format != IHS_DENSE) return m_blk;
  const int64_t bpw = gather_rows_per_wave(sk->m, batch, A->d);
  return (m_blk + bpw - 1) / bpw;
}

SketchPlan make_plan(const Layout& L, const ihs_sketch* sk, const PassBuffers& B, uint64_t iter) {
  SketchPlan P{};
  P.probs = B.probs;
  P.batch = L.batch;
  P.s = sk->s;
  P.m = sk->m;
  P.m_blk = sk->m / sk->s;
  P.seed = sk->seed;
  P.iter = iter;
  P.tile_rows = L.tile_rows;
  P.tiles_per_chunk = kTilesPerChunk;
  P.total_tiles = L.total_tiles;
  P.total_chunks = L.total_chunks;
  int32_t bits = 0;
  while ((int64_t(1) << bits) < sk->m) ++bits;
  P.bucket_bits = bits;
  P.entries = L.n * sk->s;
  P.keys = B.keys;
  P.tile_count = B.tile_count;
  P.chunk_part = B.chunk_part;
  P.bucket_start = B.bucket_start;
  P.perm = B.perm;
  const bool paired = !L.csr && gather_rows_per_wave(sk->m, L.batch, L.d) == 2 &&
                      P.m_blk <= kPairMaxBlock;
  P.border = paired ? B.border : nullptr;
  return P;
}

// Carries a failure that another stream recorded at or before step `iter`
// into `to`, so that the kernels reading `to` in that step see it.
__global__ void k_adopt_status(const DeviceStatus* from, int32_t iter, DeviceStatus* to) {
  // after the tolerance stop the other stream works on sketches no step uses
  if (threadIdx.x == 0 && !to->done && status_failed_by(from, iter))
    status_fail(to, from->code, from->failed_iter, from->failed_problem);
}

__global__ void k_zero_status(DeviceStatus* st) {
  if (threadIdx.x == 0) {
    st->code = 0;
    st->failed_iter = -1;
    st->failed_problem = -1;
    st->done = 0;
    st->iters = 0;
    st->claim = 0;
    st->unpolished = 0;
    st->objective = 0.0;
    st->last_step = 0.0;
  }
}

__global__ void k_fill(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_add(const double* a, const double* b, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

hipError_t fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

ihs_status upload_probs(const Layout& L, PassBuffers& B, hipStream_t st) {
  if (hip_failed(launch_write_probs(L.probs.data(), L.batch, B.probs, st))) return IHS_ERR_HIP;
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, B.status);
  return hip_status(hipGetLastError());
}

// ---- profiling of the gather pass ----
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
} g_prof;

void prof_begin(hipStream_t st, hipEvent_t* a) {
  *a = nullptr;
  if (!g_prof.on) return;
  if (hip_failed(hipEventCreate(a))) {
    *a = nullptr;
    return;
  }
  (void)hipEventRecord(*a, st);
}

void prof_end(hipStream_t st, hipEvent_t a) {
  if (!a) return;
  hipEvent_t b;
  if (hip_failed(hipEventCreate(&b))) return;
  (void)hipEventRecord(b, st);
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.ev.emplace_back(a, b);
}

// One sketch pass: sort by the hash of (seed, iter), then gather (with the
// fused gradient when x != nullptr).
ihs_status run_gather(const ihs_matrix* A, const ihs_sketch* sk, const PassBuffers& B,
                      const SketchPlan& P, void* SA, int32_t sa_dtype, int64_t ld_sa,
                      const double* b, const double* x, double* r_out, hipStream_t st);

ihs_status run_pass(const ihs_matrix* A, const Layout& L, const ihs_sketch* sk,
                    const PassBuffers& B, uint64_t iter, void* SA, int32_t sa_dtype,
                    int64_t ld_sa, const double* b, const double* x, double* r_out,
                    hipStream_t st) {
  SketchPlan P = make_plan(L, sk, B, iter);
  if (hip_failed(launch_sort(P, st))) return IHS_ERR_HIP;
  return run_gather(A, sk, B, P, SA, sa_dtype, ld_sa, b, x, r_out, st);
}

// The gather over A for an already sorted sketch.
ihs_status run_gather(const ihs_matrix* A, const ihs_sketch* sk, const PassBuffers& B,
                      const SketchPlan& P, void* SA, int32_t sa_dtype, int64_t ld_sa,
                      const double* b, const double* x, double* r_out, hipStream_t st) {
  const double scale = sk->s > 1 ? 1.0 / std::sqrt((double)sk->s) : 1.0;
  hipEvent_t e0 = nullptr;
  if (B.profile) prof_begin(st, &e0);
  hipError_t err;
  if (A->format == IHS_DENSE) {
    GatherArgs G{};
    G.A = A->values;
    G.a_dtype = A->dtype;
    G.ld = A->ld;
    G.d = A->d;
    G.SA = SA;
    G.sa_dtype = sa_dtype;
    G.ld_sa = ld_sa;
    G.scale = scale;
    G.b = x ? (b ? b : B.bzero) : nullptr;
    G.x = x;
    G.gpart = B.gpart;
    G.fpart = B.fpart;
    G.r_out = r_out;
    G.halt = B.halt;
    err = launch_sketch_gather(P, G, st);
  } else {
    CsrGatherArgs G{};
    G.row_ptr = A->row_ptr;
    G.col_idx = A->col_idx;
    G.values = static_cast<const double*>(A->values);
    G.d = A->d;
    G.SA = SA;
    G.sa_dtype = sa_dtype;
    G.ld_sa = ld_sa;
    G.scale = scale;
    G.b = x ? (b ? b : B.bzero) : nullptr;
    G.x = x;
    G.gpart = B.gpart;
    G.fpart = B.fpart;
    G.r_out = r_out;
    G.halt = B.halt;
    err = launch_sketch_gather_csr(P, G, st);
  }
  prof_end(st, e0);
  return hip_status(err);
}

// S A for the Gaussian or SRHT sketch of key (seed, iter) (one problem).
ihs_status run_dense_sketch(const ihs_matrix* A, const ihs_sketch* sk, uint64_t iter, void* SA,
                            int32_t sa_dtype, int64_t ld_sa, double* work, hipStream_t st) {
  DenseSketchArgs a{};
  a.kind = sk->kind;
  a.A = A->values;
  a.a_dtype = A->dtype;
  a.lda = A->ld;
  a.csr = A->format == IHS_CSR;
  a.row_ptr = A->row_ptr;
  a.col_idx = A->col_idx;
  a.n = A->n;
  a.d = A->d;
  a.m = sk->m;
  a.scale = 1.0 / std::sqrt((double)sk->m);
  a.SA = SA;
  a.sa_dtype = sa_dtype;
  a.ld_sa = ld_sa;
  a.seed = sk->seed;
  a.iter = iter;
  a.problem = 0;
  a.work = work;
  return hip_status(launch_dense_sketch(a, st));
}

// Natural-order gradient pass + reduction into B.g / B.f.
ihs_status run_gradient(const ihs_matrix* A, const Layout& L, const PassBuffers& B,
                        const double* b, const double* x, double* g, double* f, double* r_out,
                        DeviceStatus* status, int32_t iter, hipStream_t st) {
  hipError_t err;
  const double* bb = b ? b : B.bzero;
  if (A->format == IHS_DENSE) {
    err = launch_gradient_rows(B.probs, L.batch, L.total_seg, kSegRows, A->values, A->dtype,
                               A->ld, A->d, bb, x, B.gpart, B.fpart, r_out, st);
  } else {
    err = launch_gradient_rows_csr(B.probs, L.batch, L.total_seg, kSegRows, A->row_ptr,
                                   A->col_idx, static_cast<const double*>(A->values), A->d, bb,
                                   x, B.gpart, B.fpart, r_out, st);
  }
  if (hip_failed(err)) return IHS_ERR_HIP;
  if (L.total_seg == 0) {
    if (hip_failed(fill(g, (int64_t)L.batch * L.d, 0.0, st))) return IHS_ERR_HIP;
    if (f && hip_failed(fill(f, L.batch, 0.0, st))) return IHS_ERR_HIP;
    return IHS_OK;
  }
  err = launch_reduce_partials(B.gpart, B.fpart, L.batch, 0, B.probs, L.d, g, f, status, iter,
                               B.red, st);
  return hip_status(err);
}

struct SolveBuffers {
  PassBuffers pass;
  void* SA = nullptr;
  double* H = nullptr;
  void* gram_part = nullptr;
  double* H1 = nullptr;      // second (and third) sketched Hessian of the overlapped
  double* H2 = nullptr;      // constrained schedule
  double* Lf = nullptr;
  double* work = nullptr;
  // second set of the double-buffered arrays of the overlapped schedule
  uint32_t* perm1 = nullptr;
  int32_t* bstart1 = nullptr;
  int32_t* border1 = nullptr;
  void* SA1 = nullptr;
  double* Lf1 = nullptr;
  double* work1 = nullptr;
  // third set, when the overlapped schedule looks two steps ahead
  void* SA2 = nullptr;
  double* Lf2 = nullptr;
  double* work2 = nullptr;
  DeviceStatus* side_status = nullptr;
  double* Hinv0 = nullptr;   // explicit inverses of the overlapped schedule
  double* Hinv1 = nullptr;
  double* Hinv2 = nullptr;
  double* Linv = nullptr;    // triangular-inverse scratch of the second stream
  // the l1 penalty's inverses (overlapped schedule, from kInverseMinD on) serve
  // only its KKT polish; failures while forming them are kept here, apart
  // from the solve's status, and make the step polish without them
  DeviceStatus* inv_status = nullptr;
  double* dx = nullptr;
  // conjugate gradients with a fixed sketch: residual A^T (b - A x), its
  // preconditioned copy, -p, r^T z per problem, and a zero vector
  double* cg_r = nullptr;
  double* cg_z = nullptr;
  double* cg_pm = nullptr;
  double* cg_rho = nullptr;
  double* cg_zero = nullptr;
  // the tolerance stop: x^t before each update, and per-row products
  double* xprev = nullptr;
  double* stepq = nullptr;
  double* dsk = nullptr;     // the Gaussian or SRHT sketch's own scratch
  // the l2 step's inverse formed ahead (overlapped schedule), two steps ahead
  // on two side streams: per stream a Gram partial buffer, the factor and the
  // factorisation's scratch; per step (three in flight) the shift snapshot;
  // one status record for failures while forming them
  void* gram_part1 = nullptr;
  double* Linv1 = nullptr;
  double* Lpre[2] = {nullptr, nullptr};
  double* pre_scratch[2] = {nullptr, nullptr};
  double* pre_rows[2] = {nullptr, nullptr};
  double* snap[3] = {nullptr, nullptr, nullptr};
  DeviceStatus* pre_status = nullptr;
};

// From kQpInverseMinD (rowdot.hpp) on, the overlapped schedule forms H^{-1}
// on the second stream and the critical path only applies it; below, the
// triangular solves run on the main stream directly. One constant serves the
// standalone step, the ball steps and both schedules.
constexpr int64_t kInverseMinD = kQpInverseMinD;

int32_t gram_in_of(const ihs_options* o) { return o ? o->gram_in : IHS_F64; }
int32_t gram_acc_of(const ihs_options* o) { return o ? o->gram_acc : IHS_F64; }

size_t carve_solve(Carver& c, const Layout& L, const ihs_options* o, SolveBuffers& S) {
  carve_pass(c, L, &o->sketch, S.pass);
  const int64_t m = o->sketch.m;
  S.SA = c.take<char>((size_t)(L.batch * m * L.d * dtype_size(gram_in_of(o))));
  S.H = c.take<double>((size_t)(L.batch * L.d * L.d));
  S.gram_part = c.take<char>(
      gram_partials_bytes(m, L.d, L.batch, gram_in_of(o), gram_acc_of(o)));
  S.Lf = c.take<double>((size_t)(L.batch * L.d * L.d));
  S.work = c.take<double>((size_t)L.batch * qp_work_doubles(L.d, o->constraint));
  const int64_t entries = L.n * o->sketch.s;
  S.perm1 = c.take<uint32_t>((size_t)std::max<int64_t>(entries, 1));
  S.bstart1 = c.take<int32_t>((size_t)(L.batch * m + 1));
  S.border1 = c.take<int32_t>((size_t)(L.batch * m));
  S.SA1 = c.take<char>((size_t)(L.batch * m * L.d * dtype_size(gram_in_of(o))));
  S.Lf1 = c.take<double>((size_t)(L.batch * L.d * L.d));
  S.work1 = c.take<double>((size_t)L.batch * qp_work_doubles(L.d, o->constraint));
  S.side_status = c.take<DeviceStatus>(1);
  if (o->constraint != IHS_UNCONSTRAINED && o->schedule != 1)
    S.H1 = c.take<double>((size_t)(L.batch * L.d * L.d));
  const bool l2pre = o->constraint == IHS_L2_BALL && o->schedule != 1;
  const bool ahead2 = (o->schedule == 2 && o->constraint == IHS_UNCONSTRAINED) || l2pre;
  if (ahead2) {
    S.SA2 = c.take<char>((size_t)(L.batch * m * L.d * dtype_size(gram_in_of(o))));
    if (!l2pre) {  // the l2 step's side work keeps its factors apart (Lpre)
      S.Lf2 = c.take<double>((size_t)(L.batch * L.d * L.d));
      S.work2 = c.take<double>((size_t)L.batch * qp_work_doubles(L.d, o->constraint));
    }
  }
  if (l2pre) {
    const size_t bdd = (size_t)(L.batch * L.d * L.d);
    S.H2 = c.take<double>(bdd);
    S.gram_part1 = c.take<char>(
        gram_partials_bytes(m, L.d, L.batch, gram_in_of(o), gram_acc_of(o)));
    S.Linv1 = c.take<double>(bdd);
    for (int q = 0; q < 2; ++q) {
      S.Lpre[q] = c.take<double>(bdd);
      S.pre_scratch[q] = c.take<double>((size_t)L.batch * (64 * 64 + L.d));
      S.pre_rows[q] = c.take<double>((size_t)(L.batch * L.d));
    }
    for (int q = 0; q < 3; ++q) S.snap[q] = c.take<double>((size_t)(4 * L.batch));
    S.pre_status = c.take<DeviceStatus>(1);
  }
  const bool pen_inv =
      L.d >= kInverseMinD && o->constraint == IHS_L1_PENALTY && o->schedule != 1;
  if ((L.d >= kInverseMinD &&
       (o->constraint == IHS_UNCONSTRAINED || o->constraint == IHS_L1_BALL)) || l2pre ||
      pen_inv) {
    S.Hinv0 = c.take<double>((size_t)(L.batch * L.d * L.d));
    S.Hinv1 = c.take<double>((size_t)(L.batch * L.d * L.d));
    if (ahead2) S.Hinv2 = c.take<double>((size_t)(L.batch * L.d * L.d));
    S.Linv = c.take<double>((size_t)(L.batch * L.d * L.d));
  }
  if (pen_inv) S.inv_status = c.take<DeviceStatus>(1);
  S.dx = c.take<double>((size_t)(L.batch * L.d));
  if (o->method == IHS_METHOD_FIXED_SKETCH_CG) {
    const size_t bd = (size_t)(L.batch * L.d);
    S.cg_r = c.take<double>(bd);
    S.cg_z = c.take<double>(bd);
    S.cg_pm = c.take<double>(bd);
    S.cg_rho = c.take<double>((size_t)L.batch);
    S.cg_zero = c.take<double>(bd);
  }
  if (o->tol > 0.0) {
    S.xprev = c.take<double>((size_t)(L.batch * L.d));
    S.stepq = c.take<double>((size_t)(L.batch * L.d));
  }
  if (dense_kind(&o->sketch))
    S.dsk = c.take<double>(dense_sketch_workspace_bytes(o->sketch.kind, m, L.n, L.d, L.csr) /
                           sizeof(double));
  return c.used;
}

// ---- the extra streams of the overlapped schedule (kept per device) ----
// which = 0: Gram / factorisation / inverse; which = 1: bucket sorts;
// which = 2: the second Gram / factorisation / inverse stream (l2 ball).
hipStream_t side_stream(int which) {
  static std::mutex mu;
  static std::vector<hipStream_t> streams;
  int dev = 0;
  if (hip_failed(hipGetDevice(&dev))) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  const size_t slot = (size_t)dev * 3 + (size_t)which;
  if (streams.size() <= slot) streams.resize(slot + 1, nullptr);
  if (!streams[slot]) {
    hipStream_t s = nullptr;
    if (hip_failed(hipStreamCreateWithFlags(&s, hipStreamNonBlocking))) return nullptr;
    streams[slot] = s;
  }
  return streams[slot];
}

// A ring of timing-free events; a slot is re-recorded only after every wait
// on its previous record has been enqueued.
struct EventRing {
  std::vector<hipEvent_t> ev;
  bool ok = true;
  explicit EventRing(int n) : ev(n, nullptr) {
    for (auto& e : ev)
      if (hip_failed(hipEventCreateWithFlags(&e, hipEventDisableTiming))) ok = false;
  }
  ~EventRing() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  hipEvent_t at(int64_t i) { return ev[(size_t)(((i % (int64_t)ev.size()) + ev.size()) % ev.size())]; }
};

// Balls need a positive radius; the penalty a finite weight >= 0.
bool valid_constraint(int32_t c, double radius) {
  if (c == IHS_UNCONSTRAINED) return true;
  if (c == IHS_L1_BALL || c == IHS_L2_BALL) return radius > 0.0 && std::isfinite(radius);
  if (c == IHS_L1_PENALTY) return radius >= 0.0 && std::isfinite(radius);
  return false;
}

bool valid_gram_types(int32_t in, int32_t acc) {
  if (in == IHS_F64) return acc == IHS_F64;
  if (in == IHS_F32) return acc == IHS_F64 || acc == IHS_F32;
  if (in == IHS_BF16) return acc == IHS_F32;
  return false;
}

ihs_status check_options(const ihs_options* o, bool need_loop) {
  if (!o) return IHS_ERR_INVALID_ARG;
  ihs_status s = check_sketch(&o->sketch);
  if (s != IHS_OK) return s;
  if (!valid_constraint(o->constraint, o->radius)) return IHS_ERR_INVALID_ARG;
  if (need_loop && o->max_iter < 1) return IHS_ERR_INVALID_ARG;
  if (!valid_gram_types(o->gram_in, o->gram_acc)) return IHS_ERR_INVALID_ARG;
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol) || o->qp_tol < 0.0 || o->qp_max_inner < 0)
    return IHS_ERR_INVALID_ARG;
  if (o->schedule < 0 || o->schedule > 2) return IHS_ERR_INVALID_ARG;
  if (o->method != IHS_METHOD_IHS && o->method != IHS_METHOD_FIXED_SKETCH_CG)
    return IHS_ERR_INVALID_ARG;
  if (o->method == IHS_METHOD_FIXED_SKETCH_CG &&
      (o->constraint != IHS_UNCONSTRAINED || o->tol > 0.0))
    return IHS_ERR_UNSUPPORTED;
  return IHS_OK;
}

ihs_status read_status(DeviceStatus* dev, DeviceStatus* host, hipStream_t st) {
  if (hip_failed(hipMemcpyAsync(host, dev, sizeof(DeviceStatus), hipMemcpyDeviceToHost, st)))
    return IHS_ERR_HIP;
  if (hip_failed(hipStreamSynchronize(st))) return IHS_ERR_HIP;
  return IHS_OK;
}

// The outcome of a solve from its failure record f and the main stream's
// record m: a failure names its step and keeps the last good iterate; with
// tol > 0 the solve either stopped at m.iters steps or ran all max_iter steps
// without meeting tol (IHS_ERR_NOT_CONVERGED, x holds x^N).
ihs_status finish_report(const DeviceStatus& f, const DeviceStatus& m, const ihs_options* opt,
                         ihs_report* rep) {
  int32_t code = f.code;
  if (code == IHS_OK && opt->tol > 0.0 && !m.done) code = IHS_ERR_NOT_CONVERGED;
  if (rep) {
    *rep = ihs_report{};
    rep->status = code;
    rep->failed_iter = f.code ? f.failed_iter : -1;
    rep->failed_problem = f.code ? f.failed_problem : -1;
    rep->iters = f.code ? std::max(0, f.failed_iter) : (m.done ? m.iters : opt->max_iter);
    rep->objective = m.objective;
    rep->last_step = m.last_step;
    rep->qp_unpolished = m.unpolished;
  }
  return (ihs_status)code;
}

// The overlapped schedule of the IHS loop (unconstrained problems). Step t
// needs the factor of H_t = (S_t A)^T (S_t A) and g(x^t); since S_t does not
// depend on x, the pass that forms g(x^t) also forms S_{t+LA} A (LA = 1, or 2
// for schedule 2), a sorter stream sorts rows for the sketch after that, and
// a side stream forms H_{t+LA}, factors it and (for wider problems) inverts
// it during the next LA passes, so the step itself only applies H_t^{-1} to
// g. LA sketch-only passes first form S_0 A .. S_{LA-1} A. Looking two steps
// ahead gives the side stream two passes of time, for passes that are short
// against the factorisation (float32 data), at the price of one more
// sketch-only pass.
// Sketches and factors are bitwise those of the sequential loop; g(x^t) is
// summed in the row order of S_{t+LA} instead of S_t, and H_t^{-1} g is a
// product with the explicit inverse, so iterates agree with the sequential
// loop to rounding.
// A host thread that queues the side stream's work (a Gram, a factorisation
// and an inverse: some sixty launches per step) in order, so that the thread
// that runs the step never waits for those launches before its own. Jobs
// return false when a launch fails; every later job is then skipped. The
// destructor drops jobs not yet started and joins the thread.
class SideQueue {
 public:
  explicit SideQueue(int device) : dev_(device), th_([this] { loop(); }) {}
  ~SideQueue() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    th_.join();
  }
  // returns the job's number (1, 2, ...)
  int64_t post(std::function<bool()> f) {
    std::lock_guard<std::mutex> lk(mu_);
    q_.push_back(std::move(f));
    cv_.notify_all();
    return ++posted_;
  }
  // waits until job n (and every earlier one) has run; false if any failed
  bool wait(int64_t n) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return done_ >= n; });
    return ok_;
  }
  bool drain() {
    int64_t n;
    {
      std::lock_guard<std::mutex> lk(mu_);
      n = posted_;
    }
    return wait(n);
  }

 private:
  void loop() {
    const bool dev_ok = !hip_failed(hipSetDevice(dev_));
    for (;;) {
      std::function<bool()> f;
      bool run;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
        if (stop_) return;
        f = std::move(q_.front());
        q_.pop_front();
        run = ok_ && dev_ok;
      }
      const bool r = run && f();
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (!r) ok_ = false;
        ++done_;
      }
      cv_.notify_all();
    }
  }
  int dev_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::function<bool()>> q_;
  int64_t posted_ = 0, done_ = 0;
  bool ok_ = true, stop_ = false;
  std::thread th_;  // last: starts once the members above exist
};

ihs_status solve_overlap(const ihs_matrix* A, const Layout& L, const ihs_options* opt,
                         SolveBuffers& S, const double* b, double* x, double* x_hist,
                         double* factors, ihs_report* rep, hipStream_t stream) {
  // l2 ball: the factorisations run two steps ahead, alternating between two
  // side streams, so that two of these latency-bound chains run at once
  const bool l2pre = S.pre_status != nullptr;
  hipStream_t side = side_stream(0);
  hipStream_t side2 = l2pre ? side_stream(2) : side;
  hipStream_t sorter = side_stream(1);
  if (!side || !side2 || !sorter) return IHS_ERR_HIP;
  auto side_of = [&](int64_t k) { return (k % 2) ? side2 : side; };
  PassBuffers& B = S.pass;
  const int32_t N = opt->max_iter;
  const int64_t d = A->d, m = opt->sketch.m;
  const int64_t bd = (int64_t)L.batch * d;
  EventRing evSort(4), evPass(4), evChol(4), evMisc(3), evHash(4);
  if (!evSort.ok || !evPass.ok || !evChol.ok || !evMisc.ok || !evHash.ok) return IHS_ERR_HIP;
  auto ck = [](hipError_t e) { return !hip_failed(e); };
  // the extra streams start after everything already queued on the caller's
  // stream, the cleared side status records included
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, stream, S.side_status);
  if (l2pre) hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, stream, S.pre_status);
  if (S.inv_status)
    hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, stream, S.inv_status);
  if (!ck(hipEventRecord(evMisc.at(0), stream)) || !ck(hipStreamWaitEvent(side, evMisc.at(0), 0)) ||
      !ck(hipStreamWaitEvent(side2, evMisc.at(0), 0)) ||
      !ck(hipStreamWaitEvent(sorter, evMisc.at(0), 0)))
    return IHS_ERR_HIP;

  auto plan_for = [&](int64_t k) {  // sketch S_k, sorted into buffer set k % 2
    SketchPlan P = make_plan(L, &opt->sketch, B, opt->sketch.iter + (uint64_t)k);
    if (k % 2) {
      P.perm = S.perm1;
      P.bucket_start = S.bstart1;
      if (P.border != nullptr) P.border = S.border1;
    }
    return P;
  };
  // LA: how many steps ahead the passes form sketches; slots k % (LA + 1).
  // l1 steps look one step ahead (their side work is the Gram and a factor),
  // l2 steps two (each factorisation has two steps' time on its stream).
  const bool constrained = opt->constraint != IHS_UNCONSTRAINED;
  const int LA = ((opt->schedule == 2 && !constrained) || l2pre) ? 2 : 1;
  const int NS = LA + 1;
  auto sa_buf = [&](int64_t k) {
    const int64_t q = k % NS;
    return q == 0 ? S.SA : (q == 1 ? S.SA1 : S.SA2);
  };
  auto l_buf = [&](int64_t k) {
    const int64_t q = k % NS;
    return factors ? factors + k * L.batch * d * d : (q == 0 ? S.Lf : (q == 1 ? S.Lf1 : S.Lf2));
  };
  auto w_buf = [&](int64_t k) {
    const int64_t q = k % NS;
    return q == 0 ? S.work : (q == 1 ? S.work1 : S.work2);
  };
  const bool use_inv = d >= kInverseMinD;
  auto hinv_buf = [&](int64_t k) {
    const int64_t q = k % NS;
    return q == 0 ? S.Hinv0 : (q == 1 ? S.Hinv1 : S.Hinv2);
  };
  auto h_buf = [&](int64_t k) {
    if (!constrained) return S.H;
    if (l2pre) return k % 3 == 0 ? S.H : (k % 3 == 1 ? S.H1 : S.H2);
    return k % 2 ? S.H1 : S.H;
  };
  auto factor = [&](int64_t k) -> bool {  // side stream: H_k, its factor (and inverse)
    const hipStream_t sk = side_of(k);
    // the l2 step's Gram runs beside the step's latency-bound series products:
    // three workgroups per CU leave each SIMD registers for them
    if (!ck(launch_gram(sa_buf(k), opt->gram_in, m, d, d, L.batch, opt->gram_acc, h_buf(k),
                        (k % 2 && l2pre) ? S.gram_part1 : S.gram_part, sk, l2pre ? 3 : 4)))
      return false;
    // The constrained QPs work from H_k itself; the l1 ball's also needs the
    // unconstrained minimiser, so H_k is factored (and, from kInverseMinD
    // on, inverted) here, beside the pass. From kInverseMinD on the l1
    // penalty's polish uses H_k^{-1} too.
    if (constrained) {
      if (opt->constraint == IHS_L2_BALL) {
        // step k's QP (k >= 1, warm) iterates on (H_k + mu I)^{-1}, mu from
        // the snapshot taken before pass k - LA
        if (k < 1 || !l2pre) return true;
        const int q = (int)(k % 2);
        return ck(launch_l2_prefactor(h_buf(k), d, L.batch, S.snap[k % 3], S.Lpre[q],
                                      hinv_buf(k), q ? S.Linv1 : S.Linv, S.pre_scratch[q],
                                      S.pre_rows[q], S.pre_status, (int32_t)k, sk));
      }
      if (opt->constraint == IHS_L1_PENALTY && S.inv_status)
        return ck(launch_cholesky(h_buf(k), l_buf(k), d, L.batch, S.inv_status, (int32_t)k, 0.0,
                                  w_buf(k), sk)) &&
               ck(launch_chol_inverse(l_buf(k), chol_rdiag(w_buf(k), L.batch), d, L.batch,
                                      hinv_buf(k), S.Linv, S.inv_status, sk));
      if (opt->constraint != IHS_L1_BALL) return true;
      if (!ck(launch_cholesky(h_buf(k), l_buf(k), d, L.batch, S.side_status, (int32_t)k, 0.0,
                              w_buf(k), sk)))
        return false;
      return !use_inv ||
             ck(launch_chol_inverse(l_buf(k), chol_rdiag(w_buf(k), L.batch), d, L.batch,
                                    hinv_buf(k), S.Linv, S.side_status, sk));
    }
    if (!ck(launch_cholesky(S.H, l_buf(k), d, L.batch, S.side_status, (int32_t)k, 0.0,
                            w_buf(k), sk)))
      return false;
    if (!use_inv) return true;
    return ck(launch_chol_inverse(l_buf(k), chol_rdiag(w_buf(k), L.batch), d, L.batch,
                                  hinv_buf(k), S.Linv, S.side_status, sk));
  };

  // prologue: sketch-only passes for S_0 A .. S_{LA-1} A with the factors of
  // H_0 .. H_{LA-1}, and the sorts of S_0 .. S_LA. The sorted rows live in two
  // buffer sets (k % 2), so S_k is sorted only after the pass that read
  // S_{k-2}'s rows has run.
  for (int k = 0; k < 2; ++k)
    if (!ck(launch_sort(plan_for(k), sorter)) || !ck(hipEventRecord(evSort.at(k), sorter)))
      return IHS_ERR_HIP;
  ihs_status s = IHS_OK;
  for (int k = 0; k < LA; ++k) {
    if (l2pre && !ck(launch_l2_snapshot(S.work, d, L.batch, S.snap[k % 3], 1, stream)))
      return IHS_ERR_HIP;
    if (!ck(hipStreamWaitEvent(stream, evSort.at(k), 0))) return IHS_ERR_HIP;
    s = run_gather(A, &opt->sketch, B, plan_for(k), sa_buf(k), opt->gram_in, d, nullptr,
                   nullptr, nullptr, stream);
    if (s != IHS_OK) return s;
    if (!ck(hipEventRecord(evPass.at(k - LA), stream)) ||
        !ck(hipStreamWaitEvent(side_of(k), evPass.at(k - LA), 0)))
      return IHS_ERR_HIP;
    if (k < N && (!factor(k) || !ck(hipEventRecord(evChol.at(k), side_of(k))))) return IHS_ERR_HIP;
    if (k + 2 <= LA) {
      if (!ck(hipStreamWaitEvent(sorter, evPass.at(k - LA), 0)) ||
          !ck(launch_sort(plan_for(k + 2), sorter)) ||
          !ck(hipEventRecord(evSort.at(k + 2), sorter)))
        return IHS_ERR_HIP;
    }
  }

  int dev = 0;
  if (!ck(hipGetDevice(&dev))) return IHS_ERR_HIP;
  // chol_job[k % 4]: the side job that records evChol(k) (0: recorded above)
  std::vector<int64_t> chol_job(4, 0);
  SideQueue sq(dev);  // after everything its jobs refer to, so it is joined first
  // side: H_{t+LA} and its factor, queued by the side thread once `after`
  // has been reached on the caller's stream
  auto post_side = [&](int32_t t, hipEvent_t after, hipEvent_t after2) {
    const int64_t job = sq.post([&, t, after, after2]() {
      const hipStream_t sk = side_of(t + LA);
      if (!ck(hipStreamWaitEvent(sk, after, 0))) return false;
      if (after2 != nullptr && !ck(hipStreamWaitEvent(sk, after2, 0))) return false;
      return t + LA >= N || (factor(t + LA) && ck(hipEventRecord(evChol.at(t + LA), sk)));
    });
    chol_job.at((size_t)((t + LA) % chol_job.size())) = job;
  };
  for (int32_t t = 0; t < N; ++t) {
    // main (l2 ball): the shift state after QP_{t-1}, for the factorisation
    // of H_{t+LA} + mu I that a side stream starts once pass t is done
    if (l2pre && t + LA < N &&
        !ck(launch_l2_snapshot(S.work, d, L.batch, S.snap[(t + LA) % 3], t == 0 ? 1 : 0, stream)))
      return IHS_ERR_HIP;
    // main: pass P_t forms g(x^t) and S_{t+LA} A
    if (!ck(hipStreamWaitEvent(stream, evSort.at(t + LA), 0))) return IHS_ERR_HIP;
    s = run_gather(A, &opt->sketch, B, plan_for(t + LA), sa_buf(t + LA), opt->gram_in, d, b, x,
                   nullptr, stream);
    if (s != IHS_OK) return s;
    if (!ck(hipEventRecord(evPass.at(t), stream))) return IHS_ERR_HIP;
    if (!ck(launch_reduce_partials(B.gpart, B.fpart, L.batch, pass_parts(A, &opt->sketch, L.batch),
                                   B.probs, d, B.g, B.f, B.status, t, B.red, stream)))
      return IHS_ERR_HIP;
    // sorter: rows for S_{t+LA+1}, once P_t is done (its scattered writes
    // would slow the pass if they ran beside it); it shares the gap between
    // passes with the tail of the side stream and the update of x. The sort
    // is what the next pass waits for; its hash is arithmetic-bound, so an
    // unconstrained step's Gram (whose factorisation has time to spare) starts
    // only once the hash is done.
    // An SJLT's sort (s times the entries) and a CSR pass's sort (beside a
    // pass bound by scattered reads, not by bandwidth) start beside pass t
    // instead: the sort rewrites the row set that pass t - 1 read, so that
    // pass is all it must wait for (2% off an s = 4 lasso step, 1% off the
    // CSR l2 step; the pass slows by most of what the gap saves).
    const bool sort_beside = opt->sketch.s > 1 || A->format == IHS_CSR;
    const bool hash_first = !constrained && t + 2 <= N;
    if (t + 2 <= N) {
      if (!ck(hipStreamWaitEvent(sorter, evPass.at(sort_beside ? t - 1 : t), 0)) ||
          !ck(launch_sort(plan_for(t + LA + 1), sorter, hash_first ? evHash.at(t) : nullptr)) ||
          !ck(hipEventRecord(evSort.at(t + LA + 1), sorter)))
        return IHS_ERR_HIP;
    }
    // side: H_{t+LA} and its factor, from the end of pass t on
    post_side(t, evPass.at(t), hash_first ? evHash.at(t) : nullptr);
    // main: x^{t+1} = x^t + H_t^{-1} g(x^t), or the constrained QP of Eq.(2)
    // with H_t (its l2 shift state carries over in S.work from step to step)
    if (!sq.wait(chol_job.at((size_t)(t % chol_job.size()))) ||
        !ck(hipStreamWaitEvent(stream, evChol.at(t), 0)))
      return IHS_ERR_HIP;
    if (S.xprev && !ck(hipMemcpyAsync(S.xprev, x, bd * sizeof(double), hipMemcpyDeviceToDevice,
                                      stream)))
      return IHS_ERR_HIP;
    if (constrained) {
      QpArgs a{};
      a.d = d;
      a.batch = L.batch;
      a.constraint = opt->constraint;
      a.radius = opt->radius;
      a.max_inner = opt->qp_max_inner;
      a.tol = opt->qp_tol;
      a.H = h_buf(t);
      a.g = B.g;
      a.x = x;
      a.x_out = x;
      a.L = S.Lf;
      a.work = S.work;
      a.status = B.status;
      a.iter = t;
      a.warm = t > 0 ? 1 : 0;
      if (l2pre && t >= 1) {
        a.hinv_pre = hinv_buf(t);   // (H_t + mu I)^{-1} from a side stream
        a.trs_pre = S.snap[t % 3];
        a.pre_status = S.pre_status;
      }
      if (opt->constraint == IHS_L1_BALL) {  // H_t's factor or inverse, from the side stream
        hipLaunchKernelGGL(k_adopt_status, dim3(1), dim3(64), 0, stream, S.side_status, t,
                           B.status);
        if (use_inv) {
          a.hinv_pre = hinv_buf(t);
        } else {
          a.L = l_buf(t);
          a.rdiag_pre = chol_rdiag(w_buf(t), L.batch);
        }
      }
      if (opt->constraint == IHS_L1_PENALTY && S.inv_status) {  // for the polish
        a.hinv_pre = hinv_buf(t);
        a.pre_status = S.inv_status;
      }
      const hipError_t e = launch_qp_step(a, stream);
      if (e == hipErrorNotSupported) return IHS_ERR_UNSUPPORTED;
      if (hip_failed(e)) return IHS_ERR_HIP;
    } else if (use_inv) {
      if (!ck(launch_inv_apply(hinv_buf(t), d, L.batch, B.g, x, x, S.dx, B.status, stream,
                               S.side_status, t)))
        return IHS_ERR_HIP;
    } else if (!ck(launch_chol_solve_update(l_buf(t), chol_rdiag(w_buf(t), L.batch), d, L.batch,
                                            B.g, x, x, B.status, stream, S.side_status, t))) {
      return IHS_ERR_HIP;
    }
    if (S.xprev && !ck(launch_step_test(constrained ? h_buf(t) : nullptr, B.g, S.xprev, x, d,
                                        L.batch, opt->tol, S.stepq, B.status, t, stream)))
      return IHS_ERR_HIP;
    if (x_hist && !ck(hipMemcpyAsync(x_hist + (int64_t)t * bd, x, bd * sizeof(double),
                                     hipMemcpyDeviceToDevice, stream)))
      return IHS_ERR_HIP;
  }
  if (!sq.drain() || !ck(hipEventRecord(evMisc.at(1), side)) ||
      !ck(hipStreamWaitEvent(stream, evMisc.at(1), 0)) ||
      !ck(hipEventRecord(evMisc.at(0), side2)) || !ck(hipStreamWaitEvent(stream, evMisc.at(0), 0)) ||
      !ck(hipEventRecord(evMisc.at(2), sorter)) || !ck(hipStreamWaitEvent(stream, evMisc.at(2), 0)))
    return IHS_ERR_HIP;
  DeviceStatus hm, hs;
  if (read_status(B.status, &hm, stream) != IHS_OK) return IHS_ERR_HIP;
  if (read_status(S.side_status, &hs, stream) != IHS_OK) return IHS_ERR_HIP;
  // the earlier of the two failures (the side stream only fails with NOT_PD);
  // after a tolerance stop the side stream's later factorisations belong to
  // sketches no step used
  DeviceStatus f = hm;
  const bool side_counts = hs.code && (!hm.done || hs.failed_iter < hm.iters);
  if (side_counts && (!hm.code || hs.failed_iter < hm.failed_iter || hm.failed_iter < 0)) {
    f.code = hs.code;
    f.failed_iter = hs.failed_iter;
    f.failed_problem = hs.failed_problem;
  }
  return finish_report(f, hm, opt, rep);
}

// The reduced-access variant: one sketch S_0 (key (seed, iter)) held fixed,
// its Hessian sketch H_0 = (S_0 A)^T S_0 A as the preconditioner of conjugate
// gradients on the normal equations A^T A x = A^T b. The first pass forms
// S_0 A and A^T (b - A x^0) in one read of A; each of the max_iter
// iterations is one natural-order pass forming q = A^T A p (the gradient
// pass with b = 0 at x = -p), then the d-sized recurrences and z = H_0^{-1} r
// (explicit inverse for d >= kInverseMinD, triangular solves below).
ihs_status solve_fixed_sketch_cg(const ihs_matrix* A, const Layout& L, const ihs_options* opt,
                                 SolveBuffers& S, const double* b, double* x, double* x_hist,
                                 ihs_report* rep, hipStream_t stream) {
  PassBuffers& B = S.pass;
  const int64_t d = A->d, m = opt->sketch.m;
  const int64_t bd = (int64_t)L.batch * d;
  const bool use_inv = d >= kInverseMinD;
  auto ck = [](hipError_t e) { return !hip_failed(e); };
  if (!ck(fill(B.bzero, A->n, 0.0, stream)) || !ck(fill(S.cg_zero, bd, 0.0, stream)))
    return IHS_ERR_HIP;
  ihs_status s;
  if (dense_kind(&opt->sketch)) {  // a dense sketch, then the gradient pass
    if ((s = run_dense_sketch(A, &opt->sketch, opt->sketch.iter, S.SA, opt->gram_in, d, S.dsk,
                              stream)) != IHS_OK ||
        (s = run_gradient(A, L, B, b, x, S.cg_r, B.f, nullptr, B.status, 0, stream)) != IHS_OK)
      return s;
  } else {
    s = run_pass(A, L, &opt->sketch, B, opt->sketch.iter, S.SA, opt->gram_in, d, b, x, nullptr,
                 stream);
    if (s != IHS_OK) return s;
    if (!ck(launch_reduce_partials(B.gpart, B.fpart, L.batch,
                                   pass_parts(A, &opt->sketch, L.batch), B.probs, d, S.cg_r, B.f,
                                   B.status, 0, B.red, stream)))
      return IHS_ERR_HIP;
  }
  if (!ck(launch_gram(S.SA, opt->gram_in, m, d, d, L.batch, opt->gram_acc, S.H, S.gram_part,
                      stream)) ||
      !ck(launch_cholesky(S.H, S.Lf, d, L.batch, B.status, 0, 0.0, S.work, stream)))
    return IHS_ERR_HIP;
  double* rdiag = chol_rdiag(S.work, L.batch);
  if (use_inv && !ck(launch_chol_inverse(S.Lf, rdiag, d, L.batch, S.Hinv0, S.Linv, B.status,
                                         stream)))
    return IHS_ERR_HIP;
  auto precondition = [&]() {  // z = H_0^{-1} r
    if (use_inv)
      return ck(launch_inv_apply(S.Hinv0, d, L.batch, S.cg_r, S.cg_zero, S.cg_z, S.dx, B.status,
                                 stream, nullptr, -1));
    return ck(launch_chol_solve_update(S.Lf, rdiag, d, L.batch, S.cg_r, S.cg_zero, S.cg_z,
                                       B.status, stream));
  };
  if (!precondition() ||
      !ck(launch_pcg_begin(S.cg_r, S.cg_z, S.cg_pm, S.cg_rho, d, L.batch, B.status, stream)))
    return IHS_ERR_HIP;
  for (int32_t t = 0; t < opt->max_iter; ++t) {
    // q = A^T (0 - A (-p)) into B.g; the objective of the pass at x^0 stays recorded
    if ((s = run_gradient(A, L, B, nullptr, S.cg_pm, B.g, nullptr, nullptr, nullptr, t,
                          stream)) != IHS_OK)
      return s;
    if (!ck(launch_pcg_x(S.cg_pm, B.g, S.cg_rho, x, S.cg_r, d, L.batch, B.status, t, stream)) ||
        !precondition() ||
        !ck(launch_pcg_p(S.cg_r, S.cg_z, S.cg_pm, S.cg_rho, d, L.batch, B.status, stream)))
      return IHS_ERR_HIP;
    if (x_hist && !ck(hipMemcpyAsync(x_hist + (int64_t)t * bd, x, bd * sizeof(double),
                                     hipMemcpyDeviceToDevice, stream)))
      return IHS_ERR_HIP;
  }
  DeviceStatus host;
  if (read_status(B.status, &host, stream) != IHS_OK) return IHS_ERR_HIP;
  if (rep) {
    rep->status = host.code;
    rep->failed_iter = host.code ? host.failed_iter : -1;
    rep->failed_problem = host.code ? host.failed_problem : -1;
    rep->iters = host.code ? std::max(0, host.failed_iter) : opt->max_iter;
    rep->objective = host.objective;
    rep->last_step = host.last_step;
    rep->qp_unpolished = host.unpolished;
  }
  return (ihs_status)host.code;
}

}  // namespace

extern "C" {

const char* ihs_status_string(int32_t status) {
  switch (status) {
    case IHS_OK: return "ok";
    case IHS_ERR_INVALID_ARG: return "invalid argument";
    case IHS_ERR_UNSUPPORTED: return "unsupported configuration";
    case IHS_ERR_WORKSPACE: return "workspace too small";
    case IHS_ERR_HIP: return "HIP runtime error";
    case IHS_ERR_NOT_PD: return "Hessian sketch not positive definite";
    case IHS_ERR_NOT_CONVERGED: return "inner QP iteration did not converge";
    case IHS_ERR_NONFINITE: return "non-finite objective or iterate";
    default: return "unknown status";
  }
}

const char* ihs_last_hip_error(int32_t* code) {
  if (code) *code = t_last_hip_error;
  return t_last_hip_error ? hipGetErrorName((hipError_t)t_last_hip_error) : "hipSuccess";
}

ihs_status ihs_sketch_hash(const ihs_sketch* sk, int64_t n, int32_t problem, int32_t* bucket,
                           int8_t* sign, hipStream_t stream) {
  if (!valid_sketch(sk) || n < 0 || problem < 0) return IHS_ERR_INVALID_ARG;
  if (dense_kind(sk)) return IHS_ERR_UNSUPPORTED;  // no hash: S is dense
  if (n > 0 && (!bucket || !sign)) return IHS_ERR_INVALID_ARG;
  if (n * (int64_t)sk->s >= (int64_t(1) << 31)) return IHS_ERR_UNSUPPORTED;
  SketchPlan P{};
  P.s = sk->s;
  P.m = sk->m;
  P.m_blk = sk->m / sk->s;
  P.seed = sk->seed;
  P.iter = sk->iter;
  clear_stale_error();
  return hip_status(launch_sketch_hash(P, n, problem, bucket, sign, stream));
}

size_t ihs_workspace_size(const ihs_matrix* A, const ihs_options* opt) {
  if (check_matrix(A) != IHS_OK || !opt || check_sketch(&opt->sketch) != IHS_OK) return 0;
  if (!valid_gram_types(opt->gram_in, opt->gram_acc)) return 0;
  const Layout L = make_layout(A, opt->sketch.m);
  Carver c(nullptr);
  SolveBuffers S;
  return carve_solve(c, L, opt, S) + 256;
}

ihs_status ihs_sketch_apply(const ihs_sketch* sk, const ihs_matrix* A, void* SA,
                            int32_t sa_dtype, int64_t ld_sa, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  ihs_status s = check_matrix(A);
  if (s != IHS_OK) return s;
  if ((s = check_sketch(sk)) != IHS_OK) return s;
  if (!SA || ld_sa < A->d) return IHS_ERR_INVALID_ARG;
  if (sa_dtype != IHS_F64 && sa_dtype != IHS_F32 && sa_dtype != IHS_BF16) return IHS_ERR_INVALID_ARG;
  if (A->n * (int64_t)sk->s >= (int64_t(1) << 31)) return IHS_ERR_UNSUPPORTED;
  if (!ws) return IHS_ERR_INVALID_ARG;
  if (dense_kind(sk)) {
    if (A->batch != 1) return IHS_ERR_UNSUPPORTED;
    if (ws_bytes < dense_sketch_workspace_bytes(sk->kind, sk->m, A->n, A->d,
                                                A->format == IHS_CSR))
      return IHS_ERR_WORKSPACE;
    clear_stale_error();
    return run_dense_sketch(A, sk, sk->iter, SA, sa_dtype, ld_sa, static_cast<double*>(ws),
                            stream);
  }
  const Layout L = make_layout(A, sk->m);
  Carver need(nullptr);
  PassBuffers tmp;
  carve_pass(need, L, sk, tmp);
  if (ws_bytes < need.used) return IHS_ERR_WORKSPACE;
  clear_stale_error();
  Carver c(ws);
  PassBuffers B;
  carve_pass(c, L, sk, B);
  if ((s = upload_probs(L, B, stream)) != IHS_OK) return s;
  return run_pass(A, L, sk, B, sk->iter, SA, sa_dtype, ld_sa, nullptr, nullptr, nullptr, stream);
}

ihs_status ihs_sketch_apply_static(const ihs_sketch* sk, const ihs_matrix* A, void* SA,
                                   int32_t sa_dtype, int64_t ld_sa, hipStream_t stream) {
  ihs_status s = check_matrix(A);
  if (s != IHS_OK) return s;
  if ((s = check_sketch(sk)) != IHS_OK) return s;
  if (!SA || ld_sa < A->d) return IHS_ERR_INVALID_ARG;
  if (sa_dtype != IHS_F64 && sa_dtype != IHS_F32 && sa_dtype != IHS_BF16) return IHS_ERR_INVALID_ARG;
  if (A->n * (int64_t)sk->s >= (int64_t(1) << 31)) return IHS_ERR_UNSUPPORTED;
  if (dense_kind(sk)) return IHS_ERR_UNSUPPORTED;
  const Layout L = make_layout(A, sk->m);
  Carver need(nullptr);
  PassBuffers tmp;
  carve_sketch_only(need, L, sk, tmp);
  if (need.used > (size_t)IHS_STATIC_SCRATCH_BYTES) return IHS_ERR_WORKSPACE;
  clear_stale_error();
  void* base = static_scratch_address();
  if (!base) return IHS_ERR_HIP;
  Carver c(base);
  PassBuffers B;
  carve_sketch_only(c, L, sk, B);
  B.profile = false;
  if ((s = upload_probs(L, B, stream)) != IHS_OK) return s;
  return run_pass(A, L, sk, B, sk->iter, SA, sa_dtype, ld_sa, nullptr, nullptr, nullptr, stream);
}

ihs_status ihs_sketch_adjoint(const ihs_sketch* sk, int64_t n, int64_t d, int32_t batch,
                              const int64_t* row_offsets, const double* G, int64_t ld_g,
                              double* out, int64_t ld_out, hipStream_t stream) {
  ihs_status s = check_sketch(sk);
  if (s != IHS_OK) return s;
  if (n < 0 || d < 1 || batch < 1 || ld_g < d || ld_out < d) return IHS_ERR_INVALID_ARG;
  if (n > 0 && (!G || !out)) return IHS_ERR_INVALID_ARG;
  if (batch > 1) {
    if (!row_offsets || row_offsets[0] != 0 || row_offsets[batch] != n) return IHS_ERR_INVALID_ARG;
    for (int32_t p = 0; p < batch; ++p)
      if (row_offsets[p + 1] < row_offsets[p]) return IHS_ERR_INVALID_ARG;
  }
  if (n >= (int64_t(1) << 31)) return IHS_ERR_UNSUPPORTED;
  if (sk->s > 16 || dense_kind(sk)) return IHS_ERR_UNSUPPORTED;
  clear_stale_error();
  for (int32_t p0 = 0; p0 < batch; p0 += kAdjointBatch) {
    AdjointBatch ab{};
    ab.count = std::min<int32_t>(kAdjointBatch, batch - p0);
    ab.first = p0;
    for (int i = 0; i <= kAdjointBatch; ++i) {
      const int32_t p = p0 + std::min<int32_t>(i, ab.count);
      ab.off[i] = batch > 1 ? row_offsets[p] : (p == 0 ? 0 : n);
    }
    if (hip_failed(launch_sketch_adjoint(ab, sk->s, sk->m, sk->seed, sk->iter,
                              G + (int64_t)p0 * sk->m * ld_g, ld_g, d, out, ld_out,
                              stream)))
      return IHS_ERR_HIP;
  }
  return IHS_OK;
}

size_t ihs_gram_workspace_size(int64_t m, int64_t d, int32_t batch, int32_t in_dtype,
                               int32_t acc_dtype) {
  if (m < 1 || d < 1 || batch < 1 || !valid_gram_types(in_dtype, acc_dtype)) return 0;
  return gram_partials_bytes(m, d, batch, in_dtype, acc_dtype) + 256;
}

ihs_status ihs_gram(const void* SA, int32_t in_dtype, int64_t m, int64_t d, int64_t ld,
                    int32_t batch, int32_t acc_dtype, double* H, void* ws, size_t ws_bytes,
                    hipStream_t stream) {
  if (!SA || !H || !ws || m < 1 || d < 1 || batch < 1 || ld < d) return IHS_ERR_INVALID_ARG;
  if (!valid_gram_types(in_dtype, acc_dtype)) return IHS_ERR_INVALID_ARG;
  if (ws_bytes < gram_partials_bytes(m, d, batch, in_dtype, acc_dtype)) return IHS_ERR_WORKSPACE;
  clear_stale_error();
  return hip_status(launch_gram(SA, in_dtype, m, d, ld, batch, acc_dtype, H, ws, stream));
}

ihs_status ihs_gradient(const ihs_matrix* A, const double* b, const double* x, double* g,
                        double* r, double* f, void* ws, size_t ws_bytes, hipStream_t stream) {
  ihs_status s = check_matrix(A);
  if (s != IHS_OK) return s;
  if (!b || !x || !g || !ws) return IHS_ERR_INVALID_ARG;
  const Layout L = make_layout(A, 1);
  Carver need(nullptr);
  PassBuffers tmp;
  carve_pass(need, L, nullptr, tmp);
  if (ws_bytes < need.used) return IHS_ERR_WORKSPACE;
  clear_stale_error();
  Carver c(ws);
  PassBuffers B;
  carve_pass(c, L, nullptr, B);
  if ((s = upload_probs(L, B, stream)) != IHS_OK) return s;
  return run_gradient(A, L, B, b, x, g, f, r, nullptr, 0, stream);
}

size_t ihs_qp_workspace_size(int64_t d, int32_t batch, const ihs_options* opt) {
  if (d < 1 || batch < 1 || !opt) return 0;
  Carver c(nullptr);
  c.take<DeviceStatus>(1);
  c.take<double>((size_t)(batch * d * d));
  c.take<double>((size_t)batch * qp_work_doubles(d, opt->constraint));
  return c.used + 256;
}

ihs_status ihs_qp_step(int64_t d, int32_t batch, const double* H, const double* g,
                       const double* x, double* x_out, const ihs_options* opt, void* ws,
                       size_t ws_bytes, hipStream_t stream, ihs_report* rep) {
  if (d < 1 || batch < 1 || !H || !g || !x || !x_out || !opt || !ws) return IHS_ERR_INVALID_ARG;
  if (!valid_constraint(opt->constraint, opt->radius)) return IHS_ERR_INVALID_ARG;
  if (ws_bytes < ihs_qp_workspace_size(d, batch, opt) - 256) return IHS_ERR_WORKSPACE;
  clear_stale_error();
  Carver c(ws);
  DeviceStatus* st = c.take<DeviceStatus>(1);
  double* Lf = c.take<double>((size_t)(batch * d * d));
  double* work = c.take<double>((size_t)batch * qp_work_doubles(d, opt->constraint));
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, stream, st);
  QpArgs a{};
  a.d = d;
  a.batch = batch;
  a.constraint = opt->constraint;
  a.radius = opt->radius;
  a.max_inner = opt->qp_max_inner;
  a.tol = opt->qp_tol;
  a.H = H;
  a.g = g;
  a.x = x;
  a.x_out = x_out;
  a.L = Lf;
  a.work = work;
  a.status = st;
  a.iter = 0;
  const hipError_t e = launch_qp_step(a, stream);
  if (e == hipErrorNotSupported) return IHS_ERR_UNSUPPORTED;
  if (hip_failed(e)) return IHS_ERR_HIP;
  DeviceStatus host;
  if (read_status(st, &host, stream) != IHS_OK) return IHS_ERR_HIP;
  if (rep) {
    *rep = ihs_report{};
    rep->iters = 1;
    rep->status = host.code;
    rep->failed_iter = host.code ? 0 : -1;
    rep->failed_problem = host.code ? host.failed_problem : -1;
    rep->qp_unpolished = host.unpolished;
  }
  return (ihs_status)host.code;
}

ihs_status ihs_solve(const ihs_matrix* A, const double* b, const ihs_options* opt, double* x,
                     double* x_hist, double* factors, ihs_report* rep, void* ws,
                     size_t ws_bytes, hipStream_t stream) {
  ihs_status s = check_matrix(A);
  if (s != IHS_OK) return s;
  if ((s = check_options(opt, true)) != IHS_OK) return s;
  if (!b || !x || !ws) return IHS_ERR_INVALID_ARG;
  if (factors && (!opt->keep_factors || opt->constraint != IHS_UNCONSTRAINED))
    return IHS_ERR_INVALID_ARG;
  if (factors && opt->method != IHS_METHOD_IHS) return IHS_ERR_UNSUPPORTED;
  if (dense_kind(&opt->sketch) && A->batch != 1) return IHS_ERR_UNSUPPORTED;
  if (A->n * (int64_t)opt->sketch.s >= (int64_t(1) << 31)) return IHS_ERR_UNSUPPORTED;
  if (A->format == IHS_CSR && opt->gram_in != IHS_F64 && opt->gram_in != IHS_F32 &&
      opt->gram_in != IHS_BF16)
    return IHS_ERR_INVALID_ARG;
  const Layout L = make_layout(A, opt->sketch.m);
  Carver need(nullptr);
  SolveBuffers tmp;
  carve_solve(need, L, opt, tmp);
  if (ws_bytes < need.used) return IHS_ERR_WORKSPACE;
  clear_stale_error();
  Carver c(ws);
  SolveBuffers S;
  carve_solve(c, L, opt, S);
  PassBuffers& B = S.pass;
  if (opt->tol > 0.0) B.halt = &B.status->done;  // a device address; read by the passes
  if ((s = upload_probs(L, B, stream)) != IHS_OK) return s;
  if (opt->method == IHS_METHOD_FIXED_SKETCH_CG)
    return solve_fixed_sketch_cg(A, L, opt, S, b, x, x_hist, rep, stream);
  // the overlapped schedule reads sorted rows; the dense sketches run in order
  if (opt->schedule != 1 && opt->max_iter >= 2 && !dense_kind(&opt->sketch))
    return solve_overlap(A, L, opt, S, b, x, x_hist, factors, rep, stream);
  const int64_t d = A->d, m = opt->sketch.m;
  const int64_t bd = (int64_t)L.batch * d;
  for (int32_t t = 0; t < opt->max_iter; ++t) {
    const uint64_t iter = opt->sketch.iter + (uint64_t)t;
    if (dense_kind(&opt->sketch)) {  // a dense sketch, then the gradient pass
      if ((s = run_dense_sketch(A, &opt->sketch, iter, S.SA, opt->gram_in, d, S.dsk, stream)) !=
              IHS_OK ||
          (s = run_gradient(A, L, B, b, x, B.g, B.f, nullptr, B.status, t, stream)) != IHS_OK)
        return s;
    } else {
      s = run_pass(A, L, &opt->sketch, B, iter, S.SA, opt->gram_in, d, b, x, nullptr, stream);
      if (s != IHS_OK) return s;
      if (hip_failed(launch_reduce_partials(B.gpart, B.fpart, L.batch,
                                            pass_parts(A, &opt->sketch, L.batch), B.probs, d, B.g,
                                            B.f, B.status, t, B.red, stream)))
        return IHS_ERR_HIP;
    }
    if (hip_failed(launch_gram(S.SA, opt->gram_in, m, d, d, L.batch, opt->gram_acc, S.H, S.gram_part,
                    stream)))
      return IHS_ERR_HIP;
    QpArgs a{};
    a.d = d;
    a.batch = L.batch;
    a.constraint = opt->constraint;
    a.radius = opt->radius;
    a.max_inner = opt->qp_max_inner;
    a.tol = opt->qp_tol;
    a.H = S.H;
    a.g = B.g;
    a.x = x;
    a.x_out = x;
    a.L = factors ? factors + (int64_t)t * L.batch * d * d : S.Lf;
    a.work = S.work;
    a.status = B.status;
    a.iter = t;
    a.warm = t > 0 ? 1 : 0;
    if (S.xprev && hip_failed(hipMemcpyAsync(S.xprev, x, bd * sizeof(double),
                                             hipMemcpyDeviceToDevice, stream)))
      return IHS_ERR_HIP;
    const hipError_t e = launch_qp_step(a, stream);
    if (e == hipErrorNotSupported) return IHS_ERR_UNSUPPORTED;
    if (hip_failed(e)) return IHS_ERR_HIP;
    if (S.xprev &&
        hip_failed(launch_step_test(opt->constraint != IHS_UNCONSTRAINED ? S.H : nullptr, B.g,
                                    S.xprev, x, d, L.batch, opt->tol, S.stepq, B.status, t,
                                    stream)))
      return IHS_ERR_HIP;
    if (x_hist && hip_failed(hipMemcpyAsync(x_hist + (int64_t)t * bd, x, bd * sizeof(double),
                                 hipMemcpyDeviceToDevice, stream)))
      return IHS_ERR_HIP;
  }
  DeviceStatus host;
  if (read_status(B.status, &host, stream) != IHS_OK) return IHS_ERR_HIP;
  return finish_report(host, host, opt, rep);
}

ihs_status ihs_adjoint_solve(const ihs_matrix* A, const double* xbar, const double* factors,
                             int32_t n_factors, double* lambda, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  ihs_status s = check_matrix(A);
  if (s != IHS_OK) return s;
  if (!xbar || !factors || !lambda || !ws || n_factors < 1) return IHS_ERR_INVALID_ARG;
  if (A->format != IHS_DENSE) return IHS_ERR_UNSUPPORTED;
  const Layout L = make_layout(A, 1);
  Carver need(nullptr);
  PassBuffers tmp;
  carve_pass(need, L, nullptr, tmp);
  need.take<double>((size_t)(2 * L.batch * A->d));
  if (ws_bytes < need.used) return IHS_ERR_WORKSPACE;
  clear_stale_error();
  Carver c(ws);
  PassBuffers B;
  carve_pass(c, L, nullptr, B);
  double* v = c.take<double>((size_t)(L.batch * A->d));
  if ((s = upload_probs(L, B, stream)) != IHS_OK) return s;
  const int64_t bd = (int64_t)L.batch * A->d;
  if (hip_failed(fill(B.bzero, A->n, 0.0, stream))) return IHS_ERR_HIP;
  if (hip_failed(fill(lambda, bd, 0.0, stream))) return IHS_ERR_HIP;
  for (int32_t k = 0; k < n_factors; ++k) {
    // v = xbar - A^T A lambda = xbar + A^T (0 - A lambda)
    if ((s = run_gradient(A, L, B, B.bzero, lambda, B.g, nullptr, nullptr, B.status, k,
                          stream)) != IHS_OK)
      return s;
    hipLaunchKernelGGL(k_add, dim3((unsigned)((bd + 255) / 256)), dim3(256), 0, stream, xbar,
                       B.g, v, bd);
    const double* Lk = factors + (int64_t)k * L.batch * A->d * A->d;
    if (hip_failed(launch_recip_diag(Lk, A->d, L.batch, B.rdiag, stream))) return IHS_ERR_HIP;
    if (hip_failed(launch_chol_solve_update(Lk, B.rdiag, A->d, L.batch, v, lambda, lambda, B.status,
                                 stream)))
      return IHS_ERR_HIP;
  }
  return hip_status(hipGetLastError());
}

ihs_status ihs_solution_grads(const ihs_matrix* A, const double* b, const double* x,
                              const double* lambda, double* dl_db, double* dl_da,
                              int64_t ld_da, hipStream_t stream) {
  ihs_status s = check_matrix(A);
  if (s != IHS_OK) return s;
  if (A->format != IHS_DENSE) return IHS_ERR_UNSUPPORTED;
  if (!b || !x || !lambda) return IHS_ERR_INVALID_ARG;
  const bool f32 = A->dtype == IHS_F32;
  if (dl_da && ld_da < A->d) return IHS_ERR_INVALID_ARG;
  const Layout L = make_layout(A, 1);
  clear_stale_error();
  for (int32_t p0 = 0; p0 < L.batch; p0 += kAdjointBatch) {
    AdjointBatch ab{};
    ab.count = std::min<int32_t>(kAdjointBatch, L.batch - p0);
    ab.first = p0;
    for (int i = 0; i <= kAdjointBatch; ++i) {
      const int32_t p = p0 + std::min<int32_t>(i, ab.count);
      ab.off[i] = p < L.batch ? L.probs[p].row0 : A->n;
    }
    if (hip_failed(launch_solution_grads(ab, A->d, A->values, f32, A->ld, b, x, lambda, dl_db,
                                         dl_da, ld_da, stream)))
      return IHS_ERR_HIP;
  }
  return IHS_OK;
}

ihs_status ihs_profile_read_ceiling(const void* buf, int64_t bytes, int32_t reps,
                                    double* ms_per_read, hipStream_t stream) {
  if (!buf || bytes < 16 || reps < 1 || !ms_per_read ||
      reinterpret_cast<uintptr_t>(buf) % 16 != 0)
    return IHS_ERR_INVALID_ARG;
  clear_stale_error();
  // the sink is never written for finite data; the buffer's first element serves
  double* sink = const_cast<double*>(static_cast<const double*>(buf));
  hipEvent_t a = nullptr, b = nullptr;
  if (hip_failed(hipEventCreate(&a))) return IHS_ERR_HIP;
  if (hip_failed(hipEventCreate(&b))) {
    (void)hipEventDestroy(a);
    return IHS_ERR_HIP;
  }
  ihs_status s = IHS_OK;
  if (hip_failed(launch_read_probe(buf, bytes / 16 * 16, sink, stream)) ||  // warm
      hip_failed(hipEventRecord(a, stream))) {
    s = IHS_ERR_HIP;
  } else {
    for (int32_t r = 0; r < reps && s == IHS_OK; ++r)
      if (hip_failed(launch_read_probe(buf, bytes / 16 * 16, sink, stream))) s = IHS_ERR_HIP;
    float ms = 0.f;
    if (s == IHS_OK && (hip_failed(hipEventRecord(b, stream)) ||
                        hip_failed(hipEventSynchronize(b)) ||
                        hip_failed(hipEventElapsedTime(&ms, a, b))))
      s = IHS_ERR_HIP;
    *ms_per_read = s == IHS_OK ? (double)ms / reps : 0.0;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return s;
}

void ihs_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto& e : g_prof.ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  g_prof.ev.clear();
  g_prof.on = on != 0;
}

ihs_status ihs_profile_read(int64_t* launches, double* total_ms) {
  if (!launches || !total_ms) return IHS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  double tot = 0.0;
  for (auto& e : g_prof.ev) {
    if (hip_failed(hipEventSynchronize(e.second))) return IHS_ERR_HIP;
    float ms = 0.f;
    if (hip_failed(hipEventElapsedTime(&ms, e.first, e.second))) return IHS_ERR_HIP;
    tot += ms;
  }
  *launches = (int64_t)g_prof.ev.size();
  *total_ms = tot;
  return IHS_OK;
}

}  // extern "C"
