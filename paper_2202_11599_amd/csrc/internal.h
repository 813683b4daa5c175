// Internal declarations shared by the translation units of libnysadmm.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nysadmm.h"

#define NYS_TRY_HIP(expr)                                                         \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      nys::set_last_hip_error(e_, #expr, __FILE__, __LINE__);                     \
      return NYS_ERR_HIP;                                                         \
    }                                                                             \
  } while (0)

#define NYS_TRY(expr)                 \
  do {                                \
    nys_status s_ = (expr);           \
    if (s_ != NYS_OK) return s_;      \
  } while (0)

namespace nys {

// Pacing of the host's spin-waits on pinned slots.  Querying the stream is a
// runtime call that, while kernels are queued, can append a marker packet
// behind the last of them, and the next dispatch then waits for that marker;
// so the wait queries the stream (to end with an error when the stream failed
// or drained without writing the slot) only once the slot has stayed unwritten
// for kPollQueryMs, and then every kPollQueryMs.
constexpr int kPollQueryMs = 5;
struct PollPace {
  std::chrono::steady_clock::time_point next =
      std::chrono::steady_clock::now() + std::chrono::milliseconds(kPollQueryMs);
  // true when poll n (n >= 1) should query the stream
  bool due(long n) {
    if ((n & 255) != 0) return false;
    const auto now = std::chrono::steady_clock::now();
    if (now < next) return false;
    next = now + std::chrono::milliseconds(kPollQueryMs);
    return true;
  }
};

void set_last_hip_error(hipError_t e, const char* what, const char* file, int line);

// A caller-provided device workspace (nys_ctx_set_workspace): first-fit
// blocks of 256-byte granularity carved from [base, base + bytes), adjacent
// free blocks merged.  All work of the context that owns it runs on one
// stream, so a released block can be handed out again at once (later work on
// that stream is ordered after the work that used it).
struct Arena {
  char* base = nullptr;
  size_t bytes = 0;
  int device = -1;
  std::mutex mu;
  std::map<size_t, size_t> free_blocks;   // offset -> size
  size_t in_use = 0, peak = 0;
  Arena(void* p, size_t n, int dev);
  void* alloc(size_t want);              // nullptr when nothing fits
  void free(void* p, size_t n);
};

// Grow-only device buffer owned by a context or factor.
// Device buffer from the library's block cache (see pool_* in api.hip): a
// released block is reused once the work queued on every live context stream
// at release time has completed, so a step that rebuilds its factor does not
// pay hipMalloc/hipFree (and the device-wide synchronisation of hipFree).
// While a CtxScope of a context with a workspace is active on the thread, the
// block is carved from that workspace instead (and returned to it).
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  int device = -1;
  std::shared_ptr<Arena> arena;      // the workspace the block came from, if any
  nys_status reserve(size_t want);   // contents are not preserved when it grows
  void release();
  template <typename T>
  T* as() const { return static_cast<T*>(ptr); }
};

// Entry points bind their context for their duration: DevBuf::reserve then
// carves from the context's workspace when it has one.  Nested scopes of the
// same context are harmless; the previous binding is restored on exit.
struct CtxScope {
  explicit CtxScope(nys_ctx ctx);
  ~CtxScope();
  CtxScope(const CtxScope&) = delete;
  CtxScope& operator=(const CtxScope&) = delete;
 private:
  std::shared_ptr<Arena> prev_;
};

// Device-side PCG bookkeeping.  Written only by kernels; read by the host at
// convergence checks.
struct PcgDev {
  int done;      // 1 once converged / broken down
  int iters;     // iterations completed when done was set
  int flags;     // kFlag* bits
  int k;         // iteration index (batched path; the single path passes it as an argument)
  double thr2;   // squared stopping threshold
  double ww;     // last ||w||^2
  double rr;     // ||rhs||^2
  double true_rr;// last ||rhs - H_rho x||^2
  double pv;     // p^T H_rho p of the iteration (pre-reduced path)
  double wwn;    // ||w||^2 after the update (pre-reduced path)
};
static_assert(sizeof(PcgDev) <= 64, "PCG state must fit a 64-byte host slot");

#ifdef __HIPCC__
// The host learns that a PCG iteration has finished from a copy of the state
// in pinned host memory.  The matvec kernel of the next iteration makes that
// copy with its first thread, before it reads the state itself: a kernel that
// writes host memory waits at its end for the write to land, which costs a
// long kernel nothing but would stall the short kernels that end an
// iteration.  done = &PcgDev::done (the first member).
__device__ __forceinline__ void publish_state(const int* done, PcgDev* note, int seq) {
  if (note != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    PcgDev h = *reinterpret_cast<const PcgDev*>(done);
    h.k = seq;
    *note = h;
  }
}
#endif
// w^T y of PCG iteration k lives in wy[k % kWyRing]: iteration k reads entry
// k and writes entry k + 1, and the kernels of one solve run in stream order,
// so a ring of four suffices whatever max_iter is.
constexpr int kWyRing = 4;
constexpr int kFlagBreakdown = 1;
constexpr int kFlagNonfinite = 2;
constexpr int kFlagZeroRhs = 4;
constexpr int kFlagAltStart = 8;   // the candidate start won the judge

// Launch geometry of the fused Gram matvec for one matrix shape.
struct GramPlan {
  int waves = 4;     // waves per workgroup
  int cpl = 4;       // 16-byte chunks per lane
  int rows = 4;      // rows per pipelined group
  int per_cu = 2;    // resident workgroups per CU the grid was sized for
  int grid = 512;    // workgroups (each owns a contiguous row range)
  int64_t rows_per_wg = 0;
  bool aligned = true;
  int ldy = 0;       // leading dimension of the per-workgroup partial sums
  // column-blocked y = A p of an explicit symmetric A (kernel SVM): blockIdx.y
  // runs over `slices` blocks of slice_cols columns; the y partials are one
  // n-vector per block, the q partials one per workgroup
  bool symv = false;
  int slices = 1;
  int slice_cols = 0;
  // sparse A (CSR + CSC passes): y is one n-vector, q one partial per row workgroup
  const nys_sparse_s* sparse = nullptr;
  // wide dense A (wide.hip): row dots per column block (slices x grid
  // workgroups), then one epilogue kernel of mgrid workgroups (the q
  // partials), then the A^T pass over the same blocks (grid y partials of
  // ldy columns).  The per-block row dots (slices x ldt) and the n-vector s
  // follow the q partials in the partial-sum buffer (wide_tmp).
  bool wide = false;
  int mgrid = 0;
  int64_t ldt = 0;
  int ny() const { return sparse ? 1 : (symv ? slices : grid); }
  int nq() const { return symv ? slices * grid : (wide ? mgrid : grid); }
  // doubles the partial-sum buffer needs after the y and q partials
  size_t tmp_doubles() const { return wide ? (size_t)(slices + 1) * (size_t)ldt : 0; }
};

enum GramMode : int {
  kModeHess = 0,     // s = D t (D NULL: s = t), q += s t
  kModeLsGrad = 1,   // s = t - b, q += s^2
  kModeLogit = 2,    // w = sigma(t)(1-sigma(t)) -> Dout, s = w t + b - sigma(t), q += loss
  kModeLogGrad = 3,  // s = sigma(t) - b, q += loss
  kModeTOnly = 4,    // s = b (no product with p), q = 0
};


// Pointers into the context workspace used by one PCG solve.
struct PcgWs {
  double* ypart = nullptr;
  double* qpart = nullptr;
  double* w = nullptr;
  double* p = nullptr;
  double* cvec = nullptr;
  double* wy = nullptr;
  PcgDev* st = nullptr;
  double* wwpart = nullptr;
  double* rrpart = nullptr;
  double* pppart = nullptr;
  double* w2 = nullptr;          // residual of a candidate start (judge)
  double* wwpart2 = nullptr;
  double* rrpart2 = nullptr;
  int nred = 0;     // ||w||^2 partials: nblk(d, rj)
  int nvec = 0;
  int rj = 16;     // columns per workgroup of the partial reduction (red_block(ny))
};

// ---- api.hip
size_t align_up(size_t x);
// Launch shape for A: the fastest of gram_candidates() timed on A itself the
// first time this (dtype, n, d, ld, alignment) is seen, cached in the context.
// NYSADMM_GRAM_PLAN forces a shape, NYSADMM_TUNE=0 uses the heuristic.
nys_status ctx_gram_plan(nys_ctx ctx, const nys_dense& A, GramPlan* out);
// launch_gram on the context's stream, timed when profiling is on
// note (may be NULL): pinned host slot that the launch's first thread fills
// with the PCG state *done belongs to (done = &PcgDev::done), sequence number
// note_seq, before the kernel reads it (see publish_state)
nys_status ctx_gram(nys_ctx ctx, const nys_dense& A, const GramPlan& plan, int mode,
                    const double* p, const double* aux, double* auxout, double* ypart,
                    double* qpart, const int* done, PcgDev* note = nullptr, int note_seq = 0);
nys_status validate_dense(const nys_dense* A);
// Device check of a caller's n-vector (kind as launch_check_vec); synchronises.
// NYS_ERR_NONFINITE for NaN/Inf, NYS_ERR_INVALID for a broken rule.
nys_status check_vector(nys_ctx ctx, const double* v, int64_t n, int kind);
nys_status pcg_workspace(nys_ctx ctx, const GramPlan& pl, int64_t d, int max_iter, PcgWs* ws);
nys_status read_pcg_state(nys_ctx ctx, const PcgWs& ws, PcgDev* out);

// ---- workspace accounting (each next to the code whose buffers it counts)
size_t admm_ws_bytes(int64_t n, int64_t d);                                   // admm.hip
size_t batch_workspace_bytes(int count, int64_t n, int64_t d, int r);         // batched.hip
void sketch_ws_bytes(const nys_dense& A, int m, int r, int num_cu, size_t* tmp,
                     size_t* factor);                                          // sketch.hip
size_t sparse_handle_bytes(int64_t n, int64_t d, int64_t nnz);               // sparse.hip

// ---- admm.hip / batched.hip
// relative KKT residual (eq. 31 or its logistic form) and objective at z
nys_status admm_kkt(nys_ctx ctx, const nys_problem& P, const double* z, double* eta, double* obj);
nys_status admm_solve_batched(nys_ctx ctx, int count, const nys_problem* P,
                              const nys_admm_opts* O, nys_admm_state* S, nys_admm_info* I);

// ---- core.hip
// C(m,n) = alpha sum_k A(m,k) w_k B(k,n) + beta C(m,n) in FP64 (w NULL: 1),
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], C(m,n) = C[m*scm + n*scn].
nys_status gemm64(hipStream_t st, int M, int N, int K, const void* A, bool a_f32, int64_t sam,
                  int64_t sak, const void* B, bool b_f32, int64_t sbk, int64_t sbn, double* C,
                  int64_t scm, int64_t scn, double alpha, double beta, double* split_ws,
                  size_t split_ws_elems, const double* wk = nullptr);
nys_status chol_upper(hipStream_t st, double* M, int r, int ld, int* fail);
nys_status trinv_upper(hipStream_t st, const double* Cm, int r, int ld, double* Z, int ldz);
nys_status power_iter(hipStream_t st, const double* G, int r, int ld, int iters, double* out);
int jacobi_pad(int r);
size_t jacobi_ws_doubles(int r);
// V0 (may be NULL): r x r column-major orthonormal start basis (the
// eigenvectors come out as V0 times the accumulated rotations); identity if NULL
// ---- sketch.hip
// A fresh factor of rank r (as nys_sketch) whose eigensolver starts from the
// projection of prev's U when prev has the same rank and dimension.
nys_status sketch_rebuild(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                          const double* omega, int r, nys_dtype prec, nys_factor prev,
                          nys_factor* F);
nys_status jacobi_eig(hipStream_t st, const double* G, int r, int ld, double* ws, int* counters,
                      int max_sweeps, void* host_pinned, void* host_pinned_dev, int* poll_seq,
                      double* sig2, double* W, int ldw, int* sweeps_out,
                      const double* V0 = nullptr, double tol = 1e-15);
// Stop when ||w|| <= max(abs_tol, tol ||rhs||) (o.tol_abs: ||w|| <= o.tol).
// hx_tag >= 0: H_rho x saved by the previous run's true-residual pass gives w0
// without a pass over A when that run had the same (A, D, x pointer, c, rho)
// and was called with hx_tag - 1 (the ADMM iteration counter of one state, so
// a new or rewound state never matches); this run saves its own with hx_tag.
// x_alt: a candidate start; PCG starts from whichever of x and x_alt has the
// smaller residual (x is overwritten by x_alt if it wins, *used_alt = 1).
nys_status pcg_run(nys_ctx ctx, const nys_dense& A, const double* D, double c, double rho,
                   nys_factor F, const double* rhs, double* x, const nys_pcg_opts& o,
                   nys_pcg_info* info, double abs_tol = 0.0, int64_t hx_tag = -1,
                   const double* x_alt = nullptr, int* used_alt = nullptr, bool symv = false);

// ---- mlp.hip
nys_status ws_propose(nys_ctx ctx, nys_ws_model m, nys_factor F, const double* rhs, double gamma,
                      double rho, double* x0, double* scratch, double* feat_out);
nys_status ws_record(nys_ctx ctx, nys_factor F, const double* rhs, double gamma, double rho,
                     const double* x, double* feat_out, double* target_out, double* scratch);
nys_status ws_analytic(nys_ctx ctx, nys_factor F, const double* rhs, double rho, double* x0,
                       double* scratch);
}  // namespace nys

// Key of the cached A^T b of the lasso right-hand side.
struct AtbKey {
  const void* A = nullptr;
  const double* b = nullptr;
  int64_t n = -1, d = -1, ld = -1;
  const void* buf = nullptr;
  bool operator==(const AtbKey& o) const {
    return A == o.A && b == o.b && n == o.n && d == o.d && ld == o.ld && buf == o.buf;
  }
};

constexpr size_t kPinnedBytes = 65536;     // pinned readback area of a context
constexpr size_t kPollOffset = 61440;      // PCG polling slots (4 x 64 bytes) in it
constexpr size_t kJacSlotOffset = kPollOffset + 512;   // eigensolver sweep slots (4 x 8 bytes)

struct nys_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  nys::DevBuf ypart;     // per-workgroup partial sums of the Gram matvec
  nys::DevBuf vecs;      // PCG / ADMM d- and n-vector temporaries
  nys::DevBuf small;     // partial-sum arrays, scalars, PcgDev
  nys::DevBuf gemm_ws;   // sketch temporaries (T = A Omega, ...)
  nys::DevBuf core_ws;   // FP64 core temporaries
  nys::DevBuf admm_ws;   // ADMM vectors (A^T b, rhs, weights, ...)
  nys::DevBuf svm_ws;    // kernel SVM vectors (rhs, H z, scalars)
  nys::DevBuf check;     // flag word of the argument checks
  std::shared_ptr<nys::Arena> arena;   // caller's workspace (nys_ctx_set_workspace), or none
  void* host_pinned = nullptr;  // pinned readback area of kPinnedBytes
  void* host_pinned_dev = nullptr;  // the same memory as seen from the device
  int poll_seq = 0;              // last sequence number of a PCG state slot write
  AtbKey atb_key;                // which (A, b) the cached A^T b in admm_ws belongs to
  int64_t atb_next_k = -1;       // ... valid for the ADMM step with this counter
  nys::DevBuf hx;                // H_rho x of the last solve (lasso ADMM sequence)
  AtbKey hx_key;                 // (A, x) it belongs to; buf = x pointer
  double hx_rho = -1.0, hx_c = -1.0;
  int64_t hx_tag = -1;           // tag of the pcg_run that may use it
  std::map<std::string, nys::GramPlan> plans;   // autotuned launch shapes per matrix shape
  std::map<std::string, std::vector<int>> bplans;  // autotuned batched shapes per batch
  hipStream_t cap_stream = nullptr;              // graph-capture stream (batched path)
  // batched path: streams on which the matvec pairs of the row-width buckets
  // after the first run concurrently (forked from and joined back to the
  // calling stream with these events)
  static constexpr int kSideStreams = 3;
  hipStream_t side_stream[kSideStreams] = {};
  hipEvent_t side_fork = nullptr;
  hipEvent_t side_join[kSideStreams] = {};
  bool prof_on = false;          // time matvec-pair launches with events
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
  long prof_skipped = 0;         // timed launches that returned at once (PCG already done)
  bool pcg_time_on = false;        // time each ADMM subproblem's PCG solve with events
  std::vector<hipEvent_t> pcg_ev;  // their event pairs
  size_t pcg_used = 0;
};

struct nys_sparse_s {
  int64_t n = 0, d = 0, nnz = 0;
  int device = 0;
  const int* rowptr = nullptr;   // caller's CSR arrays
  const int* colidx = nullptr;
  const float* val = nullptr;
  // CSC copy: colptr (d + 1 ints), then (at a 16-byte boundary) the row
  // indices and values, cap slots each; nnzc = colptr[d] entries are used
  // (nnz plus one zero entry per empty column), the rest is zero
  nys::DevBuf csc;
  int64_t cap = 0, nnzc = 0;
  int64_t row_off() const { return (d + 1 + 3) / 4 * 4; }
  int* colptr() const { return csc.as<int>(); }
  int* rows() const { return csc.as<int>() + row_off(); }
  float* cvals() const { return reinterpret_cast<float*>(csc.as<int>() + row_off() + cap); }
  nys::DevBuf s;                 // the n-vector s = f(A p) between the two passes
  // column-pass work split: cgrid workgroups of 16 wavefronts; part holds
  // wstart (16 cgrid + 1 ints: first entry of each wavefront's range, the
  // last = nnzc) and wbase (16 cgrid + 1 ints: columns starting before that
  // entry, minus one)
  nys::DevBuf part;
  int cgrid = 0;
  const int* wstart() const { return part.as<int>(); }
  const int* wbase() const { return part.as<int>() + 16 * (int64_t)cgrid + 1; }
  int num_cu = 256;              // CUs of the device (row-pass grid)
};

struct nys_factor_s {
  int64_t d = 0;
  int r = 0;
  int cap = 0;               // column capacity of Omega/Y
  double nu = 0.0;
  int mantissa_bits = 52;
  nys_dtype prec = NYS_F64;
  int device = 0;
  nys::DevBuf U;             // FP64 d x r column-major
  nys::DevBuf U32;           // FP32 copy used by the PCG preconditioner when prec != F64
  nys::DevBuf lam;           // FP64 r, descending
  nys::DevBuf Omega;         // FP64 d x cap, orthonormalised blocks
  nys::DevBuf Y;             // FP64 d x cap, sketch H Omega
  nys::DevBuf T;             // FP32 n x cap column-major, A Omega (FP32/BF16 sketches)
  nys::DevBuf Mbase;         // FP64 cap x cap, Omega^T H Omega from T (FP32/BF16 sketches)
  std::vector<double> lam_host;
  bool use_u32 = false;
  bool sym = false;          // factor of an explicit symmetric H = K + c I (kernel SVM)
  bool sparse = false;       // factor of a CSR A: FP64 products at any prec (NYS_F32 keeps U32)
  // non-owning, set only while a rebuild runs: the previous factor's U (d x r
  // FP64), whose projection starts the eigensolver near its answer
  const double* basis_hint = nullptr;
};

namespace nys {

// ---- noalloc.hip
// Look up the device address of the library's static scratch array on the
// current device (once per device; called by nys_ctx_create).
nys_status noalloc_init(int device);

// ---- block cache (api.hip)
void pool_register_stream(int device, hipStream_t st);
void pool_unregister_stream(int device, hipStream_t st);

// ---- gemv.hip
GramPlan make_gram_plan(const nys_dense& A, int num_cu);
GramPlan make_gram_plan_capped(const nys_dense& A, int num_cu, int64_t max_grid);
// columns one workgroup of the fused matvec covers (the widest plan): d above
// this takes the two-pass wide form
int64_t gram_max_cols(nys_dtype dt);
std::vector<GramPlan> gram_candidates(const nys_dense& A, int num_cu);
// Launch the fused pass  t = A p;  s = mode(t);  y_g = sum_{rows of g} s_i A_i.
nys_status launch_gram(const nys_dense& A, const GramPlan& plan, int mode, const double* p,
                       const double* aux, double* auxout, double* ypart, double* qpart,
                       const int* done, hipStream_t st,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                       PcgDev* note = nullptr, int note_seq = 0);

GramPlan make_symv_plan(const nys_dense& A, int num_cu);
nys_status launch_symv(const nys_dense& A, const GramPlan& plan, const double* p, double* ypart,
                       double* qpart, const int* done, hipStream_t st, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr, PcgDev* note = nullptr, int note_seq = 0);

// ---- wide.hip
GramPlan make_wide_plan(const nys_dense& A, int num_cu);
// start of the wide form's temporaries: after the q partials of the plan
double* wide_tmp(const GramPlan& pl, double* qpart);
nys_status launch_wide(const nys_dense& A, const GramPlan& plan, int mode, const double* p,
                       const double* aux, double* auxout, double* ypart, double* qpart,
                       const int* done, hipStream_t st, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr, PcgDev* note = nullptr, int note_seq = 0);

// ---- sparse.hip
GramPlan make_sparse_plan(const nys_sparse_s* S);
nys_status launch_sparse_pair(const nys_sparse_s* S, const GramPlan& plan, int mode,
                              const double* p, const double* aux, double* auxout, double* ypart,
                              double* qpart, const int* done, hipStream_t st,
                              hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                              PcgDev* note = nullptr, int note_seq = 0);
// Y[:, 0:m] (column-major, ld d) = A^T (D (A Om)) + c Om for sparse A, FP64 sums;
// Om column-major d x m.  ws holds (n + 2 d) m doubles.
nys_status sparse_sketch(const nys_sparse_s* S, const double* D, double c, const double* Om, int m,
                         double* Y, double* ws, hipStream_t st);
inline const nys_sparse_s* as_sparse(const nys_dense& A) {
  return A.dtype == NYS_CSR ? static_cast<const nys_sparse_s*>(A.data) : nullptr;
}

// ---- vec.hip
constexpr int kVecBlock = 32;    // entries of y per workgroup of the preconditioner update
constexpr int kVecBlockWide = 256;   // the same for d > kPreReduceDim
constexpr int kRedBlock = 16;    // columns per workgroup of the partial reduction
// columns per workgroup of the partial reduction for G partial rows: 16
// columns x 16 slices of the partials for large G, one column per thread
// (all 256 lanes busy) when there are few partial rows to add
inline int red_block(int G) { return G <= 16 ? 256 : kRedBlock; }
constexpr int kDotSlicesMax = 64; // d-slices of the U^T w partial sums (buffer size)
// the U^T w partials (kDotSlicesMax slices of 1024) and, after them, the
// reduced g = s o c and sum s c^2 of the large-d path (1025 doubles)
constexpr size_t kCvecDoubles = (size_t)1024 * (kDotSlicesMax + 2);
// slices for dimension d: 8, or one per 4096 entries up to 64 for large d
inline int dot_slices(int64_t d) {
  // slices of 4096 entries; 8192 above 32768, where one workgroup sums the
  // slices once per iteration (measured at d = 150348, rank 50: 2048, 4096,
  // 8192 and 16384 entries per slice gave 468, 482, 489 and 462 solves/s)
  const int64_t s = d > 32768 ? (d + 8191) / 8192 : (d + 4095) / 4096;
  return (int)(s < 8 ? 8 : (s > kDotSlicesMax ? kDotSlicesMax : s));
}
// Above this dimension the PCG scalars (p^T v, ||w||^2) are summed once per
// iteration by a one-workgroup kernel instead of by every workgroup of the
// vector kernels (whose partial counts grow with d).
constexpr int64_t kPreReduceDim = 32768;
// entries of y per workgroup of the preconditioner update at dimension d
// (also the count of its p^T p partials: nblk(d, vec_block(d)))
inline int vec_block(int64_t d) { return d > kPreReduceDim ? kVecBlockWide : kVecBlock; }
inline int nblk(int64_t d, int b) { return (int)((d + b - 1) / b); }

// v = sum_g ypart[g] + rho_eff * p ; then per `op`:
//   op 0 (iterate): alpha = wy[k] / (sum q + rho_eff ||p||^2); x += alpha p; w -= alpha v
//   op 1 (init):    w = rhs - v ;  ||rhs||^2 partials
//   op 2 (true):    w = rhs - v  (true residual, FP64 accumulation); v -> x if x != NULL
//   op 3 (plain):   w = v
//   op 4 (carry):   x = rhs - w  (H_rho x from the recursive residual; ypart unused)
nys_status launch_reduce_update(int op, const double* ypart, int G, int ldy, const double* qpart,
                                int64_t d, double rho_eff, const double* p, double* x, double* w,
                                const double* rhs, double* wy, int k, const double* pppart,
                                int npp, double* wwpart, double* rrpart, PcgDev* st,
                                hipStream_t stream, int Gq = -1,   // Gq: q partials (-1: G)
                                bool pre = false,                  // alpha from st->pv
                                int rj = 0);  // columns per workgroup (0: red_block(G)); the
                                              // ||w||^2 partials number nblk(d, rj)
// *slot = *st with k = seq (one thread): publish_state for an iteration that
// no matvec launch follows
nys_status launch_zero_state(PcgDev* st, hipStream_t stream);
nys_status launch_note(const PcgDev* st, PcgDev* slot, int seq, hipStream_t stream);
// st->pv = sum(a) + rho_eff sum(b) (op 0) or st->wwn = sum(a) (op 1), one
// workgroup, fixed order; skipped once st->done is set
nys_status launch_pcg_scalar(int op, const double* a, int na, const double* b, int nb,
                             double rho_eff, PcgDev* st, hipStream_t stream);
// *out = a^T b (one workgroup, fixed order)
// Judge of two PCG starts: ||w||^2 from wwpart and from wwpart2 (same fixed
// summation order); if the second is smaller, x <- x_alt, w <- w2,
// wwpart <- wwpart2 and st->flags |= kFlagAltStart.  No host synchronisation.
nys_status launch_judge(double* wwpart, const double* wwpart2, int nred, double* x,
                        const double* x_alt, double* w, const double* w2, int64_t d, PcgDev* st,
                        hipStream_t stream);
// out = U^T v (FP64 U, d x r column-major), out2 (optional) = U c for c (r)
nys_status launch_ut_v(const double* U, int64_t d, int r, const double* v, double* out,
                       hipStream_t stream);
nys_status launch_u_c(const double* U, int64_t d, int r, const double* c, double* out,
                      hipStream_t stream);
nys_status launch_dot(const double* a, const double* b, int64_t d, double* out,
                      hipStream_t stream);
// flags |= kCheck* bits of the caller vector v (n entries): kind 0 weights
// (v >= 0), kind 1 labels (v in {0, 1}); NaN/Inf set kCheckNonfinite
constexpr int kCheckBad = 1;
constexpr int kCheckNonfinite = 2;
nys_status launch_check_vec(const double* v, int64_t n, int kind, int* flags, hipStream_t stream);
// mode 0: PCG iteration k test + dots, 1: PCG init (threshold from ||rhs||) test + dots,
// 2: dots only, 3: store sum(wwpart) into st->true_rr
nys_status launch_precond_dot(const void* U, bool u32, int64_t d, int r, const double* w,
                              double* cvec, PcgDev* st, const double* wwpart, int nww,
                              const double* rrpart, int k, int mode, double tol_rel,
                              double tol_abs, hipStream_t stream, bool pre = false);
// mode 0: PCG iteration k (p = y + beta p), 1: PCG init (p = y), 2: standalone y = P^-1 w
nys_status launch_precond_update(const void* U, bool u32, int64_t d, int r, const double* lam,
                                 double lam_s, double rho, const double* cvec, const double* w,
                                 double* p, double* wy, int k, const double* wwpart, int nww,
                                 double* pppart, const PcgDev* st, int mode, hipStream_t stream,
                                 PcgDev* host_slot = nullptr, int seq = 0, bool pre = false,
                                 const double* gpre = nullptr);
// large d: g_i = s_i c_i (c summed from its slices) and sum_i s_i c_i^2 into
// gout[0, r) and gout[1024], once per iteration, for launch_precond_update
nys_status launch_c_reduce(const double* cvec, int64_t d, int r, const double* lam, double lam_s,
                           double rho, double* gout, const PcgDev* st, hipStream_t stream);

}  // namespace nys
