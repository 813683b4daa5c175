/*
 * nysadmm.h - C ABI of the NysADMM x-subproblem hot path for AMD MI355X (gfx950).
 *
 * Method: Zhao, Frangella, Udell, "NysADMM: faster composite convex
 * optimization via low-rank approximation" (ICML 2022).  The library solves
 * the ADMM x-subproblem, eq. (ADMMSubProb),
 *
 *     (A^T diag(D) A + (c + rho) I) x = rhs,
 *
 * by Nystrom-preconditioned CG (Algorithm Nystrom PCG) with the randomized
 * Nystrom factor of Algorithm RandNysAppx / AdaptiveRandNysAppx, and runs the
 * surrounding ADMM loop (Algorithm NysADMM) for the composite problem eq. (1),
 * min l(Ax; b) + c/2 ||x||^2 + gamma ||x||_1, with l the least-squares loss
 * (lasso, eq. 2; elastic net, eq. 6) or the logistic loss (eq. 9).
 *
 * Conventions shared by every entry point
 *  - Pointers named A.data, D, b, omega, w, y, rhs, x, z, u and U are DEVICE
 *    pointers; pointers to option/info structs and *_host arrays are host
 *    pointers.  The caller owns every buffer it passes; the library owns only
 *    the opaque nys_ctx / nys_factor objects and the device workspace they
 *    hold (allocated with hipMalloc on first need, grown on demand, freed by
 *    nys_ctx_destroy / nys_factor_destroy).
 *  - A is dense row-major n x d with leading dimension ld >= d (elements), in
 *    FP32 or FP64.  Rows whose byte offset is a multiple of 16 take the vector
 *    load path; any ld is accepted.
 *  - Every vector (D, b, rhs, x, z, u, w, y) is FP64 and contiguous.  D is an
 *    n-vector of non-negative Hessian weights (H^l of the loss, Section 2.1);
 *    D == NULL means the identity (least squares).  Entry points that take a
 *    caller's D (nys_sketch, nys_sketch_adaptive, nys_hessian_apply,
 *    pcg_solve) check it on the device first and synchronise the stream:
 *    a negative weight gives NYS_ERR_INVALID, a NaN or infinite one
 *    NYS_ERR_NONFINITE.  A NaN or infinity in A, b or rhs surfaces as
 *    NYS_ERR_NONFINITE from the first residual or sketch norm it reaches.
 *  - The Gaussian test-matrix entries `omega` are passed in by the caller:
 *    FP64, column-major d x r (column k at omega + k*d).  They may come from
 *    any generator; nys_gaussian draws them on the device from a seed.  The
 *    library orthonormalises them (thin QR, as in Algorithm RandNysAppx).
 *  - All work is ordered on the HIP stream given to nys_ctx_create.  Calls
 *    that return scalars (info structs, factor info) synchronise that stream.
 *    A context is not thread-safe; use one per stream.
 *  - Errors are returned as nys_status; nothing aborts or throws across the
 *    ABI.  nys_status_string() gives a static message.  On NYS_ERR_MAXITER,
 *    NYS_ERR_BREAKDOWN and NYS_ERR_NOT_SPD the outputs hold the last iterate
 *    and the info struct is filled.
 */
#ifndef NYSADMM_H
#define NYSADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NYS_OK = 0,
  NYS_ERR_INVALID = 1,       /* bad argument (NULL, size, rho <= 0, r out of range, ...) */
  NYS_ERR_HIP = 2,           /* a HIP runtime call failed */
  NYS_ERR_NOT_SPD = 3,       /* Cholesky of Omega^T Y_nu failed after 3 shift retries */
  NYS_ERR_BREAKDOWN = 4,     /* PCG met p^T (H + rho I) p <= 0 */
  NYS_ERR_MAXITER = 5,       /* PCG stopped at max_iter above its tolerance */
  NYS_ERR_NONFINITE = 6,     /* NaN or Inf in a residual or eigenvalue */
  NYS_ERR_NOMEM = 7,         /* device allocation failed */
  NYS_ERR_NOT_CONVERGED = 8  /* the FP64 eigensolver of the factor core did not converge */
} nys_status;

typedef enum { NYS_F32 = 0, NYS_F64 = 1, NYS_BF16 = 2, NYS_CSR = 3 } nys_dtype;
typedef enum { NYS_LOSS_LS = 0, NYS_LOSS_LOGISTIC = 1 } nys_loss;

typedef struct nys_ctx_s* nys_ctx;
typedef struct nys_factor_s* nys_factor;
typedef struct nys_ws_model_s* nys_ws_model;
typedef struct nys_sparse_s* nys_sparse;

/* Dense row-major matrix: element (i, j) at data + i*ld + j.
 * dtype NYS_CSR describes a sparse matrix instead: data is a nys_sparse
 * handle from nys_sparse_create, n and d its shape, ld = d; every entry point
 * that takes an A accepts it (the sketch products then run in FP64; sketch_prec
 * is NYS_F64 or NYS_F32, see nys_sketch; the batched path takes dense
 * instances only). */
typedef struct {
  int64_t n, d, ld;
  nys_dtype dtype;   /* NYS_F32, NYS_F64, or NYS_CSR */
  const void* data;  /* device (a nys_sparse handle for NYS_CSR) */
} nys_dense;

/* ----------------------------------------------------------------- context */

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL means the null stream).  *out receives the handle. */
nys_status nys_ctx_create(int device, void* hip_stream, nys_ctx* out);
nys_status nys_ctx_destroy(nys_ctx ctx);
/* Rebind the context to another stream of the same device. */
nys_status nys_ctx_set_stream(nys_ctx ctx, void* hip_stream);
const char* nys_status_string(nys_status s);
/* Bytes of device workspace currently held by the context. */
size_t nys_ctx_workspace_bytes(nys_ctx ctx);

/* Caller-supplied device memory (the boundary's "PyTorch for device memory"):
 *
 * nys_workspace_query writes to *bytes an upper bound of the device memory
 * that admm_solve needs for `count` problems shaped like A at Nystrom rank at
 * most r_max (r_max = 0: plain CG), any sketch precision and loss: the
 * matvec partial sums (and the launch-shape tuner's trial buffer), the PCG
 * and ADMM vectors, the sketch and FP64-core temporaries, max(count, 2)
 * factors with their sketch state (two for a logistic refresh, one per
 * instance when count > 1 runs batched), the batched path's buffers, and for
 * a CSR A the handle's CSC copy; plus 1/8 + 16 MiB for the first-fit
 * carving.  It covers one call at a time on the context; factors kept across
 * calls, the warm-start network and pcg/sketch calls on wider shapes need
 * their own share.
 *
 * nys_ctx_set_workspace hands the context [dev_ptr, dev_ptr + bytes), device
 * memory of the context's device owned by the caller (e.g. a torch tensor).
 * From then on every device buffer the library would allocate while serving a
 * call on this context -- its own buffers, the factors and sparse handles it
 * creates, the batched path's buffers -- is carved from that range, and a
 * request that does not fit returns NYS_ERR_NOMEM; the library calls no
 * hipMalloc for them (hipGraph instantiation in the batched path keeps its
 * own runtime memory).  Setting a workspace releases the context's current
 * buffers (the cached A^T b and H_rho x are recomputed at the next step);
 * dev_ptr = NULL, bytes = 0 returns to the library's own allocation.
 * Factors and sparse handles carved from the range keep their blocks until
 * destroyed: destroy them before the caller frees the memory.  Blocks are
 * reused in stream order; nys_ctx_set_stream synchronises the old stream of a
 * context with a workspace.  nys_ctx_workspace_peak gives the largest number
 * of bytes of the range in use at once since it was set (0 without one). */
nys_status nys_workspace_query(nys_ctx ctx, const nys_dense* A, int r_max, int count,
                               size_t* bytes);
nys_status nys_ctx_set_workspace(nys_ctx ctx, void* dev_ptr, size_t bytes);
size_t nys_ctx_workspace_peak(nys_ctx ctx);

/* Kernel timing (instrumentation, not part of the method): while enabled the
 * library brackets every launch of the fused matvec-pair kernel with HIP
 * events on the context's stream (in the batched path: every true-residual
 * pass, one launch per row-width bucket over all active instances, outside
 * the captured PCG graphs).  nys_ctx_profile_stop synchronises the
 * stream, writes the number of launches that did a full pass (launches queued
 * past PCG convergence return at once and are not counted) and the summed
 * duration in ms of all timed launches, and disables the timing. */
nys_status nys_ctx_profile_start(nys_ctx ctx);
nys_status nys_ctx_profile_stop(nys_ctx ctx, long* launches, double* total_ms);
/* PCG timing (instrumentation, separate from the above): while enabled
 * (on = 1; enabling it clears the record) admm_step / admm_solve (one problem
 * at a time) bracket each subproblem's PCG solve with HIP events on the
 * context's stream.  nys_ctx_profile_pcg synchronises the stream and writes
 * the number of solves timed and their summed duration in ms (the rate of
 * PCG alone); the record stays until timing is enabled again. */
nys_status nys_ctx_profile_pcg_enable(nys_ctx ctx, int on);
nys_status nys_ctx_profile_pcg(nys_ctx ctx, long* solves, double* total_ms);

/* ------------------------------------------------------------------ sketch */

/* Standard Gaussian entries for the test matrix of Algorithm RandNysAppx,
 * drawn on the device: out[i] = sample offset + i of the stream of `seed`,
 * i < count (FP64, device pointer, caller-owned).  The stream is
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) with Box-Muller:
 * sample e comes from the Philox call with counter (q mod 2^32, q div 2^32,
 * 0, 0), q = e div 4, and key (seed mod 2^32, seed div 2^32); the call's
 * words (w0, w1) give samples 4q, 4q + 1 as sqrt(-2 ln u1) (cos, sin)(2 pi u2)
 * with u = (w + 1/2) 2^-32, and (w2, w3) give samples 4q + 2, 4q + 3.  So a
 * d x r test matrix is count = d * r from offset 0, and the block of columns
 * [k, k + m) of it is count = d * m from offset d * k.  Stream-ordered on the
 * context's stream (no synchronisation).  count < 0, out == NULL with
 * count > 0, or offset + count past 2^64: NYS_ERR_INVALID; count == 0 does
 * nothing. */
nys_status nys_gaussian(nys_ctx ctx, uint64_t seed, uint64_t offset, int64_t count, double* out);

/* Randomized Nystrom approximation of H = A^T diag(D) A + c I
 * (Algorithm RandNysAppx; eq. NysAppx; Section 2.2):
 *   Omega = qr(omega) (thin, FP64), Y = H Omega, nu = sqrt(d) eps(||Y||_2),
 *   Y_nu = Y + nu Omega, C = chol(Omega^T Y_nu) (upper), B = Y_nu C^-1,
 *   [U, Sigma] = svd(B), Lambda = max(0, Sigma^2 - nu).
 * eps(x) is the FP64 spacing of x (2^(floor(log2 x) - 52)) when
 * sketch_prec == NYS_F64 or A is sparse, and the FP32 spacing (exponent - 23)
 * otherwise.
 * If the Cholesky fails, nu is multiplied by 10 and the step repeated, at most
 * 3 times, then NYS_ERR_NOT_SPD.
 *
 *  omega       device, FP64, column-major d x r, Gaussian entries.
 *  r           columns to sketch, 1 <= r, total rank < d, total rank <= 1024.
 *  sketch_prec precision of Y = A^T (D (A Omega)): NYS_F64 (FP64 arithmetic,
 *              any A dtype), NYS_F32 (A FP32, FP32 MFMA, FP32 accumulate) or
 *              NYS_BF16 (A FP32 rounded to BF16 on load, BF16 MFMA, FP32
 *              accumulate).  The core (shift, Cholesky, SVD) is always FP64.
 *              For a sparse A (NYS_CSR) the products are FP64 sparse passes
 *              at either NYS_F64 or NYS_F32; NYS_F32 there keeps, beside the
 *              FP64 U, an FP32 copy of U that the preconditioner applies
 *              (half the bytes per application; PCG itself stays FP64), and
 *              NYS_BF16 is NYS_ERR_INVALID.  The factor's sketch_prec and
 *              kind (dense, sparse, symmetric) are fixed by its first call.
 *  F           in/out.  *F == NULL creates a factor of rank r.  *F != NULL
 *              appends r new columns to the existing sketch (the block step of
 *              Algorithm AdaptiveRandNysAppx: only the new block is
 *              orthonormalised and sketched) and recomputes the core, giving
 *              rank r_old + r.  A, D, c must be those of the earlier call. */
nys_status nys_sketch(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                      const double* omega, int r, nys_dtype sketch_prec, nys_factor* F);

/* Algorithm AdaptiveRandNysAppx: starting at rank s0, double the rank (the
 * last step cut to s_max) until (lambda_s + rho)/rho <= tol (eq. empCondNum,
 * tol = 1 + epsilon).  omega holds d x s_max Gaussian entries; block k uses the
 * next columns in order.  *F must be NULL on entry. */
nys_status nys_sketch_adaptive(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                               const double* omega, int s0, int s_max, double rho, double tol,
                               nys_dtype sketch_prec, nys_factor* F);

/* Factor from a given eigendecomposition (U device FP64 column-major d x r,
 * lambda_host descending, r entries).  Used to run PCG with an externally
 * built preconditioner. */
nys_status nys_factor_import(nys_ctx ctx, int64_t d, int r, const double* U,
                             const double* lambda_host, double nu, nys_factor* F);

/* rank, shift nu, lambda_s (smallest retained eigenvalue) and, if
 * lambda_host != NULL, all r eigenvalues in descending order. */
nys_status nys_factor_info(nys_factor F, int* rank, double* nu, double* lambda_s,
                           double* lambda_host);
/* Copy U (FP64, column-major d x rank) to the device buffer U_out. */
nys_status nys_factor_get_U(nys_ctx ctx, nys_factor F, double* U_out);
nys_status nys_factor_destroy(nys_factor F);

/* ------------------------------------------------------------ matvec pair */

/* v = (A^T diag(D) A + (c + rho) I) p : the Hessian-vector product of the
 * subproblem eq. (ADMMSubProb) (the T_mv of Table t-ComplexityComparison), in
 * one streaming pass over A with FP64 products and sums.  If pv_host != NULL
 * it receives p^T v = sum_i D_i (A p)_i^2 + (c + rho) ||p||^2 (synchronises).
 * p, v: device FP64 d-vectors, not overlapping.  rho + c >= 0. */
nys_status nys_hessian_apply(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                             double rho, const double* p, double* v, double* pv_host);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as nys_hessian_apply, computed without any allocation.  Its
 * workgroup partial sums live in a static scratch array of 16 MiB + 33 KiB
 * that the library holds on every device it runs on until the process ends
 * (looked up by nys_ctx_create); the launch uses the heuristic shape with at
 * most as many workgroups as that array holds partial rows (no autotuning,
 * which would allocate).  Limits: dense A (NYS_F32 with d <= 8192, NYS_F64
 * with d <= 4096); a sparse A or a wider one gives NYS_ERR_INVALID.  Calls on
 * one device share the array: calls that overlap on one device (from
 * different streams or contexts) race and must be serialised by the caller;
 * calls on one stream are ordered.  With D != NULL or pv_host != NULL the
 * call synchronises the stream (D is checked as in nys_hessian_apply). */
nys_status nys_hessian_apply_noalloc(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                                     double rho, const double* p, double* v, double* pv_host);

/* --------------------------------------------------------- preconditioner */

/* y = P^-1 w with, eq. (Nyspreconditioner),
 *   P^-1 = (lambda_s + rho) U (Lambda + rho I)^-1 U^T + (I - U U^T),
 * applied in O(d r) as y = w + U (s o (U^T w)), s_i = (lambda_s + rho)/(lambda_i + rho) - 1.
 * rho > 0.  w and y are device FP64 d-vectors and must not overlap. */
nys_status nys_precond_apply(nys_ctx ctx, nys_factor F, double rho, const double* w, double* y);

/* --------------------------------------------------------------------- PCG */

typedef struct {
  double tol;        /* stop when ||w||_2 <= tol ||rhs||_2 (tol_abs: ||w||_2 <= tol) */
  int tol_abs;
  int max_iter;      /* PCG iterations; 0 means 1000 */
  int check_every;   /* iterations queued ahead of the host's convergence check (1..4;
                        0 means 2); those queued after convergence return at once */
  int true_residual; /* 1: recompute rhs - H_rho x at the end and restart if above tol
                        (in ADMM at the steps chosen by nys_admm_opts.true_res_every) */
  int max_restarts;  /* restarts allowed by the true-residual check; 0 means 2 */
} nys_pcg_opts;

typedef struct {
  int iters;            /* PCG iterations over all restarts */
  int restarts;
  double rhs_norm;      /* ||rhs||_2 */
  double res_norm;      /* recursive ||w||_2 at exit */
  double true_res_norm; /* ||rhs - H_rho x||_2 with FP64 accumulation (if requested, else -1) */
  nys_status status;
} nys_pcg_info;

/* Algorithm Nystrom PCG on (A^T diag(D) A + (c + rho) I) x = rhs (eq.
 * ADMMSubProb).  x holds the initial guess on entry and the solution on exit.
 * F == NULL runs plain CG.  rhs = 0 returns x = 0 after 0 iterations.
 * The matrix-vector products multiply the stored A exactly in FP64 (products
 * and sums) whatever its storage type. */
nys_status pcg_solve(nys_ctx ctx, const nys_dense* A, const double* D, double c, double rho,
                     nys_factor F, const double* rhs, double* x, const nys_pcg_opts* opts,
                     nys_pcg_info* info);

/* -------------------------------------------------------------------- ADMM */

typedef struct {
  nys_loss loss;     /* NYS_LOSS_LS: 1/2||Ax - b||^2; NYS_LOSS_LOGISTIC: -sum(b t - log(1+e^t)), t = Ax */
  nys_dense A;
  const double* b;   /* device FP64 n-vector; labels in {0,1} for the logistic loss (eq. 9),
                        checked on the device by admm_step / admm_solve (NYS_ERR_INVALID
                        otherwise, NYS_ERR_NONFINITE for NaN/Inf) */
  double gamma;      /* l1 weight, >= 0 */
  double c;          /* smooth ridge part c/2 ||x||^2, >= 0 (elastic net: c = 1 - gamma);
                        must be 0 for the logistic loss (eq. 9 has no ridge term) */
} nys_problem;

typedef struct {
  double rho;            /* ADMM step size, > 0 */
  int rank;              /* fixed rank, or the initial rank s0 of the adaptive sketch;
                            0: inexact ADMM with plain CG (no sketch, no preconditioner;
                            the comparison method of Table t-ComplexityComparison) */
  int rank_max;          /* adaptive: s_max; <= rank means fixed rank */
  double ada_tol;        /* adaptive: Tol = 1 + epsilon of eq. (empCondNum) */
  int resketch_every;    /* logistic: rebuild the factor every k iterations (0: never) */
  nys_dtype sketch_prec; /* NYS_F64, NYS_F32 or NYS_BF16 */
  const double* omega;   /* device FP64 column-major d x max(rank, rank_max) Gaussian entries
                            (unused when rank = 0) */
  nys_pcg_opts pcg;      /* subproblem tolerance and limits */
  int tol_schedule;      /* 1: eps^{k+1} = sqrt(||r_p|| ||r_d||) absolute (Section 5 setup) */
  int max_iter;          /* ADMM iterations (admm_solve) */
  double eps_abs, eps_rel; /* Section 2.1 residual stop; eps_rel <= 0 disables */
  double rel_change_tol; /* ||z_k - z_{k+1}||_inf / ||z_k||_inf < tol stop; <= 0 disables */
  double kkt_tol;        /* stop when the relative KKT residual (eq. 31) <= kkt_tol; <= 0 disables */
  int kkt_every;         /* KKT check cadence (one extra matvec pair each); 0 means 10 */
  nys_factor factor;     /* optional prebuilt factor of A^T A + c I for this problem (lasso):
                            used instead of sketching and not destroyed (regularisation paths
                            reuse it across gamma); NULL: admm_solve builds and frees one */
  nys_ws_model warm_start; /* optional warm-start network: each subproblem also gets the
                            candidate start x0 = U c, c = net([U^T rhs, log gamma, log rho]);
                            PCG starts from whichever of x0 and the previous x has the smaller
                            residual (one extra pass over A, decided on the device);
                            NULL: previous x only */
  int ws_analytic;       /* 1: the candidate is x0 = U (Lambda + rho I)^-1 U^T rhs instead */
  int ws_every_step;     /* 0: propose only at the first step of a run (state k = 0, where
                            the previous iterate is the cold start x); 1: at every step */
  double* ws_features;   /* optional device (rank + 2): features of the step's subproblem */
  double* ws_target;     /* optional device (rank): U^T x of the step's solution */
  int true_res_every;    /* with pcg.true_residual set: the true residual of the subproblem
                            (one more pass over A) is computed at every k-th step (state k + 1
                            a multiple of k) and at the step that reaches max_iter in
                            admm_solve; the other steps stop PCG on its recursive residual
                            and a lasso run carries H_rho x = rhs - w to the next step.
                            0 means 1 (every step) */
} nys_admm_opts;

/* Caller-owned device FP64 d-vectors; x = z = u = 0 for a cold start.  k counts
 * completed iterations (resume = pass the saved state back). */
typedef struct {
  double* x;
  double* z;
  double* u;
  int k;
} nys_admm_state;

typedef struct {
  int iters;           /* ADMM iterations done by this call */
  long pcg_iters;      /* PCG iterations summed over those */
  int pcg_max;         /* largest PCG count of one subproblem */
  double r_p, r_d;     /* last primal / dual residual norms */
  double eta;          /* last relative KKT residual (eq. 31 or its logistic form), -1 if not computed */
  double obj;          /* objective at z, -1 if not computed */
  int rank;            /* Nystrom rank in use */
  int converged;       /* a stopping rule fired */
  nys_status status;   /* the first status other than NYS_OK met by any subproblem of the
                          call (NYS_ERR_MAXITER: some PCG solve stopped at pcg.max_iter above
                          its tolerance; the run went on), else NYS_OK */
  int ws_used;         /* subproblems that started from the warm-start candidate */
  double true_res_max; /* largest ||rhs - H_rho x|| / ||rhs|| over the subproblems whose true
                          residual was computed (FP64 accumulation); -1 if none */
  int maxiter_solves;  /* subproblems whose PCG stopped at pcg.max_iter above tolerance */
} nys_admm_info;

/* One iteration of Algorithm NysADMM: right-hand side (lasso: rho(z-u) + A^T b;
 * logistic: t = A x, w = sigma(t)(1-sigma(t)), rhs = rho(z-u) + A^T(w t + b - sigma(t))),
 * PCG warm-started at x, z = S_{gamma/rho}(x + u), u += x - z, residuals.
 * *F is the factor to precondition with; for the logistic loss it is rebuilt
 * in place when state->k is a multiple of opts->resketch_every (and created
 * if NULL).  Lasso runs keep A^T b and H_rho x of the last solve on the context
 * and reuse them in the next step when it has the same data pointers and
 * state->k advanced by one; a caller that edits A, b or x in place between
 * steps must start a new run (state->k = 0). */
nys_status admm_step(nys_ctx ctx, const nys_problem* P, const nys_admm_opts* O, nys_factor* F,
                     nys_admm_state* S, nys_admm_info* I);

/* Algorithm NysADMM / AdaNysADMM: build the factor (fixed or adaptive rank,
 * or take opts->factor), then iterate until max_iter or a stopping rule.
 * count > 1 with every problem least squares: the problems are solved
 * together in lockstep (batched path): one persistent matvec launch per row-
 * width bucket covers all of them (the buckets run concurrently on streams of
 * the context that are forked from and joined back to its stream, so all
 * work stays ordered on that stream), the PCG iterations run as a captured
 * hipGraph, converged instances drop out (per-instance masks).  KKT checks
 * are made at the end only in that mode.  Otherwise the problems are solved
 * one after another.  Arrays have length count. */
nys_status admm_solve(nys_ctx ctx, int count, const nys_problem* P, const nys_admm_opts* O,
                      nys_admm_state* S, nys_admm_info* I);

/* ------------------------------------------------------------ sparse A */

/* A sparse matrix for the matvec pair A^T (D (A p)) (E2006/sector-like data,
 * Section 5).  rowptr (n + 1), colidx (nnz) and val (nnz, FP32) are device
 * arrays in CSR order (column indices within a row in any order, no
 * duplicates); they stay owned by the caller and must outlive the handle.
 * The library builds a column-major copy (CSC, rows ascending within a
 * column) for the A^T pass; every product is an FP64 product of the stored
 * FP32 value, every sum FP64 in a fixed order.  Limits: nnz + d + 1024 <
 * 2^31 and at most 2^29 entries per row; otherwise (and for a decreasing
 * rowptr, rowptr[0] != 0, rowptr[n] != nnz or a column index outside
 * [0, d)) NYS_ERR_INVALID before any entry is placed. */
nys_status nys_sparse_create(nys_ctx ctx, int64_t n, int64_t d, int64_t nnz, const int* rowptr,
                             const int* colidx, const float* val, nys_sparse* out);
nys_status nys_sparse_destroy(nys_sparse S);

/* ------------------------------------------------------ kernel SVM (eq. 8) */

/* H = diag(b) K diag(b) with the RBF kernel K_ij = exp(-gamma ||a_i - a_j||^2)
 * (Section 3, support vector machine), written explicitly in FP32.
 * X: device FP32 n x p row-major features (leading dimension ldx >= p);
 * b: device FP64 labels (+-1), or NULL for K itself; H: device FP32 n x n
 * row-major (ldh >= n), caller-owned.  The squared distances are formed in
 * FP64 (FP64 products of the FP32 features), exp in FP64, then rounded. */
nys_status nys_kernel_rbf(nys_ctx ctx, const float* X, int64_t n, int64_t p, int64_t ldx,
                          const double* b, double gamma, float* H, int64_t ldh);

/* Algorithm RandNysAppx of the explicit symmetric PSD matrix H = K + c I
 * (K n x n, FP32 or FP64), then the FP64 core as in nys_sketch.
 * prec NYS_F64: Y = K Omega + c Omega with FP64 sums; NYS_F32 (FP32 K only):
 * Omega rounded to FP32 and K Omega by FP32 MFMA tiles with FP32 sums, the
 * shift nu set for 23 mantissa bits and U kept in FP32 for the
 * preconditioner, as in nys_sketch.  *F == NULL creates a factor, else
 * appends r columns (same prec).  omega: device FP64 n x r column-major
 * Gaussian entries. */
nys_status nys_sketch_sym(nys_ctx ctx, const nys_dense* K, double c, const double* omega, int r,
                          nys_dtype prec, nys_factor* F);

/* Algorithm Nystrom PCG on (K + (c + rho) I) x = rhs for an explicit symmetric
 * K (n x n): one pass over K per iteration, in blocks of columns.  F from
 * nys_sketch_sym (or NULL: plain CG).  Otherwise as pcg_solve. */
nys_status pcg_solve_sym(nys_ctx ctx, const nys_dense* K, double c, double rho, nys_factor F,
                         const double* rhs, double* x, const nys_pcg_opts* opts,
                         nys_pcg_info* info);

typedef struct {
  nys_dense H;       /* diag(b) K diag(b), n x n symmetric (e.g. from nys_kernel_rbf with b) */
  const double* b;   /* device FP64 labels, +-1 */
  double C;          /* box bound, > 0 */
} nys_svm_problem;

typedef struct {
  double rho;          /* ADMM step size, > 0 */
  int rank;            /* Nystrom rank (0: plain CG) */
  const double* omega; /* device FP64 n x rank Gaussian entries (unless factor is given) */
  nys_pcg_opts pcg;
  int max_iter;        /* ADMM iterations; 0 means 100 */
  double gap_tol;      /* stop when the relative duality gap <= gap_tol (<= 0: never) */
  int gap_every;       /* gap check cadence (one pass over H each); 0 means 10 */
  int true_res_every;  /* as in nys_admm_opts */
  nys_factor factor;   /* optional factor of H from nys_sketch_sym (kept) */
} nys_svm_opts;

typedef struct {
  int iters;
  long pcg_iters;
  int pcg_max;
  double r_p, r_d;     /* last ||x - z||, rho ||z_old - z|| (at checks and at the end) */
  double primal, dual; /* SVM primal (bias from the free variables) and dual objective at z */
  double gap, gap_rel; /* primal - dual and (primal - dual) / (1 + |primal|) */
  double bias;
  int rank;
  int converged;       /* the gap test fired */
  nys_status status;   /* as in nys_admm_info */
  double true_res_max; /* as in nys_admm_info */
  int maxiter_solves;  /* as in nys_admm_info */
} nys_svm_info;

/* Algorithm NysADMM on the SVM dual: minimize 1/2 x^T H x - 1^T x subject to
 * b^T x = 0, 0 <= x <= C.  x-update: PCG on (H + rho I) x = rho (z - u) + 1;
 * z-update: projection of x + u onto the constraint set (clip(v - mu b, 0, C)
 * with the root mu of b^T z(mu) = 0 found exactly by safeguarded Newton steps
 * on that piecewise-linear function); u += x - z.  The state (x, z, u: device FP64
 * n-vectors, x = z = u = 0 for a cold start) is updated in place; z is the
 * feasible dual solution. */
nys_status svm_solve(nys_ctx ctx, const nys_svm_problem* P, const nys_svm_opts* O,
                     nys_admm_state* S, nys_svm_info* I);

/* --------------------------------------------------- warm-start network */

/* A small network proposing the PCG start of the ADMM subproblem in the
 * Nystrom basis (not part of the paper's method; the previous iterate stays
 * the fallback and the judge, the tolerance is never relaxed):
 *   f  = [U^T rhs, log gamma, log rho]            (n_in = rank + 2)
 *   f' = (f - in_mean) / in_std
 *   h1 = gelu(f' W1 + b1), h2 = gelu(h1 W2 + b2), o = h2 W3 + b3   (n_out = rank)
 *   c  = o * out_scale [+ (Lambda + rho I)^-1 U^T rhs if analytic_skip],
 *   x0 = U c,  gelu(a) = a/2 (1 + erf(a / sqrt 2)).
 * params_host: W1 (n_in x hidden), b1, W2 (hidden x hidden), b2,
 * W3 (hidden x n_out), b3, row-major, FP64, nys_ws_param_count() values.
 * in_mean/in_std/out_scale may be NULL (0, 1, 1); analytic_skip needs
 * n_in = n_out + 2.  All arithmetic is FP64 on
 * the device.  Training data: the loss is (1/B) sum_ik W_ik (o_ik - T_ik)^2
 * with T the targets already divided by out_scale; X rows are raw features. */
size_t nys_ws_param_count(int n_in, int hidden, int n_out);
nys_status nys_ws_create(nys_ctx ctx, int n_in, int hidden, int n_out, const double* params_host,
                         const double* in_mean, const double* in_std, const double* out_scale,
                         int analytic_skip, nys_ws_model* out);
/* Arithmetic of the network from now on (the parameters carry over):
 *  NYS_F64   FP64 throughout (the default; matches the FP64 oracle to rounding);
 *  NYS_F32   FP32 master weights, activations, gradients and Adam state, matrix
 *            products on FP32 MFMA with FP32 accumulation;
 *  NYS_BF16  as NYS_F32 with every matrix-product operand (weights, activations,
 *            back-propagated gradients) rounded to BF16 for BF16 MFMA with FP32
 *            accumulation; the FP32 master weights take the Adam steps.
 * Switching to FP32/BF16 rounds the parameters to FP32 master copies; switching
 * back widens them.  Adam state restarts.  Inputs, targets, weights, outputs
 * and gradients cross the ABI in FP64 whatever the precision. */
nys_status nys_ws_set_precision(nys_ctx ctx, nys_ws_model m, nys_dtype prec);
nys_status nys_ws_get_params(nys_ctx ctx, nys_ws_model m, double* params_host);
/* out (device, batch x n_out) = o for the batch x n_in device rows X */
nys_status nys_ws_forward(nys_ctx ctx, nys_ws_model m, const double* X, int batch, double* out);
/* loss and, if grad_out != NULL, the gradient (device, nys_ws_param_count values,
 * same layout as params) for device X, T, W (W NULL: weights 1) */
nys_status nys_ws_loss_grad(nys_ctx ctx, nys_ws_model m, const double* X, const double* T,
                            const double* W, int batch, double* loss_host, double* grad_out);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) at rate lr */
nys_status nys_ws_train_step(nys_ctx ctx, nys_ws_model m, const double* X, const double* T,
                             const double* W, int batch, double lr, double* loss_host);
nys_status nys_ws_destroy(nys_ws_model m);

#ifdef __cplusplus
}
#endif
#endif /* NYSADMM_H */
