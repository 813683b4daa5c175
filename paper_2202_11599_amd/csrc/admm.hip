// ADMM drivers: Algorithm NysADMM (lasso) and its linearised form for l1
// logistic regression (Section 3.2), on top of pcg_run and the sketch.
//
// One iteration (admm_step):
//   lasso     rhs = rho (z - u) + A^T b            (A^T b computed once, cached)
//   logistic  t = A x, w = sigma(t)(1 - sigma(t)), s = w t + b - sigma(t),
//             rhs = rho (z - u) + A^T s            (one fused pass over A)
//   x         PCG on (A^T D A + (c + rho) I) x = rhs, warm-started at x
//   z, u      z = S_{gamma/rho}(x + u), u = u + x - z   (soft threshold)
//   residuals r_p = ||x - z||, r_d = rho ||z_old - z||   (Section 2.1)
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace nys {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

constexpr int kNS = 8;   // scalars reduced per ADMM vector pass

// rhs = rho (z - u) + v
__global__ void k_rhs(int64_t d, double rho, const double* __restrict__ z,
                      const double* __restrict__ u, const double* __restrict__ v,
                      double* __restrict__ rhs) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < d) rhs[j] = rho * (z[j] - u[j]) + v[j];
}

// y += a x
__global__ void k_axpy_inplace(int64_t d, double a, const double* __restrict__ x,
                               double* __restrict__ y) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < d) y[j] += a * x[j];
}

// Block partials of kNS scalars: entries 0..5 summed, 6..7 maxed.
__device__ void store_partials(double* vals, double* __restrict__ part, int nb) {
  __shared__ double sh[kNS][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < kNS; ++s) {
    const double v = s < 6 ? wave_sum(vals[s]) : wave_max(vals[s]);
    if (lane == 0) sh[s][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < kNS) {
    const int s = threadIdx.x;
    const double v = s < 6 ? ((sh[s][0] + sh[s][1]) + sh[s][2]) + sh[s][3]
                           : fmax(fmax(sh[s][0], sh[s][1]), fmax(sh[s][2], sh[s][3]));
    part[(int64_t)s * nb + blockIdx.x] = v;
  }
}

// z_old = z; z = S_kappa(x + u); u += x - z.  Partials:
// 0 ||x - z||^2, 1 ||z_old - z||^2, 2 ||x||^2, 3 ||z||^2, 4 ||u||^2, 5 ||z||_1,
// 6 ||z_old||_inf, 7 ||z - z_old||_inf
__global__ __launch_bounds__(256) void k_prox(int64_t d, double kappa, const double* __restrict__ x,
                                              double* __restrict__ z, double* __restrict__ u,
                                              double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (j < d) {
    const double xj = x[j], zo = z[j], uj = u[j];
    const double a = xj + uj;
    const double zn = copysign(fmax(fabs(a) - kappa, 0.0), a);
    const double un = uj + xj - zn;
    z[j] = zn;
    u[j] = un;
    v[0] = (xj - zn) * (xj - zn);
    v[1] = (zo - zn) * (zo - zn);
    v[2] = xj * xj;
    v[3] = zn * zn;
    v[4] = un * un;
    v[5] = fabs(zn);
    v[6] = fabs(zo);
    v[7] = fabs(zn - zo);
  }
  store_partials(v, part, gridDim.x);
}

// KKT partials for eq. (31): 0 ||z - S_gamma(z - g)||^2, 1 ||z||^2, 2 ||g||^2, 3 ||z||_1
__global__ __launch_bounds__(256) void k_kkt(int64_t d, double gamma, const double* __restrict__ z,
                                             const double* __restrict__ g,
                                             double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (j < d) {
    const double zj = z[j], gj = g[j];
    const double a = zj - gj;
    const double pr = copysign(fmax(fabs(a) - gamma, 0.0), a);
    v[0] = (zj - pr) * (zj - pr);
    v[1] = zj * zj;
    v[2] = gj * gj;
    v[3] = fabs(zj);
  }
  store_partials(v, part, gridDim.x);
}

// Final reduction of kNS x nb partials (one workgroup), plus the sum of the G
// Gram-pass partials q (index kNS).
__global__ __launch_bounds__(256) void k_reduce_scalars(const double* __restrict__ part, int nb,
                                                        const double* __restrict__ qpart, int G,
                                                        double* __restrict__ out) {
  __shared__ double sh[4];
  for (int s = 0; s <= kNS; ++s) {
    const double* src = s < kNS ? part + (int64_t)s * nb : qpart;
    const int cnt = s < kNS ? nb : G;
    const bool mx = (s == 6 || s == 7);
    double acc = 0.0;
    if (src != nullptr)
      for (int i = threadIdx.x; i < cnt; i += 256) acc = mx ? fmax(acc, src[i]) : acc + src[i];
    acc = mx ? wave_max(acc) : wave_sum(acc);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
      out[s] = mx ? fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]))
                  : ((sh[0] + sh[1]) + sh[2]) + sh[3];
  }
}

struct AdmmWs {
  double *atb, *rhs, *g, *Dw, *part, *scal, *xalt, *wss;
  int nb;
};

constexpr int kWsScratch = 4 * 1024 + 8;   // warm-start scratch (rank <= 1024)

size_t admm_ws_bytes_of(int64_t n, int64_t d) {
  const size_t vd = align_up(sizeof(double) * d);
  const size_t vn = align_up(sizeof(double) * std::max<int64_t>(n, 1));
  const size_t pb = align_up(sizeof(double) * kNS * nblk(d, 256));
  const size_t sc = align_up(sizeof(double) * (kNS + 1));
  return 4 * vd + vn + pb + sc + sizeof(double) * kWsScratch;
}

nys_status admm_workspace(nys_ctx ctx, int64_t n, int64_t d, AdmmWs* w) {
  w->nb = nblk(d, 256);
  const size_t vd = align_up(sizeof(double) * d);
  const size_t vn = align_up(sizeof(double) * std::max<int64_t>(n, 1));
  const size_t pb = align_up(sizeof(double) * kNS * w->nb);
  const size_t sc = align_up(sizeof(double) * (kNS + 1));
  NYS_TRY(ctx->admm_ws.reserve(admm_ws_bytes_of(n, d)));
  char* p = static_cast<char*>(ctx->admm_ws.ptr);
  w->atb = reinterpret_cast<double*>(p);
  w->rhs = reinterpret_cast<double*>(p + vd);
  w->g = reinterpret_cast<double*>(p + 2 * vd);
  w->Dw = reinterpret_cast<double*>(p + 3 * vd);
  w->part = reinterpret_cast<double*>(p + 3 * vd + vn);
  w->scal = reinterpret_cast<double*>(p + 3 * vd + vn + pb);
  w->xalt = reinterpret_cast<double*>(p + 3 * vd + vn + pb + sc);
  w->wss = reinterpret_cast<double*>(p + 4 * vd + vn + pb + sc);
  return NYS_OK;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// One fused pass v = A^T f(A p) into `out` (op-3 reduction); returns the sum
// of the per-row terms q when q_out != NULL (synchronises).
nys_status gram_pass(nys_ctx ctx, const nys_dense& A, int mode, const double* p, const double* aux,
                     double* auxout, double* out, const AdmmWs& w, bool want_q) {
  GramPlan pl;
  NYS_TRY(ctx_gram_plan(ctx, A, &pl));
  PcgWs ws;
  NYS_TRY(pcg_workspace(ctx, pl, A.d, 1, &ws));
  NYS_TRY(ctx_gram(ctx, A, pl, mode, p, aux, auxout, ws.ypart, ws.qpart, nullptr));
  // y and q partial counts come from the plan (one y partial for sparse A)
  NYS_TRY(launch_reduce_update(3, ws.ypart, pl.ny(), pl.ldy, ws.qpart, A.d, 0.0, nullptr, nullptr,
                               out, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, ws.st,
                               ctx->stream, pl.nq()));
  if (want_q) {
    // q partials are summed together with the KKT scalars by the caller
    hipLaunchKernelGGL(k_reduce_scalars, dim3(1), dim3(256), 0, ctx->stream, w.part, 0, ws.qpart,
                       pl.nq(), w.scal);
  }
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status read_scalars(nys_ctx ctx, const double* dev, double* host, int cnt) {
  NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, dev, sizeof(double) * cnt, hipMemcpyDeviceToHost,
                             ctx->stream));
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(host, ctx->host_pinned, sizeof(double) * cnt);
  return NYS_OK;
}

// Relative KKT residual at z (eq. 31 for lasso; the same form with the
// logistic gradient) and the objective at z.
nys_status kkt_and_objective(nys_ctx ctx, const nys_problem& P, const double* z, const AdmmWs& w,
                             double* eta, double* obj) {
  const nys_dense& A = P.A;
  const int mode = P.loss == NYS_LOSS_LS ? kModeLsGrad : kModeLogGrad;
  NYS_TRY(gram_pass(ctx, A, mode, z, P.b, nullptr, w.g, w, true));
  double q[kNS + 1];
  NYS_TRY(read_scalars(ctx, w.scal, q, kNS + 1));
  const double loss_term = q[kNS];   // ||Az - b||^2 (LS) or the logistic loss
  // the ridge part c z enters the smooth gradient
  if (P.c != 0.0)
    hipLaunchKernelGGL(k_axpy_inplace, dim3(blocks(A.d)), dim3(256), 0, ctx->stream, A.d, P.c, z,
                       w.g);
  hipLaunchKernelGGL(k_kkt, dim3(w.nb), dim3(256), 0, ctx->stream, A.d, P.gamma, z, w.g, w.part);
  hipLaunchKernelGGL(k_reduce_scalars, dim3(1), dim3(256), 0, ctx->stream, w.part, w.nb, nullptr,
                     0, w.scal);
  double s[kNS + 1];
  NYS_TRY(read_scalars(ctx, w.scal, s, kNS + 1));
  const double nz = std::sqrt(s[1]);
  if (P.loss == NYS_LOSS_LS) {
    *eta = std::sqrt(s[0]) / (1.0 + nz + std::sqrt(loss_term));
    *obj = 0.5 * loss_term + 0.5 * P.c * s[1] + P.gamma * s[3];
  } else {
    *eta = std::sqrt(s[0]) / (1.0 + nz + std::sqrt(s[2]));
    *obj = loss_term + P.gamma * s[3];
  }
  return NYS_OK;
}

}  // namespace

// pcg_abs > 0: the subproblem tolerance is max(pcg_abs, pcg_rel ||rhs||)
// (the schedule of the experiments section); otherwise O.pcg as given.
// last: the run ends with this step (its true residual is checked).
// host_scalars: read the residual norms back (a host round trip); without
// them the step leaves r_p, r_d and converged unset and the GPU runs on into
// the next step without waiting for the host.
nys_status admm_iter(nys_ctx ctx, const nys_problem& P, const nys_admm_opts& O, nys_factor* F,
                     nys_admm_state* S, nys_admm_info* I, double pcg_rel, double pcg_abs,
                     bool last, bool host_scalars) {
  const nys_dense& A = P.A;
  const int64_t d = A.d;
  AdmmWs w;
  NYS_TRY(admm_workspace(ctx, A.n, d, &w));
  hipStream_t st = ctx->stream;
  const double* D = nullptr;
  if (P.loss == NYS_LOSS_LS) {
    // A^T b is recomputed at the first step of a run (k = 0) and whenever the
    // previous step was on other data, so b may change between runs
    AtbKey key{A.data, P.b, A.n, d, A.ld, ctx->admm_ws.ptr};
    if (!(S->k > 0 && ctx->atb_key == key && ctx->atb_next_k == S->k)) {
      NYS_TRY(gram_pass(ctx, A, kModeTOnly, nullptr, P.b, nullptr, w.atb, w, false));
      ctx->atb_key = key;
    }
    ctx->atb_next_k = (int64_t)S->k + 1;
    hipLaunchKernelGGL(k_rhs, dim3(blocks(d)), dim3(256), 0, st, d, O.rho, S->z, S->u, w.atb,
                       w.rhs);
  } else {
    NYS_TRY(gram_pass(ctx, A, kModeLogit, S->x, P.b, w.Dw, w.g, w, false));
    hipLaunchKernelGGL(k_rhs, dim3(blocks(d)), dim3(256), 0, st, d, O.rho, S->z, S->u, w.g,
                       w.rhs);
    D = w.Dw;
    if (O.rank > 0 && (*F == nullptr || (O.resketch_every > 0 && S->k % O.resketch_every == 0))) {
      nys_factor nf = nullptr;
      NYS_TRY(sketch_rebuild(ctx, &A, D, P.c, O.omega, O.rank, O.sketch_prec, *F, &nf));
      if (*F != nullptr) nys_factor_destroy(*F);
      *F = nf;
    }
  }
  NYS_TRY_HIP(hipGetLastError());
  nys_pcg_opts po = O.pcg;
  const int tr_every = O.true_res_every > 0 ? O.true_res_every : 1;
  if (po.true_residual && !last && (S->k + 1) % tr_every != 0) po.true_residual = 0;
  double abs_tol = 0.0;
  if (pcg_rel > 0.0) {
    po.tol = pcg_rel;
    po.tol_abs = 0;
    abs_tol = pcg_abs;
  }
  // warm-start candidate (network or analytic) next to the previous iterate
  const double* x_alt = nullptr;
  const bool propose = O.ws_every_step != 0 || S->k == 0;
  if (*F != nullptr && (O.warm_start != nullptr || O.ws_analytic) && propose) {
    if (O.warm_start != nullptr)
      NYS_TRY(ws_propose(ctx, O.warm_start, *F, w.rhs, P.gamma, O.rho, w.xalt, w.wss,
                         O.ws_features));
    else
      NYS_TRY(ws_analytic(ctx, *F, w.rhs, O.rho, w.xalt, w.wss));
    x_alt = w.xalt;
  }
  if (*F != nullptr && O.ws_features != nullptr && (O.warm_start == nullptr || !propose))
    NYS_TRY(ws_record(ctx, *F, w.rhs, P.gamma, O.rho, nullptr, O.ws_features, nullptr, w.wss));
  nys_pcg_info pinfo{};
  int used_alt = 0;
  // lasso: within a run x is only changed by PCG, so H_rho x carries over
  // from one step's solve to the next (tagged with the step counter)
  // instrumentation: HIP events around the PCG solve (rate of PCG alone)
  const bool tpcg = ctx->pcg_time_on;
  if (tpcg) {
    while (ctx->pcg_ev.size() < ctx->pcg_used + 2) {
      hipEvent_t e;
      NYS_TRY_HIP(hipEventCreate(&e));
      ctx->pcg_ev.push_back(e);
    }
    NYS_TRY_HIP(hipEventRecord(ctx->pcg_ev[ctx->pcg_used], st));
  }
  nys_status ps = pcg_run(ctx, A, D, P.c, O.rho, *F, w.rhs, S->x, po, &pinfo, abs_tol,
                          P.loss == NYS_LOSS_LS ? (int64_t)S->k : -1, x_alt, &used_alt);
  if (tpcg) {
    NYS_TRY_HIP(hipEventRecord(ctx->pcg_ev[ctx->pcg_used + 1], st));
    ctx->pcg_used += 2;
  }
  if (*F != nullptr && O.ws_target != nullptr && (ps == NYS_OK || ps == NYS_ERR_MAXITER))
    NYS_TRY(ws_record(ctx, *F, nullptr, P.gamma, O.rho, S->x, nullptr, O.ws_target, w.wss));
  if (ps != NYS_OK && ps != NYS_ERR_MAXITER) {
    if (I) I->status = ps;
    return ps;
  }
  hipLaunchKernelGGL(k_prox, dim3(w.nb), dim3(256), 0, st, d, P.gamma / O.rho, S->x, S->z, S->u,
                     w.part);
  double s[kNS + 1];
  if (host_scalars) {
    hipLaunchKernelGGL(k_reduce_scalars, dim3(1), dim3(256), 0, st, w.part, w.nb, nullptr, 0,
                       w.scal);
    NYS_TRY(read_scalars(ctx, w.scal, s, kNS + 1));
  } else {
    NYS_TRY_HIP(hipGetLastError());
  }
  S->k += 1;
  if (I) {
    I->iters += 1;
    I->pcg_iters += pinfo.iters;
    I->pcg_max = std::max(I->pcg_max, pinfo.iters);
    I->rank = (*F) ? (*F)->r : 0;
    I->status = ps;
    I->maxiter_solves = ps == NYS_ERR_MAXITER ? 1 : 0;
    I->ws_used = used_alt;
    I->true_res_max = (pinfo.true_res_norm >= 0.0 && pinfo.rhs_norm > 0.0)
                          ? pinfo.true_res_norm / pinfo.rhs_norm
                          : (pinfo.true_res_norm >= 0.0 ? 0.0 : -1.0);
    I->converged = 0;
    if (!host_scalars) return ps == NYS_ERR_MAXITER ? NYS_OK : ps;
    I->r_p = std::sqrt(s[0]);
    I->r_d = O.rho * std::sqrt(s[1]);
    // Section 2.1 residual stop
    bool stop = false;
    if (O.eps_rel > 0.0) {
      const double tp = O.eps_abs + O.eps_rel * std::max(std::sqrt(s[2]), std::sqrt(s[3]));
      const double td = O.eps_abs + O.eps_rel * O.rho * std::sqrt(s[4]);
      stop = (I->r_p <= tp) && (I->r_d <= td);
    }
    if (O.rel_change_tol > 0.0 && S->k > 1 && s[6] > 0.0 && s[7] / s[6] < O.rel_change_tol)
      stop = true;
    I->converged = stop ? 1 : 0;
  }
  return ps == NYS_ERR_MAXITER ? NYS_OK : ps;
}

size_t admm_ws_bytes(int64_t n, int64_t d) { return admm_ws_bytes_of(n, d); }

nys_status admm_kkt(nys_ctx ctx, const nys_problem& P, const double* z, double* eta, double* obj) {
  AdmmWs w;
  NYS_TRY(admm_workspace(ctx, P.A.n, P.A.d, &w));
  return kkt_and_objective(ctx, P, z, w, eta, obj);
}

nys_status validate_problem(const nys_problem* P, const nys_admm_opts* O) {
  if (P == nullptr || O == nullptr) return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(&P->A));
  if (P->b == nullptr || !(P->gamma >= 0.0) || !(P->c >= 0.0)) return NYS_ERR_INVALID;
  if (P->loss != NYS_LOSS_LS && P->loss != NYS_LOSS_LOGISTIC) return NYS_ERR_INVALID;
  // eq. (9) has no ridge term: the logistic objective and KKT residual are
  // defined for c = 0 only
  if (P->loss == NYS_LOSS_LOGISTIC && P->c != 0.0) return NYS_ERR_INVALID;
  if (!(O->rho > 0.0) || O->rank < 0 || O->rank >= P->A.d) return NYS_ERR_INVALID;
  if (O->rank == 0) {
    // inexact ADMM with plain CG: no sketch, no factor, no warm-start candidate
    if (O->rank_max > 0 || O->factor != nullptr || O->warm_start != nullptr ||
        O->ws_analytic || O->ws_features != nullptr || O->ws_target != nullptr)
      return NYS_ERR_INVALID;
    return NYS_OK;
  }
  if (O->omega == nullptr) return NYS_ERR_INVALID;
  if (O->warm_start != nullptr && !(P->gamma > 0.0)) return NYS_ERR_INVALID;
  if (O->rank_max > O->rank && (O->rank_max >= P->A.d || O->rank_max > 1024))
    return NYS_ERR_INVALID;
  return NYS_OK;
}

}  // namespace nys

using namespace nys;

extern "C" {

nys_status admm_step(nys_ctx ctx, const nys_problem* P, const nys_admm_opts* O, nys_factor* F,
                     nys_admm_state* S, nys_admm_info* I) {
  if (ctx == nullptr || F == nullptr || S == nullptr) return NYS_ERR_INVALID;
  NYS_TRY(validate_problem(P, O));
  if (S->x == nullptr || S->z == nullptr || S->u == nullptr) return NYS_ERR_INVALID;
  if (*F != nullptr && (*F)->d != P->A.d) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  // logistic labels b in {0, 1} (eq. 9)
  if (P->loss == NYS_LOSS_LOGISTIC) NYS_TRY(check_vector(ctx, P->b, P->A.n, 1));
  if (I) *I = nys_admm_info{};
  if (I) I->eta = I->obj = -1.0;
  if (O->rank == 0 && *F != nullptr) return NYS_ERR_INVALID;
  if (P->loss == NYS_LOSS_LS && *F == nullptr && O->rank > 0) {
    NYS_TRY(nys_sketch(ctx, &P->A, nullptr, P->c, O->omega, O->rank, O->sketch_prec, F));
  }
  return admm_iter(ctx, *P, *O, F, S, I, 0.0, 0.0, false, true);
}

nys_status admm_solve(nys_ctx ctx, int count, const nys_problem* P, const nys_admm_opts* O,
                      nys_admm_state* S, nys_admm_info* I) {
  if (ctx == nullptr || count < 1 || P == nullptr || O == nullptr || S == nullptr)
    return NYS_ERR_INVALID;
  for (int q = 0; q < count; ++q) {
    NYS_TRY(validate_problem(&P[q], &O[q]));
    if (S[q].x == nullptr || S[q].z == nullptr || S[q].u == nullptr) return NYS_ERR_INVALID;
  }
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  for (int q = 0; q < count; ++q)
    if (P[q].loss == NYS_LOSS_LOGISTIC) NYS_TRY(check_vector(ctx, P[q].b, P[q].A.n, 1));
  ctx->atb_key = AtbKey{};   // b may have changed in place since an earlier call
  ctx->hx_key = AtbKey{};    // and x since an earlier solve
  bool batched = count > 1;
  for (int q = 0; q < count; ++q) {
    if (P[q].loss != NYS_LOSS_LS || O[q].tol_schedule || O[q].kkt_tol > 0.0 || O[q].rank == 0 ||
        P[q].A.dtype == NYS_CSR || P[q].A.d > gram_max_cols(P[q].A.dtype))
      batched = false;
    if (O[q].warm_start != nullptr || O[q].ws_analytic || O[q].ws_features != nullptr ||
        O[q].ws_target != nullptr)
      batched = false;
    if (O[q].factor != nullptr && O[q].factor->d != P[q].A.d) return NYS_ERR_INVALID;
  }
  if (batched) return admm_solve_batched(ctx, count, P, O, S, I);
  nys_status worst = NYS_OK;
  for (int q = 0; q < count; ++q) {
    const nys_problem& p = P[q];
    const nys_admm_opts& o = O[q];
    nys_admm_info info{};
    info.eta = info.obj = info.true_res_max = -1.0;
    nys_factor F = o.factor;
    const bool own = (F == nullptr);
    nys_status s = NYS_OK;
    if (p.loss == NYS_LOSS_LS && F == nullptr && o.rank > 0) {
      if (o.rank_max > o.rank && o.ada_tol >= 1.0)
        s = nys_sketch_adaptive(ctx, &p.A, nullptr, p.c, o.omega, o.rank, o.rank_max, o.rho,
                                o.ada_tol, o.sketch_prec, &F);
      else
        s = nys_sketch(ctx, &p.A, nullptr, p.c, o.omega, o.rank, o.sketch_prec, &F);
    }
    AdmmWs w;
    if (s == NYS_OK) s = admm_workspace(ctx, p.A.n, p.A.d, &w);
    double eps_next = 0.0;
    const int kkt_every = o.kkt_every > 0 ? o.kkt_every : 10;
    const int max_iter = o.max_iter > 0 ? o.max_iter : 100;
    for (int it = 0; s == NYS_OK && it < max_iter; ++it) {
      nys_admm_info step{};
      // schedule: eps^0 = 1e-2 ||rhs||, then max(sqrt(r_p r_d), pcg.tol ||rhs||)
      double rel = 0.0, abs_tol = 0.0;
      if (o.tol_schedule) {
        rel = (it == 0) ? 1e-2 : o.pcg.tol;
        abs_tol = (it == 0) ? 0.0 : eps_next;
      }
      const bool last = it + 1 == max_iter;
      const bool kkt_now = o.kkt_tol > 0.0 && (it + 1) % kkt_every == 0;
      // the residual norms are needed on the host by the residual stopping
      // rules, the tolerance schedule, a KKT check and at the end
      const bool host = last || kkt_now || o.tol_schedule || o.eps_rel > 0.0 ||
                        o.rel_change_tol > 0.0;
      s = admm_iter(ctx, p, o, &F, &S[q], &step, rel, abs_tol, last, host);
      if (s != NYS_OK) break;
      info.iters += 1;
      info.pcg_iters += step.pcg_iters;
      info.pcg_max = std::max(info.pcg_max, step.pcg_max);
      if (host) {
        info.r_p = step.r_p;
        info.r_d = step.r_d;
      }
      info.rank = step.rank;
      if (info.status == NYS_OK) info.status = step.status;   // sticky: first non-OK
      info.maxiter_solves += step.maxiter_solves;
      info.ws_used += step.ws_used;
      info.true_res_max = std::max(info.true_res_max, step.true_res_max);
      if (o.tol_schedule) eps_next = std::sqrt(step.r_p * step.r_d);
      bool stop = step.converged != 0;
      if (o.kkt_tol > 0.0 && ((it + 1) % kkt_every == 0 || stop)) {
        s = kkt_and_objective(ctx, p, S[q].z, w, &info.eta, &info.obj);
        if (s != NYS_OK) break;
        stop = info.eta <= o.kkt_tol;
        if (o.eps_rel > 0.0 || o.rel_change_tol > 0.0) stop = stop || step.converged;
      }
      if (stop) {
        info.converged = 1;
        break;
      }
    }
    if (s == NYS_OK && info.eta < 0.0)
      s = kkt_and_objective(ctx, p, S[q].z, w, &info.eta, &info.obj);
    if (s != NYS_OK) info.status = s;
    if (F && own) nys_factor_destroy(F);
    if (I) I[q] = info;
    if (s != NYS_OK && worst == NYS_OK) worst = s;
  }
  return worst;
}

}  // extern "C"
