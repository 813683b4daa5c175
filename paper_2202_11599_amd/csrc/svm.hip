// Kernel SVM dual (Section 3, eq. 8) by NysADMM:
//
//   minimize 1/2 x^T H x - 1^T x   s.t.  b^T x = 0,  0 <= x <= C,
//   H = diag(b) K diag(b),  K_ij = exp(-gamma ||a_i - a_j||^2)  (RBF)
//
// The matrix H is formed once, explicitly, in FP32 (n x n; 1.6 GB at
// n = 20000, 10 GB at n = 50000 -- HBM holds it, and a pass over it is far
// cheaper than regenerating the kernel on the fly: one n x n x p GEMM per
// matvec).  Then, per ADMM iteration:
//   x   PCG on (H + rho I) x = rho (z - u) + 1, Nystrom-preconditioned, one
//       column-blocked pass over H per iteration (k_rowdot)
//   z   projection of x + u onto {0 <= z <= C, b^T z = 0}: clip(v - mu b)
//       with the multiplier mu found by safeguarded Newton steps on the
//       piecewise-linear b^T z(mu) (one workgroup)
//   u   u + x - z
// and every gap_every iterations the duality gap between the SVM primal (bias
// from the free variables, as LIBSVM) and the dual at the feasible z.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace nys {
namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block reductions over NW wavefronts in a fixed order; every thread gets the
// result
enum RedOp { kSum, kMin, kMax };
template <RedOp OP, int NW = 16>
__device__ double block_reduce(double v, double* sh) {
  v = OP == kSum ? wsum(v) : (OP == kMin ? wmin(v) : wmax(v));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < NW; ++i)
    r = OP == kSum ? r + sh[i] : (OP == kMin ? fmin(r, sh[i]) : fmax(r, sh[i]));
  __syncthreads();
  return r;
}

// sq_i = ||a_i||^2 (FP64 sums of the FP32 features)
__global__ __launch_bounds__(256) void k_rownorm2(const float* __restrict__ X, int64_t n, int64_t p,
                                                  int64_t ldx, double* __restrict__ sq) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t k = lane; k < p; k += 64) {
    const double v = X[i * ldx + k];
    s = fma(v, v, s);
  }
  s = wsum(s);
  if (lane == 0) sq[i] = s;
}

// H rows i0 .. i0+rows-1 from G = X_rows X^T (FP64):
// H_ij = b_i b_j exp(-gamma max(0, sq_i + sq_j - 2 G_ij)) rounded to FP32
__global__ __launch_bounds__(256) void k_rbf_rows(const double* __restrict__ G, int64_t rows,
                                                  int64_t n, int64_t i0,
                                                  const double* __restrict__ sq,
                                                  const double* __restrict__ b, double gamma,
                                                  float* __restrict__ H, int64_t ldh) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * n) return;
  const int64_t r = e / n, j = e % n;
  const int64_t i = i0 + r;
  const double d2 = fmax(0.0, sq[i] + sq[j] - 2.0 * G[e]);
  double v = exp(-gamma * d2);
  if (b != nullptr) v *= b[i] * b[j];
  H[i * ldh + j] = (float)v;
}

// rhs = rho (z - u) + 1
__global__ void k_svm_rhs(int64_t n, double rho, const double* __restrict__ z,
                          const double* __restrict__ u, double* __restrict__ rhs) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < n) rhs[j] = rho * (z[j] - u[j]) + 1.0;
}

constexpr int kSvmNS = 8;   // scalars of the projection pass

// Sum of NV values over a block of NW wavefronts in a fixed order; every
// thread gets the sums.  sh holds (NW + 1) NV doubles.  Thread k < NV adds the
// NW wavefront partials of value k, so each thread reads NV sums back rather
// than all NV x NW partials.
template <int NV, int NW>
__device__ void block_sums(double (&v)[NV], double* sh) {
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wsum(v[k]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * NW + (threadIdx.x >> 6)] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double r = 0.0;
    for (int w = 0; w < NW; ++w) r += sh[threadIdx.x * NW + w];
    sh[NV * NW + threadIdx.x] = r;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = sh[NV * NW + k];
  __syncthreads();
}

// phi(mu) = b^T clip(v - mu b, 0, C) and the four clip counts (b = +1 at C,
// b = +1 at 0, b = -1 at 0, b = -1 at C) at the three points mu[0..2] in one
// pass: out[5 m + 0] = phi(mu[m]), out[5 m + 1..4] = the counts.  Each count
// moves one way as mu grows, so equal counts at both ends of a bracket mean no
// entry changes side inside it and phi is linear there; n minus the counts is
// the number of free entries, the slope of -phi.  VPT > 0: the thread's
// entries i = tid + kPT k are held in registers (v, sign bits); VPT = 0: read
// v = x + u and b from memory.
constexpr int kPT = 512;   // threads of the projection workgroup
constexpr int kPM = 3;     // points per pass
template <int VPT>
__device__ void phi_counts(const double (&vr)[VPT > 0 ? VPT : 1], unsigned long long sgn,
                           const double* __restrict__ x, const double* __restrict__ u,
                           const double* __restrict__ b, int64_t n, double C,
                           const double (&mu)[kPM], double (&out)[5 * kPM], double* sh) {
  double f[kPM];
  int cnt[4 * kPM];   // per-thread counts (integers: fewer registers)
#pragma unroll
  for (int m = 0; m < kPM; ++m) f[m] = 0.0;
#pragma unroll
  for (int k = 0; k < 4 * kPM; ++k) cnt[k] = 0;
  auto one = [&](double v, bool pos) {
#pragma unroll
    for (int m = 0; m < kPM; ++m) {
      const double a = pos ? v - mu[m] : v + mu[m];
      const double c = fmin(fmax(a, 0.0), C);
      f[m] += pos ? c : -c;
      cnt[4 * m + (pos ? 0 : 3)] += (a >= C) ? 1 : 0;
      cnt[4 * m + (pos ? 1 : 2)] += (a <= 0.0) ? 1 : 0;
    }
  };
  if (VPT > 0) {
#pragma unroll
    for (int k = 0; k < (VPT > 0 ? VPT : 1); ++k)
      if ((int64_t)threadIdx.x + kPT * k < n) one(vr[k], (sgn >> k) & 1ull);
  } else {
    for (int64_t i = threadIdx.x; i < n; i += kPT) one(x[i] + u[i], b[i] > 0.0);
  }
#pragma unroll
  for (int m = 0; m < kPM; ++m) {
    out[5 * m] = f[m];
#pragma unroll
    for (int q = 0; q < 4; ++q) out[5 * m + 1 + q] = (double)cnt[4 * m + q];
  }
  block_sums<5 * kPM, kPT / 64>(out, sh);
}

// z = projection of v = x + u onto {0 <= z <= C, b^T z = 0}, u += x - z, and
// out[0..7] = ||x - z||^2, ||z_old - z||^2, ||x||^2, ||z||^2, ||u||^2, b^T z,
// mu, passes.  One workgroup; every decision is block-uniform (all threads
// hold the same sums).  phi is non-increasing and piecewise linear in mu; the
// bracket [lo, hi] (phi(lo) > 0 >= phi(hi)) shrinks by passes that each
// evaluate three points: a Newton step from either end along the slope given
// by that end's free count (exact when that end lies on the root's linear
// piece) and the midpoint (which bounds the work by that of bisection).  Once
// the counts agree at both ends, the secant step on the linear piece is exact.
template <int VPT>
__global__ __launch_bounds__(kPT) void k_svm_project(int64_t n, const double* __restrict__ x,
                                                      const double* __restrict__ b, double C,
                                                      double* __restrict__ z,
                                                      double* __restrict__ u,
                                                      double* __restrict__ out) {
  __shared__ double sh[5 * kPM * (kPT / 64 + 1)];
  if (n <= 0) return;
  double vr[VPT > 0 ? VPT : 1];
  unsigned long long sgn = 0;
  // bracket: below lo every b = +1 entry clips to C and every b = -1 entry to
  // 0 (phi >= 0); above hi the reverse (phi <= 0)
  double lo_l = 0.0, hi_l = 0.0;
  auto brk = [&](double v, bool pos) {
    if (pos) {
      lo_l = fmin(lo_l, v - C);
      hi_l = fmax(hi_l, v);
    } else {
      lo_l = fmin(lo_l, -v);
      hi_l = fmax(hi_l, C - v);
    }
  };
  constexpr int CH = VPT >= 8 ? 8 : (VPT > 0 ? VPT : 1);   // entries loaded together
  if (VPT > 0) {
#pragma unroll
    for (int k0 = 0; k0 < (VPT > 0 ? VPT : 1); k0 += CH) {
      // in-bounds loads for every lane (index 0 past the end), issued together
      double xs[CH], us[CH], bs[CH];
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int64_t i = (int64_t)threadIdx.x + kPT * (k0 + t);
        const int64_t ic = i < n ? i : 0;
        xs[t] = x[ic];
        us[t] = u[ic];
        bs[t] = b[ic];
      }
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int64_t i = (int64_t)threadIdx.x + kPT * (k0 + t);
        vr[k0 + t] = 0.0;
        if (i < n) {
          vr[k0 + t] = xs[t] + us[t];
          const bool pos = bs[t] > 0.0;
          if (pos) sgn |= 1ull << (k0 + t);
          brk(vr[k0 + t], pos);
        }
      }
    }
  } else {
    vr[0] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kPT) brk(x[i] + u[i], b[i] > 0.0);
  }
  double lo = block_reduce<kMin, kPT / 64>(lo_l, sh);
  double hi = block_reduce<kMax, kPT / 64>(hi_l, sh);
  double elo[5], ehi[5], e[5 * kPM];
  {
    const double m0[kPM] = {lo, hi, hi};
    phi_counts<VPT>(vr, sgn, x, u, b, n, C, m0, e, sh);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      elo[k] = e[k];
      ehi[k] = e[5 + k];
    }
  }
  const double nd = (double)n;
  int passes = 1;
  for (; passes < 200; ++passes) {
    if (elo[1] == ehi[1] && elo[2] == ehi[2] && elo[3] == ehi[3] && elo[4] == ehi[4]) break;
    if (elo[0] == 0.0 || ehi[0] == 0.0) break;   // an end is a root
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    double m[kPM];
    const double flo = nd - (((elo[1] + elo[2]) + elo[3]) + elo[4]);
    const double fhi = nd - (((ehi[1] + ehi[2]) + ehi[3]) + ehi[4]);
    m[0] = flo > 0.0 ? lo + elo[0] / flo : mid;
    m[1] = fhi > 0.0 ? hi + ehi[0] / fhi : mid;
    m[2] = mid;
    if (!(m[0] > lo && m[0] < hi)) m[0] = mid;
    if (!(m[1] > lo && m[1] < hi)) m[1] = mid;
    phi_counts<VPT>(vr, sgn, x, u, b, n, C, m, e, sh);
    // lo = the largest point with phi > 0, hi = the smallest with phi <= 0
#pragma unroll
    for (int q = 0; q < kPM; ++q) {
      if (e[5 * q] > 0.0) {
        if (m[q] > lo) {
          lo = m[q];
#pragma unroll
          for (int k = 0; k < 5; ++k) elo[k] = e[5 * q + k];
        }
      } else if (m[q] < hi) {
        hi = m[q];
#pragma unroll
        for (int k = 0; k < 5; ++k) ehi[k] = e[5 * q + k];
      }
    }
  }
  const double flo = elo[0], fhi = ehi[0];
  // phi is linear on the final bracket: one secant step (exact; an end that
  // is a root is returned as it is)
  double mu = (flo == fhi) ? lo : lo + flo * (hi - lo) / (flo - fhi);
  mu = fmin(fmax(mu, lo), hi);
  double st[6] = {0, 0, 0, 0, 0, 0};
  auto fin = [&](int64_t i, double v, double bi, double xi, double zo) {
    const double zn = fmin(fmax(v - mu * bi, 0.0), C);
    const double un = v - zn;            // u + x - z with v = x + u
    z[i] = zn;
    u[i] = un;
    st[0] = fma(xi - zn, xi - zn, st[0]);
    st[1] = fma(zo - zn, zo - zn, st[1]);
    st[2] = fma(xi, xi, st[2]);
    st[3] = fma(zn, zn, st[3]);
    st[4] = fma(un, un, st[4]);
    st[5] = fma(bi, zn, st[5]);
  };
  // eight entries per lane per trip, their loads issued together (in-bounds
  // index 0 for lanes past the end); v = x + u again, as in the first pass
  for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * kPT) {
    double xs[8], us[8], bs[8], zs[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t i = i0 + kPT * t;
      const int64_t ic = i < n ? i : 0;
      xs[t] = x[ic];
      us[t] = u[ic];
      bs[t] = b[ic];
      zs[t] = z[ic];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t i = i0 + kPT * t;
      if (i < n) fin(i, xs[t] + us[t], bs[t], xs[t], zs[t]);
    }
  }
  block_sums<6, kPT / 64>(st, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k] = st[k];
    out[6] = mu;
    out[7] = passes;
  }
}

// Duality gap sums at the feasible z, w = H z (g_i = b_i w_i):
// pass 0: out[0] = z^T w, out[1] = 1^T z, out[2] = sum over free z of
// b_i - g_i, out[3] = free count, out[4] = max over the lower-bound set of
// b_i - g_i, out[5] = min over the upper-bound set; pass 1: out[6] = sum of
// max(0, 1 - w_i - b_i beta).
__global__ __launch_bounds__(kPT) void k_svm_gap(int64_t n, const double* __restrict__ z,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ b, double C,
                                                  int pass, double beta,
                                                  double* __restrict__ out) {
  __shared__ double sh[16];
  if (pass == 0) {
    double zw = 0.0, sz = 0.0, fs = 0.0, fc = 0.0, lo = -INFINITY, hi = INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += kPT) {
      const double zi = z[i], bi = b[i], wi = w[i];
      const double r = bi - bi * wi;   // b_i - g_i
      zw = fma(zi, wi, zw);
      sz += zi;
      if (zi > 0.0 && zi < C) {
        fs += r;
        fc += 1.0;
      } else if ((zi <= 0.0) == (bi > 0.0)) {
        lo = fmax(lo, r);    // z = 0, b = +1  or  z = C, b = -1
      } else {
        hi = fmin(hi, r);    // z = 0, b = -1  or  z = C, b = +1
      }
    }
    const double a0 = block_reduce<kSum, kPT / 64>(zw, sh);
    const double a1 = block_reduce<kSum, kPT / 64>(sz, sh);
    const double a2 = block_reduce<kSum, kPT / 64>(fs, sh);
    const double a3 = block_reduce<kSum, kPT / 64>(fc, sh);
    const double a4 = block_reduce<kMax, kPT / 64>(lo, sh);
    const double a5 = block_reduce<kMin, kPT / 64>(hi, sh);
    if (threadIdx.x == 0) {
      out[0] = a0;
      out[1] = a1;
      out[2] = a2;
      out[3] = a3;
      out[4] = a4;
      out[5] = a5;
    }
  } else {
    double hs = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kPT) hs += fmax(0.0, 1.0 - w[i] - b[i] * beta);
    const double a6 = block_reduce<kSum, kPT / 64>(hs, sh);
    if (threadIdx.x == 0) out[6] = a6;
  }
}

inline unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

struct SvmWs {
  double *rhs, *w, *scal;
};

nys_status svm_workspace(nys_ctx ctx, int64_t n, SvmWs* ws) {
  const size_t vn = align_up(sizeof(double) * (size_t)n);
  NYS_TRY(ctx->svm_ws.reserve(2 * vn + align_up(sizeof(double) * 32)));
  char* p = static_cast<char*>(ctx->svm_ws.ptr);
  ws->rhs = reinterpret_cast<double*>(p);
  ws->w = reinterpret_cast<double*>(p + vn);
  ws->scal = reinterpret_cast<double*>(p + 2 * vn);
  return NYS_OK;
}

nys_status read_svm(nys_ctx ctx, const double* dev, double* host, int cnt) {
  NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, dev, sizeof(double) * cnt, hipMemcpyDeviceToHost,
                             ctx->stream));
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(host, ctx->host_pinned, sizeof(double) * cnt);
  return NYS_OK;
}

// out = H p (one column-blocked pass, fixed-order reduction)
nys_status svm_matvec(nys_ctx ctx, const nys_dense& H, const double* p, double* out) {
  GramPlan pl = make_symv_plan(H, ctx->num_cu);
  PcgWs ws;
  NYS_TRY(pcg_workspace(ctx, pl, H.d, 1, &ws));
  NYS_TRY(ctx_gram(ctx, H, pl, kModeHess, p, nullptr, nullptr, ws.ypart, ws.qpart, nullptr));
  return launch_reduce_update(3, ws.ypart, pl.ny(), pl.ldy, ws.qpart, H.d, 0.0, nullptr, nullptr,
                              out, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, ws.st,
                              ctx->stream, pl.nq());
}

// Duality gap at the feasible z (reading in oracle/svm.py): fills gap fields.
nys_status svm_gap(nys_ctx ctx, const nys_svm_problem& P, const double* z, const SvmWs& ws,
                   nys_svm_info* I) {
  const int64_t n = P.H.n;
  NYS_TRY(svm_matvec(ctx, P.H, z, ws.w));
  hipLaunchKernelGGL(k_svm_gap, dim3(1), dim3(kPT), 0, ctx->stream, n, z, ws.w, P.b, P.C, 0, 0.0,
                     ws.scal + 16);
  double g[6];
  NYS_TRY(read_svm(ctx, ws.scal + 16, g, 6));
  double beta;
  if (g[3] > 0.0) {
    beta = g[2] / g[3];
  } else if (std::isfinite(g[4]) && std::isfinite(g[5])) {
    beta = 0.5 * (g[4] + g[5]);
  } else {
    beta = std::isfinite(g[4]) ? g[4] : (std::isfinite(g[5]) ? g[5] : 0.0);
  }
  hipLaunchKernelGGL(k_svm_gap, dim3(1), dim3(kPT), 0, ctx->stream, n, z, ws.w, P.b, P.C, 1,
                     beta, ws.scal + 16);
  double hinge;
  NYS_TRY(read_svm(ctx, ws.scal + 22, &hinge, 1));
  const double zHz = g[0];
  const double primal = 0.5 * zHz + P.C * hinge;
  const double dual = g[1] - 0.5 * zHz;
  I->primal = primal;
  I->dual = dual;
  I->gap = primal - dual;
  I->gap_rel = (primal - dual) / (1.0 + std::fabs(primal));
  I->bias = beta;
  return NYS_OK;
}

}  // namespace

}  // namespace nys

using namespace nys;

extern "C" {

nys_status nys_kernel_rbf(nys_ctx ctx, const float* X, int64_t n, int64_t p, int64_t ldx,
                          const double* b, double gamma, float* H, int64_t ldh) {
  if (ctx == nullptr || X == nullptr || H == nullptr || n < 1 || p < 1 || ldx < p || ldh < n ||
      !(gamma > 0.0) || n > ((int64_t)1 << 31) - 1 || p > ((int64_t)1 << 31) - 1)
    return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  hipStream_t st = ctx->stream;
  // G rows in blocks of at most 2^25 doubles (256 MB)
  int64_t blk = std::max<int64_t>(64, ((int64_t)1 << 25) / n / 64 * 64);
  blk = std::min(blk, n);
  const size_t gb = align_up(sizeof(double) * (size_t)(blk * n));
  NYS_TRY(ctx->gemm_ws.reserve(gb + align_up(sizeof(double) * (size_t)n)));
  double* G = ctx->gemm_ws.as<double>();
  double* sq = reinterpret_cast<double*>(static_cast<char*>(ctx->gemm_ws.ptr) + gb);
  hipLaunchKernelGGL(k_rownorm2, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, X, n, p, ldx,
                     sq);
  NYS_TRY_HIP(hipGetLastError());
  for (int64_t i0 = 0; i0 < n; i0 += blk) {
    const int64_t rows = std::min(blk, n - i0);
    // G = X[i0 : i0 + rows] X^T  (FP64 products and sums of the FP32 features)
    NYS_TRY(gemm64(st, (int)rows, (int)n, (int)p, X + i0 * ldx, true, ldx, 1, X, true, 1, ldx, G,
                   n, 1, 1.0, 0.0, nullptr, 0));
    hipLaunchKernelGGL(k_rbf_rows, dim3(blocks256(rows * n)), dim3(256), 0, st, G, rows, n, i0,
                       sq, b, gamma, H, ldh);
    NYS_TRY_HIP(hipGetLastError());
  }
  return NYS_OK;
}

nys_status svm_solve(nys_ctx ctx, const nys_svm_problem* P, const nys_svm_opts* O,
                     nys_admm_state* S, nys_svm_info* I) {
  if (ctx == nullptr || P == nullptr || O == nullptr || S == nullptr) return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(&P->H));
  const int64_t n = P->H.n;
  if (P->H.d != n || P->b == nullptr || !(P->C > 0.0) || !(O->rho > 0.0) || O->rank < 0 ||
      O->rank >= n || (O->rank > 0 && O->omega == nullptr && O->factor == nullptr))
    return NYS_ERR_INVALID;
  if (S->x == nullptr || S->z == nullptr || S->u == nullptr) return NYS_ERR_INVALID;
  if (O->factor != nullptr && (O->factor->d != n || !O->factor->sym)) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  hipStream_t st = ctx->stream;
  nys_svm_info info{};
  info.gap = info.gap_rel = info.primal = info.dual = info.true_res_max = -1.0;
  nys_factor F = O->factor;
  const bool own = (F == nullptr && O->rank > 0);
  if (own) NYS_TRY(nys_sketch_sym(ctx, &P->H, 0.0, O->omega, O->rank, NYS_F64, &F));
  info.rank = F ? F->r : 0;
  SvmWs ws;
  nys_status s = svm_workspace(ctx, n, &ws);
  ctx->hx_key = AtbKey{};
  const int max_iter = O->max_iter > 0 ? O->max_iter : 100;
  const int gap_every = O->gap_every > 0 ? O->gap_every : 10;
  const int tr_every = O->true_res_every > 0 ? O->true_res_every : 1;
  for (int it = 0; s == NYS_OK && it < max_iter; ++it) {
    hipLaunchKernelGGL(k_svm_rhs, dim3(blocks256(n)), dim3(256), 0, st, n, O->rho, S->z, S->u,
                       ws.rhs);
    const bool last = it + 1 == max_iter;
    nys_pcg_opts po = O->pcg;
    if (po.true_residual && !last && (S->k + 1) % tr_every != 0) po.true_residual = 0;
    nys_pcg_info pinfo{};
    // H is constant: H x of one solve carries to the next (tagged by k)
    nys_status ps = pcg_run(ctx, P->H, nullptr, 0.0, O->rho, F, ws.rhs, S->x, po, &pinfo, 0.0,
                            (int64_t)S->k, nullptr, nullptr, true);
    if (ps != NYS_OK && ps != NYS_ERR_MAXITER) {
      s = ps;
      break;
    }
    // entries of v held in registers when n <= 512 x 64, else read per step
    if (n <= kPT * 16)
      hipLaunchKernelGGL(k_svm_project<16>, dim3(1), dim3(kPT), 0, st, n, S->x, P->b, P->C, S->z,
                         S->u, ws.scal);
    else if (n <= kPT * 64)
      hipLaunchKernelGGL(k_svm_project<64>, dim3(1), dim3(kPT), 0, st, n, S->x, P->b, P->C,
                         S->z, S->u, ws.scal);
    else
      hipLaunchKernelGGL(k_svm_project<0>, dim3(1), dim3(kPT), 0, st, n, S->x, P->b, P->C,
                         S->z, S->u, ws.scal);
    S->k += 1;
    info.iters += 1;
    info.pcg_iters += pinfo.iters;
    info.pcg_max = std::max(info.pcg_max, pinfo.iters);
    if (info.status == NYS_OK) info.status = ps;   // sticky: first non-OK
    if (ps == NYS_ERR_MAXITER) info.maxiter_solves += 1;
    if (pinfo.true_res_norm >= 0.0)
      info.true_res_max = std::max(info.true_res_max, pinfo.rhs_norm > 0.0
                                                          ? pinfo.true_res_norm / pinfo.rhs_norm
                                                          : 0.0);
    const bool check = O->gap_tol > 0.0 && ((it + 1) % gap_every == 0);
    if (last || check) {
      double sc[kSvmNS];
      s = read_svm(ctx, ws.scal, sc, kSvmNS);
      if (s != NYS_OK) break;
      info.r_p = std::sqrt(sc[0]);
      info.r_d = O->rho * std::sqrt(sc[1]);
    }
    if (check) {
      s = svm_gap(ctx, *P, S->z, ws, &info);
      if (s != NYS_OK) break;
      if (info.gap_rel <= O->gap_tol) {
        info.converged = 1;
        break;
      }
    }
  }
  if (s == NYS_OK && !info.converged) s = svm_gap(ctx, *P, S->z, ws, &info);
  if (s != NYS_OK) info.status = s;
  if (own && F != nullptr) nys_factor_destroy(F);
  if (I) *I = info;
  return s;
}

}  // extern "C"
