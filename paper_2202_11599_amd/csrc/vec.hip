// d-vector kernels of the PCG loop (Algorithm Nystrom PCG) and of the
// preconditioner apply (eq. Nyspreconditioner).  Every reduction is written
// as per-workgroup partial sums that the next kernel adds in a fixed order, so
// results are bitwise reproducible.  Each workgroup that needs a scalar
// (alpha, beta, ||w||^2) recomputes it from the same partials in the same
// order, which makes the value identical across workgroups without a grid
// barrier.  Kernels of an iteration return at once when PcgDev::done is set,
// so the host can enqueue several iterations between convergence checks.
#include <algorithm>

#include "internal.h"

namespace nys {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// a[t] + a[t + step] + ... (indices below n) with four loads in flight: four
// running sums, combined in a fixed order
__device__ __forceinline__ double strided_sum(const double* __restrict__ a, int n, int t,
                                              int step) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = t;
  for (; i + 3 * step < n; i += 4 * step) {
    s0 += a[i];
    s1 += a[i + step];
    s2 += a[i + 2 * step];
    s3 += a[i + 3 * step];
  }
  for (; i < n; i += step) s0 += a[i];
  return (s0 + s1) + (s2 + s3);
}

// Sum of a[0..n) with a 256-thread block in a fixed order; every thread gets it.
__device__ double block_sum_array(const double* __restrict__ a, int n, double* sh4) {
  double s = strided_sum(a, n, threadIdx.x, 256);
  s = wave_sum(s);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = s;
  __syncthreads();
  return ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
}

// Sum of one value per thread over a 256-thread block; every thread gets it.
__device__ double block_sum_value(double v, double* sh4) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
}

// Block sums whose loads are issued early: pre_load puts a[t + 256 i]
// (i < 4, thread t) in registers for n <= kPreMax without waiting for them (an
// index past n reads a[n - 1], dropped by pre_sum); pre_sum adds them in
// ascending i and sums over the block.  Larger n is summed by block_sum_array.
constexpr int kPreMax = 1024;
__device__ __forceinline__ void pre_load(const double* __restrict__ a, int n, double v[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = 0.0;
  if (n > 0 && n <= kPreMax) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = (int)threadIdx.x + 256 * i;
      v[i] = a[e < n ? e : n - 1];
    }
  }
}
__device__ __forceinline__ double pre_sum(const double* __restrict__ a, int n, const double v[4],
                                          double* sh4) {
  if (n > kPreMax) return block_sum_array(a, n, sh4);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) s += ((int)threadIdx.x + 256 * i < n) ? v[i] : 0.0;
  return block_sum_value(s, sh4);
}

// c[0] + c[1024] + ... + c[(nsl - 1) * 1024] with eight loads in flight (an
// index past nsl reads the last slice and adds nothing); eight running sums
// combined in a fixed order
__device__ __forceinline__ double slice_sum(const double* __restrict__ c, int nsl) {
  double s[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) s[t] = 0.0;
  for (int h0 = 0; h0 < nsl; h0 += 8) {
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int h = h0 + t;
      v[t] = c[(int64_t)(h < nsl ? h : nsl - 1) * 1024];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) s[t] += (h0 + t < nsl) ? v[t] : 0.0;
  }
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// 256 threads: RJ lanes x (256 / RJ) slices of the workgroup partials, each
// lane summing VW adjacent columns; the slices are combined in a fixed order
// through LDS.
template <int RJ, int VW>
__global__ __launch_bounds__(256) void k_reduce_update(
    int op, const double* __restrict__ ypart, int G, int ldy, const double* __restrict__ qpart,
    int64_t d, double rho_eff, const double* __restrict__ p, double* __restrict__ x,
    double* __restrict__ w, const double* __restrict__ rhs, double* __restrict__ wy, int k,
    const double* __restrict__ pppart, int npp, double* __restrict__ wwpart,
    double* __restrict__ rrpart, PcgDev* __restrict__ st, int Gq, int pre) {
  constexpr int S = 256 / RJ;
  constexpr int CW = RJ * VW;   // columns per workgroup
  __shared__ double part[S][CW];
  __shared__ double sh4[4];
  const int tid = threadIdx.x;
  const int lane = tid % RJ;
  const int grp = tid / RJ;
  // thread tid < CW finishes column blockIdx.x * CW + tid; its entries and the
  // partials of the step's scalars are loaded before the partial sums, so the
  // round trips overlap
  const int64_t jf = (int64_t)blockIdx.x * CW + tid;
  const bool own = tid < CW && jf < d;
  double qv[4], pv4[4];
  pre_load(qpart, (op == 0 && !pre) ? Gq : 0, qv);
  pre_load(pppart, (op == 0 && !pre) ? npp : 0, pv4);
  const double wyk = (op == 0) ? wy[k & (kWyRing - 1)] : 0.0;
  if (op == 0 && st->done) return;
  double pj = 0.0, xj = 0.0, wj = 0.0, rj = 0.0;
  if (own) {
    if (p != nullptr) pj = p[jf];
    if (op == 0) {
      xj = x[jf];
      wj = w[jf];
    } else if (op == 1 || op == 2) {
      rj = rhs[jf];
    } else if (op == 4) {
      rj = rhs[jf];
      wj = w[jf];
    }
  }

  if constexpr (VW == 1) {
    // eight independent running sums (rows g, g+S, ..., g+7S, ...) keep eight
    // loads in flight per lane; combined in a fixed order
    const int64_t j = (int64_t)blockIdx.x * RJ + lane;
    double a[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) a[t] = 0.0;
    if (j < d) {
      int g = grp;
      for (; g + 7 * S < G; g += 8 * S) {
#pragma unroll
        for (int t = 0; t < 8; ++t) a[t] += ypart[(int64_t)(g + t * S) * ldy + j];
      }
      for (; g < G; g += S) a[0] += ypart[(int64_t)g * ldy + j];
    }
    part[grp][lane] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  } else {
    // two adjacent columns per 16-byte load (ldy even, ypart 16-byte aligned;
    // the column past an odd d lies inside the padded row and is dropped) and
    // sixteen rows per lane issued together: a row past G reads row G - 1 and
    // adds nothing.  Sixteen running sums, combined in a fixed order.
    static_assert(VW == 2, "two columns per lane");
    const int64_t j = (int64_t)blockIdx.x * CW + 2 * lane;
    double2 a[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) a[t] = make_double2(0.0, 0.0);
    if (j < d) {
      for (int g = grp; g < G; g += 16 * S) {
        double2 v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int gt = g + t * S;
          const int gc = gt < G ? gt : G - 1;
          v[t] = *reinterpret_cast<const double2*>(ypart + (int64_t)gc * ldy + j);
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const bool in = g + t * S < G;
          a[t].x += in ? v[t].x : 0.0;
          a[t].y += in ? v[t].y : 0.0;
        }
      }
    }
    double2 q[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      q[t].x = (a[4 * t].x + a[4 * t + 1].x) + (a[4 * t + 2].x + a[4 * t + 3].x);
      q[t].y = (a[4 * t].y + a[4 * t + 1].y) + (a[4 * t + 2].y + a[4 * t + 3].y);
    }
    part[grp][2 * lane] = (q[0].x + q[1].x) + (q[2].x + q[3].x);
    part[grp][2 * lane + 1] = (q[0].y + q[1].y) + (q[2].y + q[3].y);
  }

  double alpha = 0.0;
  if (op == 0) {
    // q = sum qpart, pp = sum pppart (fixed order, identical in every
    // workgroup), or the sum made once by k_pcg_scalar (pre)
    double pv;
    if (pre) {
      pv = st->pv;
    } else {
      const double qs = pre_sum(qpart, Gq, qv, sh4);
      __syncthreads();
      const double ps = pre_sum(pppart, npp, pv4, sh4);
      pv = qs + rho_eff * ps;
    }
    if (!(pv > 0.0)) {
      if (blockIdx.x == 0 && tid == 0) {
        st->flags |= (pv != pv) ? kFlagNonfinite : kFlagBreakdown;
        st->iters = k;
        st->done = 1;
      }
      return;
    }
    alpha = wyk / pv;
  }
  __syncthreads();

  const int64_t j = jf;
  double ww = 0.0, rr = 0.0;
  if (own) {
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) sum += part[i][tid];
    const double v = sum + rho_eff * pj;
    if (op == 0) {
      x[j] = xj + alpha * pj;
      const double wn = wj - alpha * v;
      w[j] = wn;
      ww = wn * wn;
    } else if (op == 1 || op == 2) {
      const double wn = rj - v;
      w[j] = wn;
      ww = wn * wn;
      rr = rj * rj;
      if (op == 2 && x != nullptr) x[j] = v;   // keep H_rho x for the next solve's w0
    } else if (op == 4) {   // H_rho x = rhs - w from the recursive residual
      x[j] = rj - wj;
    } else {  // op 3: plain reduction
      w[j] = v;
    }
  }
  if (op >= 3) return;
  __syncthreads();
  ww = block_sum_value(ww, sh4);
  __syncthreads();
  rr = block_sum_value(rr, sh4);
  if (tid == 0) {
    wwpart[blockIdx.x] = ww;
    if (rrpart != nullptr) rrpart[blockIdx.x] = rr;
  }
}

// mode 0: PCG iteration k (convergence test, then c = U^T w)
// mode 1: PCG init (threshold from ||rhs||, test, then c = U^T w)
// mode 2: standalone c = U^T w
// mode 3: record sum(wwpart) as the true residual, no dots
// c is left as dot_slices(d) partial sums over slices of d (cvec[s * 1024 +
// i], one slice per blockIdx.y), added in slice order by k_precond_update.
// pre: ||w||^2 was summed once by k_pcg_scalar into st->wwn.
template <typename UT>
__global__ __launch_bounds__(256) void k_precond_dot(
    const UT* __restrict__ U, int64_t d, int r, const double* __restrict__ w,
    double* __restrict__ cvec, PcgDev* __restrict__ st, const double* __restrict__ wwpart,
    int nww, const double* __restrict__ rrpart, int k, int mode, double tol_rel, double tol_abs,
    int pre) {
  __shared__ double sh4[4];
  const int tid = threadIdx.x;
  // the partials of the norms are loaded with the state, and this
  // workgroup's slice of U^T w is summed before the test, so their round
  // trips overlap
  double wv[4], rv[4];
  pre_load(wwpart, ((mode == 0 && !pre) || mode == 1 || mode == 3) ? nww : 0, wv);
  pre_load(rrpart, mode == 1 ? nww : 0, rv);
  if ((mode == 0 || mode == 1) && st->done) return;
  // partial c = U^T w over d-slice blockIdx.y: cpart[slice * 1024 + col]
  const int lane = tid & 63;
  const int col = blockIdx.x * 4 + (tid >> 6);
  double acc = 0.0;
  if (mode != 3 && col < r) {
    const int nsl = (int)gridDim.y;
    const int64_t chunk = ((d + nsl - 1) / nsl + 63) / 64 * 64;
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < d ? j0 + chunk : d;
    const UT* u = U + (int64_t)col * d;
    // eight running sums so that eight loads of U (and of w) are in flight
    // per lane; combined in a fixed order
    double a[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) a[t] = 0.0;
    int64_t j = j0 + lane;
    for (; j + 7 * 64 < j1; j += 8 * 64) {
#pragma unroll
      for (int t = 0; t < 8; ++t) a[t] = fma((double)u[j + 64 * t], w[j + 64 * t], a[t]);
    }
    // the (fewer than eight) remaining terms, their loads issued together: an
    // index past the slice reads its last entry and adds nothing
    if (j < j1) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int64_t jt = j + 64 * t;
        const int64_t jc = jt < j1 ? jt : j1 - 1;
        const double v = fma((double)u[jc], w[jc], a[t]);
        a[t] = jt < j1 ? v : a[t];
      }
    }
    acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    acc = wave_sum(acc);
  }
  if (mode == 0 || mode == 1) {
    const double ww = (pre && mode == 0) ? st->wwn : pre_sum(wwpart, nww, wv, sh4);
    double thr2;
    bool zero_rhs = false;
    if (mode == 1) {
      __syncthreads();
      const double rr = pre_sum(rrpart, nww, rv, sh4);
      thr2 = fmax(tol_abs * tol_abs, tol_rel * tol_rel * rr);
      zero_rhs = (rr == 0.0);
      if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) {
        st->rr = rr;
        st->thr2 = thr2;
      }
    } else {
      thr2 = st->thr2;
    }
    const bool bad = !(ww == ww) || (ww > 1.7e308);
    const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && tid == 0;
    if (lead) st->ww = ww;
    if (zero_rhs || bad || ww <= thr2) {
      if (lead) {
        if (bad) st->flags |= kFlagNonfinite;
        if (zero_rhs) st->flags |= kFlagZeroRhs;
        st->iters = (mode == 1) ? 0 : k + 1;
        st->done = 1;
      }
      return;
    }
  } else if (mode == 3) {
    const double ww = pre_sum(wwpart, nww, wv, sh4);
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) st->true_rr = ww;
    return;
  }
  if (col < r && lane == 0) cvec[(int64_t)blockIdx.y * 1024 + col] = acc;
}

// y = w + U (s o c), s_i = (lambda_s + rho)/(lambda_i + rho) - 1 ;
// w^T y = ||w||^2 + sum s_i c_i^2.
// mode 0: p = y + beta p (beta = (w^T y)/wy[k]), wy[k+1] = w^T y
// mode 1: p = y, wy[0] = w^T y
// mode 2: p (output) = y, standalone apply
template <typename UT, int NU, int VJ>
__global__ __launch_bounds__(256) void k_precond_update(
    const UT* __restrict__ U, int64_t d, int r, const double* __restrict__ lam, double lam_s,
    double rho, const double* __restrict__ cvec, const double* __restrict__ w,
    double* __restrict__ p, double* __restrict__ wy, int k, const double* __restrict__ wwpart,
    int nww, double* __restrict__ pppart, const PcgDev* __restrict__ st, int mode,
    PcgDev* __restrict__ host_slot, int seq, int nsl, int pre, const double* __restrict__ gpre) {
  // host_slot (pinned host memory, may be NULL): receives the state at the end
  // of the iteration, read by the host once the kernel has completed.
  // gpre (may be NULL): g and sum s c^2 already reduced by k_c_reduce
  // VJ entries of y per workgroup, VS slices of the rank index
  constexpr int VS = 256 / VJ;
  __shared__ double g[1024];
  __shared__ double ys[VS][VJ];
  __shared__ double sh4[4];
  const int tid = threadIdx.x;
  const int jl = tid % VJ, sl = tid / VJ;
  const int64_t j = (int64_t)blockIdx.x * VJ + jl;
  const UT* u = U + j;
  // loaded with the state, so the round trips overlap: the partials of
  // ||w||^2, this lane's entries of w and p, and wy[k]
  double wv[4];
  pre_load(wwpart, (mode != 2 && !(pre && mode == 0)) ? nww : 0, wv);
  double wj = 0.0, pold = 0.0;
  if (sl == 0 && j < d) {
    wj = w[j];
    if (mode == 0) pold = p[j];
  }
  const double wyk = (mode == 0) ? wy[k & (kWyRing - 1)] : 0.0;
  if (mode != 2 && st->done) {
    if (host_slot != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
      PcgDev h = *st;
      h.k = seq;              // sequence number the host waits for
      *host_slot = h;
    }
    return;
  }
  // the lane's first NU terms of U (rank i = sl + VS t; an index past r reads
  // row r - 1, dropped below), loaded with the slices of c
  UT u0[NU];
#pragma unroll
  for (int t = 0; t < NU; ++t) u0[t] = UT(0);
  if (j < d && r > 0) {
#pragma unroll
    for (int t = 0; t < NU; ++t) {
      const int it = sl + t * VS;
      u0[t] = u[(int64_t)(it < r ? it : r - 1) * d];
    }
  }
  double sc = 0.0;
  if (gpre != nullptr) {
    for (int i = tid; i < r; i += 256) g[i] = gpre[i];
  } else {
    for (int i = tid; i < r; i += 256) {
      const double ci = slice_sum(cvec + i, nsl);   // slices in a fixed order
      const double s = (lam_s + rho) / (lam[i] + rho) - 1.0;
      g[i] = s * ci;
      sc += s * ci * ci;
    }
  }
  double wy_new = 0.0;
  if (mode != 2) {
    const double ww = (pre && mode == 0) ? st->wwn : pre_sum(wwpart, nww, wv, sh4);
    __syncthreads();
    wy_new = ww + (gpre != nullptr ? gpre[1024] : block_sum_value(sc, sh4));
  } else {
    __syncthreads();
  }
  double part = 0.0;
  if (j < d && r > 0) {
    // NU running sums over the rank index (i = sl, sl + VS, ...), combined in
    // a fixed order; after the preloaded terms, NU loads of U are in flight
    // per lane, the last (partial) group issued together with clamped indices
    double a[NU];
#pragma unroll
    for (int t = 0; t < NU; ++t) {
      const int it = sl + t * VS;
      const int ic = it < r ? it : r - 1;
      a[t] = it < r ? (double)u0[t] * g[ic] : 0.0;
    }
    for (int i = sl + NU * VS; i < r; i += NU * VS) {
      UT v[NU];
#pragma unroll
      for (int t = 0; t < NU; ++t) {
        const int it = i + t * VS;
        v[t] = u[(int64_t)(it < r ? it : r - 1) * d];
      }
#pragma unroll
      for (int t = 0; t < NU; ++t) {
        const int it = i + t * VS;
        const int ic = it < r ? it : r - 1;
        const double f = fma((double)v[t], g[ic], a[t]);
        a[t] = it < r ? f : a[t];
      }
    }
    double q[NU / 4];
#pragma unroll
    for (int t = 0; t < NU / 4; ++t)
      q[t] = (a[4 * t] + a[4 * t + 1]) + (a[4 * t + 2] + a[4 * t + 3]);
    part = (q[0] + q[1]);
    if constexpr (NU == 16) part += (q[2] + q[3]);
  }
  ys[sl][jl] = part;
  __syncthreads();
  double pj = 0.0;
  if (sl == 0 && j < d) {
    double y = wj;
#pragma unroll
    for (int h = 0; h < VS; ++h) y += ys[h][jl];
    if (mode == 0) {
      const double beta = wy_new / wyk;
      pj = y + beta * pold;
    } else {
      pj = y;
    }
    p[j] = pj;
  }
  if (mode == 2) return;
  __syncthreads();
  const double pp = block_sum_value(pj * pj, sh4);
  if (tid == 0) {
    pppart[blockIdx.x] = pp;
    if (blockIdx.x == 0) {
      wy[mode == 1 ? 0 : (k + 1) & (kWyRing - 1)] = wy_new;
      if (host_slot != nullptr) {
        PcgDev h = *st;
        h.k = seq;            // sequence number the host waits for
        *host_slot = h;
      }
    }
  }
}

// Large d: c_i from its slice partials (in slice order), g_i = s_i c_i into
// gout[i] and sum_i s_i c_i^2 (wavefront sums, then the 16 in order) into
// gout[1024]; one workgroup per iteration instead of the slice sums being
// repeated by each of the d / 32 workgroups of k_precond_update.
__global__ __launch_bounds__(1024) void k_c_reduce(const double* __restrict__ cvec, int nsl,
                                                   int r, const double* __restrict__ lam,
                                                   double lam_s, double rho,
                                                   double* __restrict__ gout,
                                                   const PcgDev* __restrict__ st) {
  __shared__ double sh[16];
  if (st->done) return;
  const int i = threadIdx.x;
  double v = 0.0;
  if (i < r) {
    const double ci = slice_sum(cvec + i, nsl);
    const double s = (lam_s + rho) / (lam[i] + rho) - 1.0;
    gout[i] = s * ci;
    v = s * ci * ci;
  }
  v = wave_sum(v);
  if ((i & 63) == 0) sh[i >> 6] = v;
  __syncthreads();
  if (i == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sh[w];
    gout[1024] = t;
  }
}

// Clears the PCG state at the start of a solve (one lane per 4-byte word; a
// plain kernel launch costs the host less than a runtime fill)
__global__ void k_zero_state(PcgDev* __restrict__ st) {
  constexpr int kWords = (int)(sizeof(PcgDev) / sizeof(int));
  static_assert(sizeof(PcgDev) % sizeof(int) == 0 && kWords <= 64, "state words");
  if ((int)threadIdx.x < kWords) reinterpret_cast<int*>(st)[threadIdx.x] = 0;
}

// st->pv = sum(a) + rho_eff sum(b) (op 0), st->wwn = sum(a) (op 1): the
// PCG scalars summed once per iteration, in a fixed order, for large d
__global__ __launch_bounds__(1024) void k_pcg_scalar(int op, const double* __restrict__ a, int na,
                                                     const double* __restrict__ b, int nb,
                                                     double rho_eff, PcgDev* __restrict__ st) {
  __shared__ double sh[16];
  if (st->done) return;
  auto bsum = [&](const double* v, int cnt) {
    double s = strided_sum(v, cnt, threadIdx.x, 1024);
    s = wave_sum(s);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < 16; ++i) r += sh[i];
    __syncthreads();
    return r;
  };
  const double sa = bsum(a, na);
  if (op == 0) {
    const double sb = bsum(b, nb);
    if (threadIdx.x == 0) st->pv = sa + rho_eff * sb;
  } else {
    if (threadIdx.x == 0) st->wwn = sa;
  }
}

__global__ void k_note(const PcgDev* __restrict__ st, PcgDev* __restrict__ slot, int seq) {
  publish_state(&st->done, slot, seq);
}

__global__ __launch_bounds__(256) void k_dot(const double* __restrict__ a,
                                             const double* __restrict__ b, int64_t d,
                                             double* __restrict__ out) {
  __shared__ double sh4[4];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < d; j += 256) s = fma(a[j], b[j], s);
  s = block_sum_value(s, sh4);
  if (threadIdx.x == 0) *out = s;
}

// Decide between two starts; one block so the partials can be rewritten safely.
__global__ __launch_bounds__(256) void k_judge_decide(double* __restrict__ wwpart,
                                                      const double* __restrict__ wwpart2, int n,
                                                      PcgDev* __restrict__ st) {
  __shared__ double sh4[4];
  const double a = block_sum_array(wwpart, n, sh4);
  __syncthreads();
  const double b = block_sum_array(wwpart2, n, sh4);
  if (!(b < a)) return;
  for (int i = threadIdx.x; i < n; i += 256) wwpart[i] = wwpart2[i];
  if (threadIdx.x == 0) st->flags |= kFlagAltStart;
}

__global__ void k_judge_apply(double* __restrict__ x, const double* __restrict__ x_alt,
                              double* __restrict__ w, const double* __restrict__ w2, int64_t d,
                              const PcgDev* __restrict__ st) {
  if (!(st->flags & kFlagAltStart)) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < d) {
    x[j] = x_alt[j];
    w[j] = w2[j];
  }
}

// out_i = sum_j U[j, i] v_j: one wave per column, fixed order
__global__ __launch_bounds__(256) void k_ut_v(const double* __restrict__ U, int64_t d, int r,
                                              const double* __restrict__ v,
                                              double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= r) return;
  const double* u = U + (int64_t)col * d;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t j = lane;
  for (; j + 192 < d; j += 256) {
    a0 = fma(u[j], v[j], a0);
    a1 = fma(u[j + 64], v[j + 64], a1);
    a2 = fma(u[j + 128], v[j + 128], a2);
    a3 = fma(u[j + 192], v[j + 192], a3);
  }
  for (; j < d; j += 64) a0 = fma(u[j], v[j], a0);
  double acc = (a0 + a1) + (a2 + a3);
  acc = wave_sum(acc);
  if (lane == 0) out[col] = acc;
}

// out_j = sum_i U[j, i] c_i: one thread per row, columns read coalesced
__global__ __launch_bounds__(256) void k_u_c(const double* __restrict__ U, int64_t d, int r,
                                             const double* __restrict__ c,
                                             double* __restrict__ out) {
  __shared__ double cs[1024];
  for (int i = threadIdx.x; i < r; i += 256) cs[i] = c[i];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= d) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = 0;
  for (; i + 3 < r; i += 4) {
    a0 = fma(U[(int64_t)i * d + j], cs[i], a0);
    a1 = fma(U[(int64_t)(i + 1) * d + j], cs[i + 1], a1);
    a2 = fma(U[(int64_t)(i + 2) * d + j], cs[i + 2], a2);
    a3 = fma(U[(int64_t)(i + 3) * d + j], cs[i + 3], a3);
  }
  for (; i < r; ++i) a0 = fma(U[(int64_t)i * d + j], cs[i], a0);
  out[j] = (a0 + a1) + (a2 + a3);
}

// Argument check of a caller's n-vector: bit kCheckBad when an entry breaks
// the rule of `kind` (0 weights: v >= 0; 1 labels: v in {0, 1}), bit
// kCheckNonfinite when an entry is NaN or infinite.  One atomicOr per wave
// that found something.
__global__ __launch_bounds__(256) void k_check_vec(const double* __restrict__ v, int64_t n,
                                                   int kind, int* __restrict__ flags) {
  int bits = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const double x = v[i];
    if (!(fabs(x) <= 1.7976931348623157e308)) bits |= kCheckNonfinite;
    else if (kind == 0 ? !(x >= 0.0) : !(x == 0.0 || x == 1.0)) bits |= kCheckBad;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) bits |= __shfl_xor(bits, off, 64);
  if ((threadIdx.x & 63) == 0 && bits != 0) atomicOr(flags, bits);
}

}  // namespace

nys_status launch_check_vec(const double* v, int64_t n, int kind, int* flags,
                            hipStream_t stream) {
  if (n <= 0) return NYS_OK;
  const int64_t g = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_check_vec, dim3((unsigned)g), dim3(256), 0, stream, v, n, kind, flags);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_dot(const double* a, const double* b, int64_t d, double* out,
                      hipStream_t stream) {
  hipLaunchKernelGGL(k_dot, dim3(1), dim3(256), 0, stream, a, b, d, out);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_reduce_update(int op, const double* ypart, int G, int ldy, const double* qpart,
                                int64_t d, double rho_eff, const double* p, double* x, double* w,
                                const double* rhs, double* wy, int k, const double* pppart,
                                int npp, double* wwpart, double* rrpart, PcgDev* st,
                                hipStream_t stream, int Gq, bool pre, int rj) {
  if (rj == 0) rj = red_block(G);
  // the wide form reads column pairs: rows of even length, 16-byte aligned
  const bool wide = (ldy % 2 == 0) && (reinterpret_cast<uintptr_t>(ypart) % 16 == 0);
  if (rj == 256)
    hipLaunchKernelGGL((k_reduce_update<256, 1>), dim3(nblk(d, 256)), dim3(256), 0, stream, op,
                       ypart, G, ldy, qpart, d, rho_eff, p, x, w, rhs, wy, k, pppart, npp, wwpart,
                       rrpart, st, Gq < 0 ? G : Gq, pre ? 1 : 0);
  else if (rj == kRedBlock && wide)
    hipLaunchKernelGGL((k_reduce_update<kRedBlock / 2, 2>), dim3(nblk(d, kRedBlock)), dim3(256),
                       0, stream, op, ypart, G, ldy, qpart, d, rho_eff, p, x, w, rhs, wy, k,
                       pppart, npp, wwpart, rrpart, st, Gq < 0 ? G : Gq, pre ? 1 : 0);
  else if (rj == kRedBlock)
    hipLaunchKernelGGL((k_reduce_update<kRedBlock, 1>), dim3(nblk(d, kRedBlock)), dim3(256), 0,
                       stream, op, ypart, G, ldy, qpart, d, rho_eff, p, x, w, rhs, wy, k, pppart,
                       npp, wwpart, rrpart, st, Gq < 0 ? G : Gq, pre ? 1 : 0);
  else
    return NYS_ERR_INVALID;
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_zero_state(PcgDev* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, stream, st);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_note(const PcgDev* st, PcgDev* slot, int seq, hipStream_t stream) {
  hipLaunchKernelGGL(k_note, dim3(1), dim3(64), 0, stream, st, slot, seq);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_pcg_scalar(int op, const double* a, int na, const double* b, int nb,
                             double rho_eff, PcgDev* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_pcg_scalar, dim3(1), dim3(1024), 0, stream, op, a, na, b, nb, rho_eff, st);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_precond_dot(const void* U, bool u32, int64_t d, int r, const double* w,
                              double* cvec, PcgDev* st, const double* wwpart, int nww,
                              const double* rrpart, int k, int mode, double tol_rel,
                              double tol_abs, hipStream_t stream, bool pre) {
  const unsigned gx = r > 0 ? (unsigned)((r + 3) / 4) : 1u;
  const dim3 grid(gx, (mode == 0 || mode == 1 || mode == 2) ? dot_slices(d) : 1);
  if (u32)
    hipLaunchKernelGGL(k_precond_dot<float>, grid, dim3(256), 0, stream,
                       static_cast<const float*>(U), d, r, w, cvec, st, wwpart, nww, rrpart, k,
                       mode, tol_rel, tol_abs, pre ? 1 : 0);
  else
    hipLaunchKernelGGL(k_precond_dot<double>, grid, dim3(256), 0, stream,
                       static_cast<const double*>(U), d, r, w, cvec, st, wwpart, nww, rrpart, k,
                       mode, tol_rel, tol_abs, pre ? 1 : 0);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_c_reduce(const double* cvec, int64_t d, int r, const double* lam, double lam_s,
                           double rho, double* gout, const PcgDev* st, hipStream_t stream) {
  if (r < 0 || r > 1024) return NYS_ERR_INVALID;
  hipLaunchKernelGGL(k_c_reduce, dim3(1), dim3(1024), 0, stream, cvec, dot_slices(d), r, lam, lam_s,
                     rho, gout, st);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_precond_update(const void* U, bool u32, int64_t d, int r, const double* lam,
                                 double lam_s, double rho, const double* cvec, const double* w,
                                 double* p, double* wy, int k, const double* wwpart, int nww,
                                 double* pppart, const PcgDev* st, int mode, hipStream_t stream,
                                 PcgDev* host_slot, int seq, bool pre, const double* gpre) {
  if (r > 1024) return NYS_ERR_INVALID;
  const int vj = vec_block(d);
  const int grid = nblk(d, vj);
  const int nsl = dot_slices(d);
  // eight rank terms per lane in flight up to rank 64 (every term in one
  // group); sixteen up to rank 256, where the pass is latency bound and the
  // lane's terms fit two groups; eight above, where U streams from HBM and
  // the clamped tail of a wider group only adds loads
  const int vs = 256 / vj;
  const bool wide = r > 8 * vs && r <= 32 * vs;
  auto go = [&](auto kern, const auto* u) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, stream, u, d, r, lam, lam_s, rho, cvec, w,
                       p, wy, k, wwpart, nww, pppart, st, mode, host_slot, seq, nsl, pre ? 1 : 0,
                       gpre);
  };
  if (u32) {
    const float* u = static_cast<const float*>(U);
    if (vj == kVecBlock) {
      if (wide) go(k_precond_update<float, 16, kVecBlock>, u);
      else go(k_precond_update<float, 8, kVecBlock>, u);
    } else {
      if (wide) go(k_precond_update<float, 16, kVecBlockWide>, u);
      else go(k_precond_update<float, 8, kVecBlockWide>, u);
    }
  } else {
    const double* u = static_cast<const double*>(U);
    if (vj == kVecBlock) {
      if (wide) go(k_precond_update<double, 16, kVecBlock>, u);
      else go(k_precond_update<double, 8, kVecBlock>, u);
    } else {
      if (wide) go(k_precond_update<double, 16, kVecBlockWide>, u);
      else go(k_precond_update<double, 8, kVecBlockWide>, u);
    }
  }
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

}  // namespace nys

namespace nys {

nys_status launch_judge(double* wwpart, const double* wwpart2, int nred, double* x,
                        const double* x_alt, double* w, const double* w2, int64_t d, PcgDev* st,
                        hipStream_t stream) {
  hipLaunchKernelGGL(k_judge_decide, dim3(1), dim3(256), 0, stream, wwpart, wwpart2, nred, st);
  hipLaunchKernelGGL(k_judge_apply, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, stream, x,
                     x_alt, w, w2, d, st);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_ut_v(const double* U, int64_t d, int r, const double* v, double* out,
                       hipStream_t stream) {
  if (r < 1 || r > 1024) return NYS_ERR_INVALID;
  hipLaunchKernelGGL(k_ut_v, dim3((unsigned)((r + 3) / 4)), dim3(256), 0, stream, U, d, r, v, out);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_u_c(const double* U, int64_t d, int r, const double* c, double* out,
                      hipStream_t stream) {
  if (r < 1 || r > 1024) return NYS_ERR_INVALID;
  hipLaunchKernelGGL(k_u_c, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, stream, U, d, r, c,
                     out);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

}  // namespace nys
