// Fused Gram matvec: one streaming pass over A computes, per workgroup row
// range,
//     t_i = A_i p            (FP64 products of the stored A, FP64 sums)
//     s_i = f_mode(t_i)      (D_i t_i, t_i - b_i, logistic weights ...)
//     y_g = sum_i s_i A_i    (FP64)
// so H p = A^T D A p costs one read of A instead of two.  Partial sums y_g and
// q_g are written per workgroup and reduced in a fixed order by the vector
// kernels (deterministic, no float atomics).
//
// Layout: A row-major; a workgroup of WAVES wavefronts covers a full row, each
// lane owning CPL 16-byte chunks (4 floats or 2 doubles) at chunk index
// lane + m * 64 * WAVES, so every load instruction of a wavefront reads 1 KiB
// of one row contiguously.  Rows are streamed in groups of R; the R row dots
// are reduced across the wavefront with butterfly shuffles and across
// wavefronts through LDS (one barrier per group, double-buffered).  The group
// stays in registers for the A^T pass.
#include "internal.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>

namespace nys {
namespace {

// rows streamed per group (one LDS barrier per group)
constexpr int rows_for(int cpl) { return cpl >= 4 ? 4 : 8; }

template <typename T> struct Chunk;
template <> struct Chunk<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  static constexpr int N = 4;
};
template <> struct Chunk<double> {
  typedef double V __attribute__((ext_vector_type(2)));
  static constexpr int N = 2;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double sigm(double t) {
  const double e = exp(-fabs(t));
  return t >= 0.0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}


template <typename T, int WAVES, int CPL, int R, bool ALIGNED>
__global__ __launch_bounds__(WAVES * 64, (WAVES >= 4 ? 2 : 1)) void k_gram(
    const T* __restrict__ A, int64_t n, int d, int64_t ld, int64_t rows_per_wg, int mode,
    const double* __restrict__ p, const double* __restrict__ aux, double* __restrict__ auxout,
    double* __restrict__ ypart, int ldy, double* __restrict__ qpart,
    const int* __restrict__ done) {
  constexpr int NT = WAVES * 64;
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
  if (done != nullptr && *done) return;

  __shared__ double red[2][R][WAVES];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = (r0 + rows_per_wg < n) ? r0 + rows_per_wg : n;
  const bool tonly = (mode == kModeTOnly);

  double pr[CPL][VN], yr[CPL][VN];
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    const int c0 = (tid + m * NT) * VN;
#pragma unroll
    for (int v = 0; v < VN; ++v) {
      pr[m][v] = (!tonly && c0 + v < d) ? p[c0 + v] : 0.0;
      yr[m][v] = 0.0;
    }
  }
  double q = 0.0;
  int buf = 0;

  for (int64_t row = r0; row < r1; row += R) {
    V a[R][CPL];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t rr = row + i;
      const bool ok = rr < r1;
      const T* arow = A + rr * ld;
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        const int c0 = (tid + m * NT) * VN;
        V val = (V)(T)0;
        if (ok && c0 < d) {
          if (ALIGNED && c0 + VN <= d) {
            val = __builtin_nontemporal_load(reinterpret_cast<const V*>(arow + c0));
          } else {
#pragma unroll
            for (int v = 0; v < VN; ++v) val[v] = (c0 + v < d) ? arow[c0 + v] : (T)0;
          }
        }
        a[i][m] = val;
      }
    }

    double t[R];
    if (!tonly) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < CPL; ++m)
#pragma unroll
          for (int v = 0; v < VN; ++v) acc = fma((double)a[i][m][v], pr[m][v], acc);
        t[i] = wave_sum(acc);
      }
      // The FP64 copies made for the dot products die here: the A^T pass
      // converts the FP32 row again instead of keeping twice the registers
      // live across the barrier.
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int m = 0; m < CPL; ++m) asm volatile("" : "+v"(a[i][m]));
      if (WAVES > 1) {
        if (lane == 0) {
#pragma unroll
          for (int i = 0; i < R; ++i) red[buf][i][wv] = t[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < R; ++i) {
          double s = 0.0;
#pragma unroll
          for (int w = 0; w < WAVES; ++w) s += red[buf][i][w];
          t[i] = s;
        }
        buf ^= 1;
      }
    }

#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t rr = row + i;
      double s = 0.0;
      if (rr < r1) {
        const double ti = tonly ? 0.0 : t[i];
        switch (mode) {
          case kModeHess: {
            const double dv = aux ? aux[rr] : 1.0;
            s = dv * ti;
            q = fma(s, ti, q);
          } break;
          case kModeLsGrad: {
            s = ti - aux[rr];
            q = fma(s, s, q);
          } break;
          case kModeLogit: {
            const double sg = sigm(ti);
            const double w = sg * sigm(-ti);
            const double bi = aux[rr];
            s = w * ti + bi - sg;
            if (auxout != nullptr && tid == 0) auxout[rr] = w;
            q += log1p(exp(-fabs(ti))) + fmax(ti, 0.0) - bi * ti;
          } break;
          case kModeLogGrad: {
            const double bi = aux[rr];
            s = sigm(ti) - bi;
            q += log1p(exp(-fabs(ti))) + fmax(ti, 0.0) - bi * ti;
          } break;
          default:  // kModeTOnly
            s = aux[rr];
            break;
        }
      }
#pragma unroll
      for (int m = 0; m < CPL; ++m)
#pragma unroll
        for (int v = 0; v < VN; ++v) yr[m][v] = fma(s, (double)a[i][m][v], yr[m][v]);
    }
  }

  double* yp = ypart + (int64_t)blockIdx.x * ldy;
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    const int c0 = (tid + m * NT) * VN;
#pragma unroll
    for (int v = 0; v < VN; ++v)
      if (c0 + v < d) yp[c0 + v] = yr[m][v];
  }
  if (tid == 0) qpart[blockIdx.x] = q;
}

template <typename T, int WAVES, int CPL>
nys_status launch_t(const nys_dense& A, const GramPlan& pl, int mode, const double* p,
                    const double* aux, double* auxout, double* ypart, double* qpart,
                    const int* done, hipStream_t st) {
  const T* a = static_cast<const T*>(A.data);
  if (pl.aligned)
    hipLaunchKernelGGL((k_gram<T, WAVES, CPL, rows_for(CPL), true>), dim3(pl.grid), dim3(WAVES * 64), 0, st, a,
                       A.n, (int)A.d, A.ld, pl.rows_per_wg, mode, p, aux, auxout, ypart, pl.ldy,
                       qpart, done);
  else
    hipLaunchKernelGGL((k_gram<T, WAVES, CPL, rows_for(CPL), false>), dim3(pl.grid), dim3(WAVES * 64), 0, st, a,
                       A.n, (int)A.d, A.ld, pl.rows_per_wg, mode, p, aux, auxout, ypart, pl.ldy,
                       qpart, done);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

template <typename T>
nys_status launch_dt(const nys_dense& A, const GramPlan& pl, int mode, const double* p,
                     const double* aux, double* auxout, double* ypart, double* qpart,
                     const int* done, hipStream_t st) {
#define NYS_CASE(W, C)                                                                      \
  if (pl.waves == W && pl.cpl == C)                                                         \
    return launch_t<T, W, C>(A, pl, mode, p, aux, auxout, ypart, qpart, done, st);
  NYS_CASE(1, 2) NYS_CASE(1, 4) NYS_CASE(2, 2) NYS_CASE(2, 4)
  NYS_CASE(4, 2) NYS_CASE(4, 4) NYS_CASE(8, 2) NYS_CASE(8, 4)
#undef NYS_CASE
  return NYS_ERR_INVALID;
}

}  // namespace

GramPlan make_gram_plan(const nys_dense& A, int num_cu) {
  GramPlan pl;
  const int vn = A.dtype == NYS_F64 ? 2 : 4;
  const int64_t d = A.d;
  // smallest (waves, cpl) covering d, preferring 2 chunks per lane
  static const int cand[][2] = {{1, 2}, {2, 2}, {4, 2}, {8, 2}, {8, 4}};
  pl.waves = 8;
  pl.cpl = 4;
  for (auto& c : cand) {
    if ((int64_t)c[0] * 64 * c[1] * vn >= d) {
      pl.waves = c[0];
      pl.cpl = c[1];
      break;
    }
  }
  // workgroups resident per CU at 2 waves per SIMD (4 SIMDs)
  int per_cu = std::max(1, 8 / pl.waves);
  // tuning override "waves,cpl,wg_per_cu" (sweeps of launch shapes)
  if (const char* e = getenv("NYSADMM_GRAM_PLAN")) {
    int w = 0, c = 0, g = 0;
    if (sscanf(e, "%d,%d,%d", &w, &c, &g) == 3 && (int64_t)w * 64 * c * vn >= d &&
        (w == 1 || w == 2 || w == 4 || w == 8) && (c == 2 || c == 4) && g >= 1) {
      pl.waves = w;
      pl.cpl = c;
      per_cu = g;
    }
  }
  const int R = rows_for(pl.cpl);
  const int esize = A.dtype == NYS_F64 ? 8 : 4;
  pl.aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
  pl.ldy = (int)((d + 63) / 64 * 64);
  if (A.n <= 0) {
    pl.grid = 0;
    pl.rows_per_wg = 0;
    return pl;
  }
  // one full round of resident workgroups, each streaming a contiguous row range
  int64_t groups = (A.n + R - 1) / R;
  int64_t g = std::min<int64_t>((int64_t)per_cu * num_cu, std::max<int64_t>(1, groups / 2));
  pl.rows_per_wg = ((A.n + g - 1) / g + R - 1) / R * R;
  pl.grid = (int)((A.n + pl.rows_per_wg - 1) / pl.rows_per_wg);
  return pl;
}

nys_status launch_gram(const nys_dense& A, const GramPlan& pl, int mode, const double* p,
                       const double* aux, double* auxout, double* ypart, double* qpart,
                       const int* done, hipStream_t st) {
  const int vn = A.dtype == NYS_F64 ? 2 : 4;
  if ((int64_t)pl.waves * 64 * pl.cpl * vn < A.d) return NYS_ERR_INVALID;
  if (A.n == 0 || pl.grid == 0) return NYS_OK;
  if (A.dtype == NYS_F64)
    return launch_dt<double>(A, pl, mode, p, aux, auxout, ypart, qpart, done, st);
  if (A.dtype == NYS_F32)
    return launch_dt<float>(A, pl, mode, p, aux, auxout, ypart, qpart, done, st);
  return NYS_ERR_INVALID;
}

}  // namespace nys
