// Matvec pair for wide dense A (d above the widest single-workgroup row,
// 8192 FP32 / 4096 FP64 columns): the shapes of the paper's random-feature
// data (Section 5: 13000 x 27648, 60000 x 60000, ...).
//
// The fused pass keeps one row in the registers of one workgroup between its
// dot product and its A^T update; a row of d = 27648 floats would need more
// registers than a CU has next to the FP64 accumulators of y.  So the pair is
// split at the row dot, column block by column block:
//   1. t^(s)_i = A_i[block s] . p[block s]    (one workgroup per row range and
//      column block; FP64 products and sums, as the fused pass)
//   2. t_i = sum_s t^(s)_i (blocks in order), s_i = f_mode(t_i), q partials
//   3. y^(g)[block s] = sum_{i in rows of g} s_i A_i[block s]
// A is read twice per pair (the unfused cost of Table t-ComplexityComparison's
// T_mv); every sum has a fixed order, so results are bitwise reproducible.
// Steps 2-3 return at once when the PCG state says done, and step 1 publishes
// that state to the host's pinned slot like the fused kernel does.
#include <hip/hip_ext.h>

#include <algorithm>

#include "internal.h"
#include "gram_device.h"

namespace nys {
namespace {

using namespace gram;

constexpr int kWW = 4;   // waves per workgroup
constexpr int kWC = 4;   // 16-byte chunks per lane
constexpr int kWR = 2;   // rows per pipelined group

template <typename T, bool ALIGNED>
__global__ __launch_bounds__(kWW * 64, 2) void k_wide_rowdot(
    const T* __restrict__ A, int64_t n, int64_t ncols, int64_t ld, int slice_cols,
    int64_t rows_per_wg, const double* __restrict__ p, double* __restrict__ tpart, int64_t ldt,
    const int* __restrict__ done, PcgDev* __restrict__ note, int note_seq) {
  constexpr int NT = kWW * 64;
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
  publish_state(done, note, note_seq);
  if (done != nullptr && *done) return;
  __shared__ double red[2][kWR][kWW];
  const int tid = threadIdx.x;
  const int64_t c0s = (int64_t)blockIdx.y * slice_cols;
  const int d = (int)((ncols - c0s < slice_cols) ? ncols - c0s : slice_cols);
  const T* As = A + c0s;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = (r0 + rows_per_wg < n) ? r0 + rows_per_wg : n;
  double pr[kWC][VN];
#pragma unroll
  for (int m = 0; m < kWC; ++m) {
    const int c0 = col0<T, kWC, ALIGNED, NT>(tid, m);
#pragma unroll
    for (int v = 0; v < VN; ++v) pr[m][v] = (c0 + v < d) ? p[c0s + c0 + v] : 0.0;
  }
  double* out = tpart + (int64_t)blockIdx.y * ldt;
  double q = 0.0;   // no per-row weight here: stays 0
  int buf = 0;
  V a0[kWR][kWC], a1[kWR][kWC];
  T e0[kWR][Extra<T>::N], e1[kWR][Extra<T>::N];
  double v0[kWR], v1[kWR];
  load_group<T, kWC, kWR, ALIGNED, NT>(a0, e0, v0, As, nullptr, r0, r1, d, ld, tid);
  for (int64_t row = r0; row < r1; row += 2 * kWR) {
    load_group<T, kWC, kWR, ALIGNED, NT>(a1, e1, v1, As, nullptr, row + kWR, r1, d, ld, tid);
    realign_group<T, kWC, kWR, ALIGNED, NT>(a0, e0, As, row, d, ld, tid);
    rowdot_group<T, kWW, kWC, kWR>(a0, v0, row, r1, pr, q, out, red, buf, tid);
    if (row + kWR >= r1) break;
    load_group<T, kWC, kWR, ALIGNED, NT>(a0, e0, v0, As, nullptr, row + 2 * kWR, r1, d, ld, tid);
    realign_group<T, kWC, kWR, ALIGNED, NT>(a1, e1, As, row + kWR, d, ld, tid);
    rowdot_group<T, kWW, kWC, kWR>(a1, v1, row + kWR, r1, pr, q, out, red, buf, tid);
  }
}

// t_i = sum over column blocks (in block order), then the epilogue of the
// mode (as the fused kernel's): s_i to svec, per-workgroup sums of q.
__global__ __launch_bounds__(256) void k_wide_mode(int64_t n, int slices,
                                                   const double* __restrict__ tpart, int64_t ldt,
                                                   int mode, const double* __restrict__ aux,
                                                   double* __restrict__ auxout,
                                                   double* __restrict__ svec,
                                                   double* __restrict__ qpart,
                                                   const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double q = 0.0;
  if (i < n) {
    double t = 0.0;
    if (mode != kModeTOnly)
      for (int s = 0; s < slices; ++s) t += tpart[(int64_t)s * ldt + i];
    double s = 0.0;
    if (mode == kModeHess) {
      s = (aux != nullptr ? aux[i] : 1.0) * t;
      q = s * t;
    } else if (mode == kModeLsGrad) {
      s = t - aux[i];
      q = s * s;
    } else if (mode == kModeLogit || mode == kModeLogGrad) {
      const double b = aux[i];
      const double sg = sigm(t);
      q = log1p(exp(-fabs(t))) + fmax(t, 0.0) - b * t;
      if (mode == kModeLogit) {
        const double w = sg * sigm(-t);
        s = w * t + b - sg;
        if (auxout != nullptr) auxout[i] = w;
      } else {
        s = sg - b;
      }
    } else {   // kModeTOnly
      s = aux[i];
    }
    svec[i] = s;
  }
  q = wave_sum(q);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) qpart[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

template <typename T, bool ALIGNED>
__global__ __launch_bounds__(kWW * 64, 2) void k_wide_colsum(
    const T* __restrict__ A, int64_t n, int64_t ncols, int64_t ld, int slice_cols,
    int64_t rows_per_wg, const double* __restrict__ svec, double* __restrict__ ypart, int ldy,
    const int* __restrict__ done) {
  constexpr int NT = kWW * 64;
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
  if (done != nullptr && *done) return;
  __shared__ double red[2][kWR][kWW];
  const int tid = threadIdx.x;
  const int64_t c0s = (int64_t)blockIdx.y * slice_cols;
  const int d = (int)((ncols - c0s < slice_cols) ? ncols - c0s : slice_cols);
  const T* As = A + c0s;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = (r0 + rows_per_wg < n) ? r0 + rows_per_wg : n;
  double pr[kWC][VN], yr[kWC][VN];
#pragma unroll
  for (int m = 0; m < kWC; ++m)
#pragma unroll
    for (int v = 0; v < VN; ++v) {
      pr[m][v] = 0.0;
      yr[m][v] = 0.0;
    }
  double q = 0.0;
  int buf = 0;
  V a0[kWR][kWC], a1[kWR][kWC];
  T e0[kWR][Extra<T>::N], e1[kWR][Extra<T>::N];
  double v0[kWR], v1[kWR];
  // the rows' s_i travel with the rows (load_group's per-row input)
  load_group<T, kWC, kWR, ALIGNED, NT>(a0, e0, v0, As, svec, r0, r1, d, ld, tid);
  for (int64_t row = r0; row < r1; row += 2 * kWR) {
    load_group<T, kWC, kWR, ALIGNED, NT>(a1, e1, v1, As, svec, row + kWR, r1, d, ld, tid);
    realign_group<T, kWC, kWR, ALIGNED, NT>(a0, e0, As, row, d, ld, tid);
    process_group<T, kWW, kWC, kWR>(a0, v0, row, r1, kModeTOnly, pr, yr, q, svec, nullptr, red,
                                    buf, tid);
    if (row + kWR >= r1) break;
    load_group<T, kWC, kWR, ALIGNED, NT>(a0, e0, v0, As, svec, row + 2 * kWR, r1, d, ld, tid);
    realign_group<T, kWC, kWR, ALIGNED, NT>(a1, e1, As, row + kWR, d, ld, tid);
    process_group<T, kWW, kWC, kWR>(a1, v1, row + kWR, r1, kModeTOnly, pr, yr, q, svec, nullptr,
                                    red, buf, tid);
  }
  double* yp = ypart + (int64_t)blockIdx.x * ldy + c0s;
#pragma unroll
  for (int m = 0; m < kWC; ++m) {
    const int c0 = col0<T, kWC, ALIGNED, NT>(tid, m);
#pragma unroll
    for (int v = 0; v < VN; ++v)
      if (c0 + v < d) yp[c0 + v] = yr[m][v];
  }
}

template <typename T, bool AL>
nys_status launch_wide_t(const nys_dense& A, const GramPlan& pl, int mode, const double* p,
                         const double* aux, double* auxout, double* ypart, double* qpart,
                         const int* done, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                         PcgDev* note, int note_seq) {
  const T* a = static_cast<const T*>(A.data);
  double* tpart = wide_tmp(pl, qpart);
  double* svec = tpart + (int64_t)pl.slices * pl.ldt;
  const dim3 grid(pl.grid, pl.slices);
  if (mode != kModeTOnly) {
    if (ev0 != nullptr)
      hipExtLaunchKernelGGL((k_wide_rowdot<T, AL>), grid, dim3(kWW * 64), 0, st, ev0, nullptr, 0, a,
                            A.n, A.d, A.ld, pl.slice_cols, pl.rows_per_wg, p, tpart, pl.ldt, done,
                            note, note_seq);
    else
      hipLaunchKernelGGL((k_wide_rowdot<T, AL>), grid, dim3(kWW * 64), 0, st, a, A.n, A.d, A.ld,
                         pl.slice_cols, pl.rows_per_wg, p, tpart, pl.ldt, done, note, note_seq);
  } else if (note != nullptr) {
    NYS_TRY(launch_note(reinterpret_cast<const PcgDev*>(done), note, note_seq, st));
  }
  if (ev0 != nullptr && mode == kModeTOnly)
    hipExtLaunchKernelGGL(k_wide_mode, dim3(pl.mgrid), dim3(256), 0, st, ev0, nullptr, 0, A.n,
                          pl.slices, tpart, pl.ldt, mode, aux, auxout, svec, qpart, done);
  else
    hipLaunchKernelGGL(k_wide_mode, dim3(pl.mgrid), dim3(256), 0, st, A.n, pl.slices, tpart,
                       pl.ldt, mode, aux, auxout, svec, qpart, done);
  if (ev1 != nullptr)
    hipExtLaunchKernelGGL((k_wide_colsum<T, AL>), grid, dim3(kWW * 64), 0, st, nullptr, ev1, 0, a,
                          A.n, A.d, A.ld, pl.slice_cols, pl.rows_per_wg, svec, ypart, pl.ldy,
                          done);
  else
    hipLaunchKernelGGL((k_wide_colsum<T, AL>), grid, dim3(kWW * 64), 0, st, a, A.n, A.d, A.ld,
                       pl.slice_cols, pl.rows_per_wg, svec, ypart, pl.ldy, done);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

}  // namespace

double* wide_tmp(const GramPlan& pl, double* qpart) {
  return qpart + align_up(sizeof(double) * (size_t)std::max(pl.nq(), 1)) / sizeof(double);
}

GramPlan make_wide_plan(const nys_dense& A, int num_cu) {
  GramPlan pl;
  pl.wide = true;
  pl.waves = kWW;
  pl.cpl = kWC;
  pl.rows = kWR;
  const int vn = A.dtype == NYS_F64 ? 2 : 4;
  pl.slice_cols = kWW * 64 * kWC * vn;
  pl.slices = (int)std::max<int64_t>(1, (A.d + pl.slice_cols - 1) / pl.slice_cols);
  const int esize = A.dtype == NYS_F64 ? 8 : 4;
  pl.aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
  pl.ldy = (int)((A.d + 63) / 64 * 64);
  pl.ldt = (std::max<int64_t>(A.n, 1) + 63) / 64 * 64;
  pl.mgrid = (int)std::max<int64_t>(1, (A.n + 255) / 256);
  pl.per_cu = 2;
  if (A.n <= 0) {
    pl.grid = 0;
    pl.rows_per_wg = 0;
    return pl;
  }
  // row ranges x column blocks: about two workgroups per CU in each pass
  const int64_t groups = (A.n + pl.rows - 1) / pl.rows;
  const int64_t want = std::max<int64_t>(1, ((int64_t)pl.per_cu * num_cu + pl.slices - 1) /
                                                pl.slices);
  const int64_t g = std::min<int64_t>(want, std::max<int64_t>(1, groups / 2));
  pl.rows_per_wg = ((A.n + g - 1) / g + pl.rows - 1) / pl.rows * pl.rows;
  pl.grid = (int)((A.n + pl.rows_per_wg - 1) / pl.rows_per_wg);
  return pl;
}

nys_status launch_wide(const nys_dense& A, const GramPlan& pl, int mode, const double* p,
                       const double* aux, double* auxout, double* ypart, double* qpart,
                       const int* done, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                       PcgDev* note, int note_seq) {
  if (!pl.wide || pl.waves != kWW || pl.cpl != kWC || pl.rows != kWR) return NYS_ERR_INVALID;
  if (A.n == 0 || pl.grid == 0) {
    if (note != nullptr)
      NYS_TRY(launch_note(reinterpret_cast<const PcgDev*>(done), note, note_seq, st));
    return NYS_OK;
  }
  if (A.dtype == NYS_F32)
    return pl.aligned ? launch_wide_t<float, true>(A, pl, mode, p, aux, auxout, ypart, qpart,
                                                   done, st, ev0, ev1, note, note_seq)
                      : launch_wide_t<float, false>(A, pl, mode, p, aux, auxout, ypart, qpart,
                                                    done, st, ev0, ev1, note, note_seq);
  if (A.dtype == NYS_F64)
    return pl.aligned ? launch_wide_t<double, true>(A, pl, mode, p, aux, auxout, ypart, qpart,
                                                    done, st, ev0, ev1, note, note_seq)
                      : launch_wide_t<double, false>(A, pl, mode, p, aux, auxout, ypart, qpart,
                                                     done, st, ev0, ev1, note, note_seq);
  return NYS_ERR_INVALID;
}

}  // namespace nys
