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
#include <hip/hip_ext.h>

#include "gram_device.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>

namespace nys {
namespace {

using namespace gram;

// Rows are streamed in groups of R with two register buffers: the loads of
// the next group are issued before the current group's cross-wave barrier, so
// every workgroup keeps reads in flight while it reduces and updates.
template <typename T, int WAVES, int CPL, int R, bool ALIGNED>
__global__ __launch_bounds__(WAVES * 64, (WAVES >= 4 ? 2 : 1)) void k_gram(
    const T* __restrict__ A, int64_t n, int d, int64_t ld, int64_t rows_per_wg, int mode,
    const double* __restrict__ p, const double* __restrict__ aux, double* __restrict__ auxout,
    double* __restrict__ ypart, int ldy, double* __restrict__ qpart,
    const int* __restrict__ done, PcgDev* __restrict__ note, int note_seq) {
  constexpr int NT = WAVES * 64;
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
  publish_state(done, note, note_seq);
  if (done != nullptr && *done) return;

  __shared__ double red[2][R][WAVES];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = (r0 + rows_per_wg < n) ? r0 + rows_per_wg : n;
  const bool tonly = (mode == kModeTOnly);

  double pr[CPL][VN], yr[CPL][VN];
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    const int c0 = col0<T, CPL, ALIGNED, NT>(tid, m);
#pragma unroll
    for (int v = 0; v < VN; ++v) {
      pr[m][v] = (!tonly && c0 + v < d) ? p[c0 + v] : 0.0;
      yr[m][v] = 0.0;
    }
  }
  double q = 0.0;
  int buf = 0;

  V a0[R][CPL], a1[R][CPL];
  T e0[R][Extra<T>::N], e1[R][Extra<T>::N];
  double v0[R], v1[R];
  load_group<T, CPL, R, ALIGNED, NT>(a0, e0, v0, A, aux, r0, r1, d, ld, tid);
  for (int64_t row = r0; row < r1; row += 2 * R) {
    load_group<T, CPL, R, ALIGNED, NT>(a1, e1, v1, A, aux, row + R, r1, d, ld, tid);
    realign_group<T, CPL, R, ALIGNED, NT>(a0, e0, A, row, d, ld, tid);
    process_group<T, WAVES, CPL, R>(a0, v0, row, r1, mode, pr, yr, q, aux, auxout, red, buf,
                                    tid);
    if (row + R >= r1) break;
    load_group<T, CPL, R, ALIGNED, NT>(a0, e0, v0, A, aux, row + 2 * R, r1, d, ld, tid);
    realign_group<T, CPL, R, ALIGNED, NT>(a1, e1, A, row + R, d, ld, tid);
    process_group<T, WAVES, CPL, R>(a1, v1, row + R, r1, mode, pr, yr, q, aux, auxout, red, buf,
                                    tid);
  }

  double* yp = ypart + (int64_t)blockIdx.x * ldy;
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    const int c0 = col0<T, CPL, ALIGNED, NT>(tid, m);
#pragma unroll
    for (int v = 0; v < VN; ++v)
      if (c0 + v < d) yp[c0 + v] = yr[m][v];
  }
  if (tid == 0) qpart[blockIdx.x] = q;
}

// y = A p for an explicit symmetric A (kernel SVM), one block of columns per
// blockIdx.y: the same streaming of rows as k_gram without the A^T pass; the
// row dots of column block s go to ypart[s * ldy + row] (summed over blocks by
// the reduction kernel) and sum_i p_i t_i to qpart[s * gridDim.x + blockIdx.x].
template <typename T, int WAVES, int CPL, int R, bool ALIGNED>
__global__ __launch_bounds__(WAVES * 64, (WAVES >= 4 ? 2 : 1)) void k_rowdot(
    const T* __restrict__ A, int64_t n, int64_t ncols, int64_t ld, int slice_cols,
    int64_t rows_per_wg, const double* __restrict__ p, double* __restrict__ ypart, int ldy,
    double* __restrict__ qpart, const int* __restrict__ done, PcgDev* __restrict__ note,
    int note_seq) {
  constexpr int NT = WAVES * 64;
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
  publish_state(done, note, note_seq);
  if (done != nullptr && *done) return;
  __shared__ double red[2][R][WAVES];
  const int tid = threadIdx.x;
  const int64_t c0s = (int64_t)blockIdx.y * slice_cols;
  const int d = (int)((ncols - c0s < slice_cols) ? ncols - c0s : slice_cols);
  const T* As = A + c0s;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = (r0 + rows_per_wg < n) ? r0 + rows_per_wg : n;
  double pr[CPL][VN];
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    const int c0 = col0<T, CPL, ALIGNED, NT>(tid, m);
#pragma unroll
    for (int v = 0; v < VN; ++v) pr[m][v] = (c0 + v < d) ? p[c0s + c0 + v] : 0.0;
  }
  double* out = ypart + (int64_t)blockIdx.y * ldy;
  double q = 0.0;
  int buf = 0;
  V a0[R][CPL], a1[R][CPL];
  T e0[R][Extra<T>::N], e1[R][Extra<T>::N];
  double v0[R], v1[R];
  load_group<T, CPL, R, ALIGNED, NT>(a0, e0, v0, As, p, r0, r1, d, ld, tid);
  for (int64_t row = r0; row < r1; row += 2 * R) {
    load_group<T, CPL, R, ALIGNED, NT>(a1, e1, v1, As, p, row + R, r1, d, ld, tid);
    realign_group<T, CPL, R, ALIGNED, NT>(a0, e0, As, row, d, ld, tid);
    rowdot_group<T, WAVES, CPL, R>(a0, v0, row, r1, pr, q, out, red, buf, tid);
    if (row + R >= r1) break;
    load_group<T, CPL, R, ALIGNED, NT>(a0, e0, v0, As, p, row + 2 * R, r1, d, ld, tid);
    realign_group<T, CPL, R, ALIGNED, NT>(a1, e1, As, row + R, d, ld, tid);
    rowdot_group<T, WAVES, CPL, R>(a1, v1, row + R, r1, pr, q, out, red, buf, tid);
  }
  if (tid == 0) qpart[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = q;
}

template <typename T, int WAVES, int CPL, int R>
nys_status launch_r(const nys_dense& A, const GramPlan& pl, int mode, const double* p,
                    const double* aux, double* auxout, double* ypart, double* qpart,
                    const int* done, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                    PcgDev* note, int note_seq) {
  const T* a = static_cast<const T*>(A.data);
  // with events, the dispatch itself stamps the kernel's start and end
  if (ev0 != nullptr) {
    if (pl.aligned)
      hipExtLaunchKernelGGL((k_gram<T, WAVES, CPL, R, true>), dim3(pl.grid), dim3(WAVES * 64), 0,
                            st, ev0, ev1, 0, a, A.n, (int)A.d, A.ld, pl.rows_per_wg, mode, p,
                            aux, auxout, ypart, pl.ldy, qpart, done, note, note_seq);
    else
      hipExtLaunchKernelGGL((k_gram<T, WAVES, CPL, R, false>), dim3(pl.grid), dim3(WAVES * 64),
                            0, st, ev0, ev1, 0, a, A.n, (int)A.d, A.ld, pl.rows_per_wg, mode, p,
                            aux, auxout, ypart, pl.ldy, qpart, done, note, note_seq);
  } else if (pl.aligned) {
    hipLaunchKernelGGL((k_gram<T, WAVES, CPL, R, true>), dim3(pl.grid), dim3(WAVES * 64), 0, st,
                       a, A.n, (int)A.d, A.ld, pl.rows_per_wg, mode, p, aux, auxout, ypart,
                       pl.ldy, qpart, done, note, note_seq);
  } else {
    hipLaunchKernelGGL((k_gram<T, WAVES, CPL, R, false>), dim3(pl.grid), dim3(WAVES * 64), 0, st,
                       a, A.n, (int)A.d, A.ld, pl.rows_per_wg, mode, p, aux, auxout, ypart,
                       pl.ldy, qpart, done, note, note_seq);
  }
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

template <typename T>
nys_status launch_dt(const nys_dense& A, const GramPlan& pl, int mode, const double* p,
                     const double* aux, double* auxout, double* ypart, double* qpart,
                     const int* done, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                     PcgDev* note, int note_seq) {
#define NYS_CASE(W, C, RR)                                                                  \
  if (pl.waves == W && pl.cpl == C && pl.rows == RR)                                        \
    return launch_r<T, W, C, RR>(A, pl, mode, p, aux, auxout, ypart, qpart, done, st, ev0, ev1, \
                                 note, note_seq);
  NYS_CASE(1, 2, 4) NYS_CASE(2, 2, 4) NYS_CASE(4, 2, 4) NYS_CASE(8, 2, 4)
  NYS_CASE(1, 2, 8) NYS_CASE(2, 2, 8) NYS_CASE(4, 2, 8) NYS_CASE(8, 2, 8)
  NYS_CASE(1, 3, 2) NYS_CASE(2, 3, 2) NYS_CASE(4, 3, 2) NYS_CASE(8, 3, 2)
  NYS_CASE(1, 4, 2) NYS_CASE(2, 4, 2) NYS_CASE(4, 4, 2) NYS_CASE(8, 4, 2)
#undef NYS_CASE
  return NYS_ERR_INVALID;
}

}  // namespace

int64_t gram_max_cols(nys_dtype dt) { return dt == NYS_F64 ? 8 * 64 * 4 * 2 : 8 * 64 * 4 * 4; }

static void finish_plan(const nys_dense& A, int num_cu, int per_cu, GramPlan* pl) {
  const int esize = A.dtype == NYS_F64 ? 8 : 4;
  pl->aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
  pl->ldy = (int)((A.d + 63) / 64 * 64);
  pl->per_cu = per_cu;
  if (A.n <= 0) {
    pl->grid = 0;
    pl->rows_per_wg = 0;
    return;
  }
  // one full round of resident workgroups, each streaming a contiguous row range
  const int R = pl->rows;
  const int64_t groups = (A.n + R - 1) / R;
  const int64_t g = std::min<int64_t>((int64_t)per_cu * num_cu, std::max<int64_t>(1, groups / 2));
  pl->rows_per_wg = ((A.n + g - 1) / g + R - 1) / R * R;
  pl->grid = (int)((A.n + pl->rows_per_wg - 1) / pl->rows_per_wg);
}

// Launch shapes worth timing for this matrix: every supported (waves, chunks,
// rows) whose row coverage is at least d and at most about twice d, with 1..2
// rounds' worth of workgroups per CU at 2 waves per SIMD.
std::vector<GramPlan> gram_candidates(const nys_dense& A, int num_cu) {
  static const int shapes[][3] = {{1, 2, 4}, {1, 2, 8}, {2, 2, 4}, {2, 2, 8}, {4, 2, 4},
                                  {4, 2, 8}, {8, 2, 4}, {8, 2, 8}, {1, 3, 2}, {2, 3, 2},
                                  {4, 3, 2}, {8, 3, 2}, {1, 4, 2}, {2, 4, 2}, {4, 4, 2},
                                  {8, 4, 2}};
  const int vn = A.dtype == NYS_F64 ? 2 : 4;
  const int64_t need = std::max<int64_t>(A.d, 1);
  int64_t best_cover = -1;
  for (auto& sh : shapes) {
    const int64_t cover = (int64_t)sh[0] * 64 * sh[1] * vn;
    if (cover >= need && (best_cover < 0 || cover < best_cover)) best_cover = cover;
  }
  // unaligned rows carry the realignment state; groups of 8 rows then spill
  const int esize = A.dtype == NYS_F64 ? 8 : 4;
  const bool aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
  std::vector<GramPlan> out;
  for (auto& sh : shapes) {
    const int64_t cover = (int64_t)sh[0] * 64 * sh[1] * vn;
    if (cover < need || cover > 2 * std::max<int64_t>(best_cover, 1)) continue;
    if (!aligned && sh[2] == 8) continue;
    const int max_per_cu = std::max(1, 8 / sh[0]);
    for (int per_cu : {max_per_cu / 2, max_per_cu}) {
      if (per_cu < 1) continue;
      GramPlan pl;
      pl.waves = sh[0];
      pl.cpl = sh[1];
      pl.rows = sh[2];
      finish_plan(A, num_cu, per_cu, &pl);
      out.push_back(pl);
    }
  }
  return out;
}

// Heuristic plan: the narrowest row coverage with 4 chunks per lane when it
// fits in at most 4 waves (two workgroups per CU, rows in double-buffered
// groups of 2), else 2 chunks per lane.  NYSADMM_GRAM_PLAN="waves,cpl,rows,
// wg_per_cu" overrides (launch-shape sweeps).
GramPlan make_gram_plan(const nys_dense& A, int num_cu) {
  GramPlan pl;
  const int vn = A.dtype == NYS_F64 ? 2 : 4;
  const int64_t d = A.d;
  static const int pref[][3] = {{1, 2, 8}, {2, 2, 8}, {2, 4, 2}, {4, 4, 2}, {8, 2, 4}, {8, 4, 2}};
  static const int pref_u[][3] = {{1, 2, 4}, {2, 2, 4}, {2, 4, 2}, {4, 4, 2}, {8, 2, 4}, {8, 4, 2}};
  const int esize = A.dtype == NYS_F64 ? 8 : 4;
  const bool aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
  pl.waves = 8;
  pl.cpl = 4;
  pl.rows = 2;
  for (auto& c : (aligned ? pref : pref_u)) {
    if ((int64_t)c[0] * 64 * c[1] * vn >= d) {
      pl.waves = c[0];
      pl.cpl = c[1];
      pl.rows = c[2];
      break;
    }
  }
  int per_cu = std::max(1, 8 / pl.waves);
  if (const char* e = getenv("NYSADMM_GRAM_PLAN")) {
    int w = 0, c = 0, rr = 0, g = 0;
    if (sscanf(e, "%d,%d,%d,%d", &w, &c, &rr, &g) == 4 && (int64_t)w * 64 * c * vn >= d &&
        (w == 1 || w == 2 || w == 4 || w == 8) &&
        ((c == 2 && (rr == 4 || rr == 8)) || ((c == 3 || c == 4) && rr == 2)) && g >= 1) {
      pl.waves = w;
      pl.cpl = c;
      pl.rows = rr;
      per_cu = g;
    }
  }
  finish_plan(A, num_cu, per_cu, &pl);
  return pl;
}

// The heuristic plan with at most max_grid workgroups (longer row ranges per
// workgroup), for callers whose partial-sum buffer has a fixed size.
GramPlan make_gram_plan_capped(const nys_dense& A, int num_cu, int64_t max_grid) {
  GramPlan pl = make_gram_plan(A, num_cu);
  if (max_grid < 1 || pl.grid <= max_grid || A.n <= 0) return pl;
  const int R = pl.rows;
  pl.rows_per_wg = ((A.n + max_grid - 1) / max_grid + R - 1) / R * R;
  pl.grid = (int)((A.n + pl.rows_per_wg - 1) / pl.rows_per_wg);
  return pl;
}

// Plan of the column-blocked y = A p (explicit symmetric A): blocks of 4096
// columns (4 waves x 4 chunks of 4 floats; 2048 for FP64), rows split so that
// blocks x row ranges give about two workgroups per CU.
GramPlan make_symv_plan(const nys_dense& A, int num_cu) {
  GramPlan pl;
  pl.symv = true;
  pl.waves = 4;
  pl.cpl = 4;
  pl.rows = 2;
  const int vn = A.dtype == NYS_F64 ? 2 : 4;
  pl.slice_cols = pl.waves * 64 * pl.cpl * vn;
  pl.slices = (int)std::max<int64_t>(1, (A.d + pl.slice_cols - 1) / pl.slice_cols);
  const int esize = A.dtype == NYS_F64 ? 8 : 4;
  pl.aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
  pl.ldy = (int)((A.n + 63) / 64 * 64);
  pl.per_cu = 2;
  if (A.n <= 0) {
    pl.grid = 0;
    pl.rows_per_wg = 0;
    return pl;
  }
  const int64_t groups = (A.n + pl.rows - 1) / pl.rows;
  const int64_t want = std::max<int64_t>(1, (int64_t)pl.per_cu * num_cu / pl.slices);
  const int64_t g = std::min<int64_t>(want, std::max<int64_t>(1, groups / 2));
  pl.rows_per_wg = ((A.n + g - 1) / g + pl.rows - 1) / pl.rows * pl.rows;
  pl.grid = (int)((A.n + pl.rows_per_wg - 1) / pl.rows_per_wg);
  return pl;
}

nys_status launch_symv(const nys_dense& A, const GramPlan& pl, const double* p, double* ypart,
                       double* qpart, const int* done, hipStream_t st, hipEvent_t ev0,
                       hipEvent_t ev1, PcgDev* note, int note_seq) {
  if (!pl.symv || pl.waves != 4 || pl.cpl != 4 || pl.rows != 2) return NYS_ERR_INVALID;
  if (A.n != A.d) return NYS_ERR_INVALID;
  if (A.n == 0 || pl.grid == 0) return NYS_OK;
  const dim3 grid(pl.grid, pl.slices);
#define NYS_SYMV(T, AL)                                                                        \
  do {                                                                                         \
    const T* a = static_cast<const T*>(A.data);                                                \
    if (ev0 != nullptr)                                                                        \
      hipExtLaunchKernelGGL((k_rowdot<T, 4, 4, 2, AL>), grid, dim3(256), 0, st, ev0, ev1, 0, a, \
                            A.n, A.d, A.ld, pl.slice_cols, pl.rows_per_wg, p, ypart, pl.ldy,   \
                            qpart, done, note, note_seq);                                      \
    else                                                                                       \
      hipLaunchKernelGGL((k_rowdot<T, 4, 4, 2, AL>), grid, dim3(256), 0, st, a, A.n, A.d,       \
                         A.ld, pl.slice_cols, pl.rows_per_wg, p, ypart, pl.ldy, qpart, done,   \
                         note, note_seq);                                                      \
  } while (0)
  if (A.dtype == NYS_F32) {
    if (pl.aligned) NYS_SYMV(float, true);
    else NYS_SYMV(float, false);
  } else if (A.dtype == NYS_F64) {
    if (pl.aligned) NYS_SYMV(double, true);
    else NYS_SYMV(double, false);
  } else {
    return NYS_ERR_INVALID;
  }
#undef NYS_SYMV
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status launch_gram(const nys_dense& A, const GramPlan& pl, int mode, const double* p,
                       const double* aux, double* auxout, double* ypart, double* qpart,
                       const int* done, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                       PcgDev* note, int note_seq) {
  const int vn = A.dtype == NYS_F64 ? 2 : 4;
  if ((int64_t)pl.waves * 64 * pl.cpl * vn < A.d) return NYS_ERR_INVALID;
  if (A.n == 0 || pl.grid == 0) return NYS_OK;
  if (A.dtype == NYS_F64)
    return launch_dt<double>(A, pl, mode, p, aux, auxout, ypart, qpart, done, st, ev0, ev1, note,
                             note_seq);
  if (A.dtype == NYS_F32)
    return launch_dt<float>(A, pl, mode, p, aux, auxout, ypart, qpart, done, st, ev0, ev1, note,
                            note_seq);
  return NYS_ERR_INVALID;
}

}  // namespace nys
