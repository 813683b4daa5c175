// Sparse A (CSR) for the NysADMM hot path: the matvec pair A^T (D (A p)) as
// two streaming passes, a row pass over the CSR arrays (t = A p and the mode
// epilogue s = f(t)) and a column pass over a CSC copy (y = A^T s), and the
// sketch A^T (D (A Omega)) as two sparse-times-dense products.  One wavefront
// per row (column); every sum is FP64 in a fixed order, so results are
// bitwise reproducible.  The CSC copy is built once by a deterministic
// counting transpose: rows are split into blocks, each block's column counts
// are prefix-summed across blocks, and each block places its entries row by
// row (within a row the columns are distinct, so no two lanes share a slot).
#include <algorithm>
#include <cmath>
#include <new>

#include "internal.h"

#include "gram_device.h"

namespace nys {
namespace {

using gram::sigm;
using gram::wave_sum;

constexpr int kTBlocks = 64;   // row blocks of the transpose
constexpr int kShortCol = 32;  // columns with at most this many entries: 8 lanes each
constexpr int kLongCol = 2048; // columns with more: a 256-thread workgroup each

// Column j goes to list 0 (short), 1 (medium) or 2 (long), each list in
// increasing column order (so a pass over a list reads the CSC arrays in
// storage order) as the triple (j, colptr[j], colptr[j + 1]), so that the
// column pass finds a column's range with one load; counts[3] are the list
// lengths.  One workgroup: thread t counts its contiguous range of columns
// per class, the counts are prefix-summed, and each thread places its range
// in order.
__device__ __forceinline__ int col_class(const int* __restrict__ colptr, int64_t j) {
  const int len = colptr[j + 1] - colptr[j];
  return len <= kShortCol ? 0 : (len <= kLongCol ? 1 : 2);
}
__global__ __launch_bounds__(1024) void k_bin_cols(const int* __restrict__ colptr, int64_t d,
                                                   int4* __restrict__ lists,
                                                   int* __restrict__ counts) {
  __shared__ int part[3][1024];
  const int t = threadIdx.x;
  const int64_t per = (d + 1023) / 1024;
  const int64_t j0 = std::min<int64_t>(d, t * per), j1 = std::min<int64_t>(d, j0 + per);
  int c[3] = {0, 0, 0};
  for (int64_t j = j0; j < j1; ++j) ++c[col_class(colptr, j)];
#pragma unroll
  for (int b = 0; b < 3; ++b) part[b][t] = c[b];
  __syncthreads();
  if (t < 3) {
    int acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const int v = part[t][i];
      part[t][i] = acc;
      acc += v;
    }
    counts[t] = acc;
  }
  __syncthreads();
  int pos[3] = {part[0][t], part[1][t], part[2][t]};
  for (int64_t j = j0; j < j1; ++j) {
    const int b = col_class(colptr, j);
    lists[(int64_t)b * d + pos[b]++] = make_int4((int)j, colptr[j], colptr[j + 1], 0);
  }
}

// *bad = 1 unless rowptr is non-decreasing (its ends were checked on the host)
__global__ __launch_bounds__(256) void k_tr_check_rows(const int* __restrict__ rowptr, int64_t n,
                                                       int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && rowptr[i + 1] < rowptr[i]) *bad = 1;
}

// cnt[b * d + j] = entries of column j in row block b; *bad = 1 on a column
// index outside [0, d) (not counted)
__global__ __launch_bounds__(256) void k_tr_count(const int* __restrict__ rowptr,
                                                  const int* __restrict__ col, int64_t n,
                                                  int64_t d, int64_t rows_per_blk,
                                                  int* __restrict__ cnt, int* __restrict__ bad) {
  const int b = blockIdx.y;
  const int64_t r0 = (int64_t)b * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_blk);
  if (r0 >= r1) return;
  const int64_t k0 = rowptr[r0], k1 = rowptr[r1];
  for (int64_t k = k0 + (int64_t)blockIdx.x * 256 + threadIdx.x; k < k1;
       k += (int64_t)gridDim.x * 256) {
    const int j = col[k];
    if (j < 0 || j >= d) {
      *bad = 1;
      continue;
    }
    atomicAdd(&cnt[(int64_t)b * d + j], 1);   // integer counts: order-free
  }
}

// colptr[j] (exclusive) and, in place, cnt[b * d + j] <- start of block b's
// entries of column j, in three passes over the counts:
//   k_tr_colsum:  per column j (one thread, coalesced over j), cnt[b * d + j]
//                 <- the entries of blocks before b, colptr[j] <- the total;
//   k_tr_colscan: exclusive scan of colptr[0, d) in place, colptr[d] = nnz
//                 (one workgroup; threads own contiguous column ranges);
//   k_tr_addbase: cnt[b * d + j] += colptr[j].
__global__ __launch_bounds__(256) void k_tr_colsum(int* __restrict__ cnt, int64_t d, int nblk,
                                                   int* __restrict__ colptr) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= d) return;
  int s = 0;
  for (int b = 0; b < nblk; ++b) {
    const int c = cnt[(int64_t)b * d + j];
    cnt[(int64_t)b * d + j] = s;
    s += c;
  }
  colptr[j] = s;
}
__global__ __launch_bounds__(1024) void k_tr_colscan(int* __restrict__ colptr, int64_t d) {
  __shared__ long long part[1024];
  const int64_t per = (d + 1023) / 1024;
  const int64_t j0 = std::min<int64_t>(d, threadIdx.x * per);
  const int64_t j1 = std::min<int64_t>(d, j0 + per);
  long long s = 0;
  for (int64_t j = j0; j < j1; ++j) s += colptr[j];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const long long v = part[i];
      part[i] = acc;
      acc += v;
    }
    colptr[d] = (int)acc;
  }
  __syncthreads();
  long long acc = part[threadIdx.x];
  for (int64_t j = j0; j < j1; ++j) {
    const int c = colptr[j];
    colptr[j] = (int)acc;
    acc += c;
  }
}
__global__ __launch_bounds__(256) void k_tr_addbase(int* __restrict__ cnt, int64_t d, int nblk,
                                                    const int* __restrict__ colptr) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= d) return;
  const int base = colptr[j];
  for (int b = 0; b < nblk; ++b) cnt[(int64_t)b * d + j] += base;
}

// Block b places its rows in order: each lane takes distinct columns of one
// row, so the slot counters cnt[b * d + col] are bumped without conflicts.
__global__ __launch_bounds__(64) void k_tr_fill(const int* __restrict__ rowptr,
                                                const int* __restrict__ col,
                                                const float* __restrict__ val, int64_t n,
                                                int64_t d, int64_t rows_per_blk,
                                                int* __restrict__ cnt, int* __restrict__ rows,
                                                float* __restrict__ cval) {
  const int b = blockIdx.x;
  const int64_t r0 = (int64_t)b * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_blk);
  int* c = cnt + (int64_t)b * d;
  for (int64_t i = r0; i < r1; ++i) {
    for (int64_t k = rowptr[i] + threadIdx.x; k < rowptr[i + 1]; k += 64) {
      const int j = col[k];
      const int pos = c[j];
      c[j] = pos + 1;
      rows[pos] = (int)i;
      cval[pos] = val[k];
    }
    __syncthreads();   // one wavefront: orders the counter updates row by row
  }
}

// sum over k = k0, k0 + step, ... (below k1) of v[k] x[idx[k]]: four terms
// in flight per lane (their index and value loads issued together, then the
// four gathers), four running sums combined in a fixed order, then the
// remaining terms one at a time.  x[i] is read from xl (LDS) for i < head.
// (Eight or more terms in flight per lane measured slower at the E2006.train
// shape: the extra registers cost more occupancy than the longer batches
// save.)
__device__ __forceinline__ double gather_dot(const int* __restrict__ idx,
                                             const float* __restrict__ v,
                                             const double* __restrict__ x, const double* xl,
                                             int head, int64_t k0, int64_t k1, int step) {
  auto X = [&](int i) { return i < head ? xl[i] : x[i]; };
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t k = k0;
  for (; k + 3 * step < k1; k += 4 * step) {
    const int i0 = idx[k], i1 = idx[k + step], i2 = idx[k + 2 * step], i3 = idx[k + 3 * step];
    const float v0 = v[k], v1 = v[k + step], v2 = v[k + 2 * step], v3 = v[k + 3 * step];
    a0 = fma((double)v0, X(i0), a0);
    a1 = fma((double)v1, X(i1), a1);
    a2 = fma((double)v2, X(i2), a2);
    a3 = fma((double)v3, X(i3), a3);
  }
  for (; k < k1; k += step) a0 = fma((double)v[k], X(idx[k]), a0);
  return (a0 + a1) + (a2 + a3);
}

// Row pass: t_i = A_i p (one wavefront per row), s_i = f_mode(t_i) into s,
// per-workgroup sum of the mode's q term into qpart.  Persistent workgroups
// of 1024 threads (one per CU): the first kCsrHead entries of p are staged in
// LDS, where the gathers of the popular (low-index) columns of bag-of-words
// data land, and wavefront w of workgroup g takes rows g * 16 + w, then
// every 16 * gridDim.x rows on; its q terms are added in row order, the 16
// wavefronts' sums in wavefront order.
constexpr int kCsrT = 1024;
constexpr int kCsrHead = 16384;
__global__ __launch_bounds__(kCsrT) void k_csr_pass(const int* __restrict__ rowptr,
                                                    const int* __restrict__ col,
                                                    const float* __restrict__ val, int64_t n,
                                                    int64_t d, int mode,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ aux,
                                                    double* __restrict__ auxout,
                                                    double* __restrict__ s,
                                                    double* __restrict__ qpart,
                                                    const int* __restrict__ done,
                                                    PcgDev* __restrict__ note, int note_seq) {
  publish_state(done, note, note_seq);
  if (done != nullptr && *done) return;
  __shared__ double pl[kCsrHead];
  __shared__ double qs[kCsrT / 64];
  const int head = (mode == kModeTOnly) ? 0 : (int)(d < kCsrHead ? d : kCsrHead);
  for (int i = threadIdx.x; i < head; i += kCsrT) pl[i] = p[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double q = 0.0;
  const int64_t stride = (int64_t)gridDim.x * (kCsrT / 64);
  for (int64_t i = (int64_t)blockIdx.x * (kCsrT / 64) + wv; i < n; i += stride) {
    double acc = 0.0;
    if (mode != kModeTOnly) acc = gather_dot(col, val, p, pl, head, rowptr[i] + lane,
                                             rowptr[i + 1], 64);
    const double t = wave_sum(acc);
    if (lane == 0) {
      double si = 0.0, qi = 0.0;
      if (mode == kModeHess) {
        si = (aux != nullptr ? aux[i] : 1.0) * t;
        qi = si * t;
      } else if (mode == kModeLsGrad) {
        si = t - aux[i];
        qi = si * si;
      } else if (mode == kModeLogit || mode == kModeLogGrad) {
        const double bi = aux[i];
        const double sg = sigm(t);
        qi = log1p(exp(-fabs(t))) + fmax(t, 0.0) - bi * t;
        if (mode == kModeLogit) {
          const double w = sg * sigm(-t);
          si = w * t + bi - sg;
          if (auxout != nullptr) auxout[i] = w;
        } else {
          si = sg - bi;
        }
      } else {   // kModeTOnly
        si = aux[i];
      }
      s[i] = si;
      q += qi;
    }
  }
  if (lane == 0) qs[wv] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kCsrT / 64; ++w) r += qs[w];
    qpart[blockIdx.x] = r;
  }
}

// Column pass: y_j = sum over column j of A_ij s_i, one launch for the three
// column lists (triples (j, begin, end)): workgroups [0, nlong) take one long
// column each (256 threads), the next ceil(nmed / 4) one medium column per
// wavefront, the rest 32 short columns each (8 lanes per column).  Long
// columns come first so that the longest work is dispatched first.  Fixed
// summation order per column.
__global__ __launch_bounds__(256) void k_csc_pass(const int* __restrict__ rows,
                                                  const float* __restrict__ cval,
                                                  const int4* __restrict__ lists, int64_t d,
                                                  int nshort, int nmed, int nlong,
                                                  const double* __restrict__ s,
                                                  double* __restrict__ y,
                                                  const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  const int bid = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int gm = (nmed + 3) / 4;
  if (bid < nlong) {
    __shared__ double red[4];
    const int4 c = lists[2 * d + bid];
    double acc = gather_dot(rows, cval, s, nullptr, 0, c.y + tid, c.z, 256);
    acc = wave_sum(acc);
    if (lane == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) y[c.x] = ((red[0] + red[1]) + red[2]) + red[3];
  } else if (bid < nlong + gm) {
    const int g = (bid - nlong) * 4 + (tid >> 6);
    if (g >= nmed) return;
    const int4 c = lists[d + g];
    double acc = gather_dot(rows, cval, s, nullptr, 0, c.y + lane, c.z, 64);
    acc = wave_sum(acc);
    if (lane == 0) y[c.x] = acc;
  } else {
    const int g = (bid - nlong - gm) * 32 + (tid >> 3);
    const int sub = tid & 7;
    double acc = 0.0;
    int j = -1;
    if (g < nshort) {
      const int4 c = lists[g];
      j = c.x;
      acc = gather_dot(rows, cval, s, nullptr, 0, c.y + sub, c.z, 8);
    }
    acc += __shfl_xor(acc, 4, 8);
    acc += __shfl_xor(acc, 2, 8);
    acc += __shfl_xor(acc, 1, 8);
    if (j >= 0 && sub == 0) y[j] = acc;
  }
}

// Omega (column-major d x m) -> row-major d x m
__global__ void k_cm_to_rm(const double* __restrict__ cm, int64_t d, int m,
                           double* __restrict__ rm) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= d * m) return;
  const int64_t j = e / m, c = e % m;
  rm[e] = cm[c * d + j];
}

// Y column-major (ld d) <- Yrm (row-major d x m) + c Om (column-major)
__global__ void k_rm_to_cm(const double* __restrict__ rm, int64_t d, int m, double c,
                           const double* __restrict__ Om, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= d * m) return;
  const int64_t col = e / d, j = e % d;
  Y[e] = rm[j * m + col] + c * Om[e];
}

// T = D (A Om) row by row (row-major n x m): one wavefront per row, each lane
// owning columns lane, lane + 64, ... of a 256-column chunk (blockIdx.y).
// acc[h] = sum over k0 <= k < k1 of v[k] B[idx[k] * m + c0 + 64 h] (h < NH,
// columns below m; lanes past m load column 0 and add zero): four nonzeros in
// flight per lane with no branch around the loads, four running sums per
// column combined in a fixed order
template <int NH>
__device__ __forceinline__ void spmm_acc(const int* __restrict__ idx, const float* __restrict__ v,
                                         const double* __restrict__ B, int64_t k0, int64_t k1,
                                         int m, int c0, double (&acc)[4]) {
  int cc[NH];
  bool ok[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    ok[h] = c0 + 64 * h < m;
    cc[h] = ok[h] ? c0 + 64 * h : 0;
  }
  double a[4][NH];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int h = 0; h < NH; ++h) a[u][h] = 0.0;
  int64_t k = k0;
  for (; k + 3 < k1; k += 4) {
    double bv[4][NH];
    float vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      vv[u] = v[k + u];
      const double* b = B + (int64_t)idx[k + u] * m;
#pragma unroll
      for (int h = 0; h < NH; ++h) bv[u][h] = b[cc[h]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int h = 0; h < NH; ++h) a[u][h] = fma((double)vv[u], ok[h] ? bv[u][h] : 0.0, a[u][h]);
  }
  for (; k < k1; ++k) {
    const double vv = v[k];
    const double* b = B + (int64_t)idx[k] * m;
#pragma unroll
    for (int h = 0; h < NH; ++h) a[0][h] = fma(vv, ok[h] ? b[cc[h]] : 0.0, a[0][h]);
  }
#pragma unroll
  for (int h = 0; h < 4; ++h)
    acc[h] = h < NH ? (a[0][h < NH ? h : 0] + a[1][h < NH ? h : 0]) +
                          (a[2][h < NH ? h : 0] + a[3][h < NH ? h : 0])
                    : 0.0;
}

template <int NH>
__global__ __launch_bounds__(256) void k_csr_spmm(const int* __restrict__ rowptr,
                                                  const int* __restrict__ col,
                                                  const float* __restrict__ val, int64_t n,
                                                  int m, const double* __restrict__ B,
                                                  const double* __restrict__ D,
                                                  double* __restrict__ T) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int c0 = blockIdx.y * 256 + lane;
  double acc[4];
  spmm_acc<NH>(col, val, B, rowptr[i], rowptr[i + 1], m, c0, acc);
  const double di = D != nullptr ? D[i] : 1.0;
#pragma unroll
  for (int h = 0; h < 4; ++h)
    if (c0 + 64 * h < m) T[i * m + c0 + 64 * h] = di * acc[h];
}

// Yrm = A^T T column by column (row-major d x m), the same layout of lanes
template <int NH>
__global__ __launch_bounds__(256) void k_csc_spmm(const int* __restrict__ colptr,
                                                  const int* __restrict__ rows,
                                                  const float* __restrict__ cval, int64_t d,
                                                  int m, const double* __restrict__ T,
                                                  double* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= d) return;
  const int c0 = blockIdx.y * 256 + lane;
  double acc[4];
  spmm_acc<NH>(rows, cval, T, colptr[j], colptr[j + 1], m, c0, acc);
#pragma unroll
  for (int h = 0; h < 4; ++h)
    if (c0 + 64 * h < m) Y[j * m + c0 + 64 * h] = acc[h];
}

inline unsigned nb256(int64_t x) { return (unsigned)((x + 255) / 256); }

}  // namespace

GramPlan make_sparse_plan(const nys_sparse_s* S) {
  GramPlan pl;
  pl.sparse = S;
  // row-pass workgroups (q partials): one per CU, fewer for small n
  pl.grid = (int)std::max<int64_t>(
      1, std::min<int64_t>(std::max(S->num_cu, 1), (S->n + kCsrT / 64 - 1) / (kCsrT / 64)));
  pl.ldy = (int)((S->d + 63) / 64 * 64);
  pl.rows_per_wg = kCsrT / 64;
  return pl;
}

nys_status launch_sparse_pair(const nys_sparse_s* S, const GramPlan& pl, int mode,
                              const double* p, const double* aux, double* auxout, double* ypart,
                              double* qpart, const int* done, hipStream_t st, hipEvent_t ev0,
                              hipEvent_t ev1, PcgDev* note, int note_seq) {
  if (S == nullptr || pl.sparse != S) return NYS_ERR_INVALID;
  double* s = S->s.as<double>();
  if (ev0 != nullptr) NYS_TRY_HIP(hipEventRecord(ev0, st));
  if (S->n > 0)
    hipLaunchKernelGGL(k_csr_pass, dim3(pl.grid), dim3(kCsrT), 0, st, S->rowptr, S->colidx,
                       S->val, S->n, S->d, mode, p, aux, auxout, s, qpart, done, note, note_seq);
  else {
    NYS_TRY_HIP(hipMemsetAsync(qpart, 0, sizeof(double), st));
    if (note != nullptr)
      NYS_TRY(launch_note(reinterpret_cast<const PcgDev*>(done), note, note_seq, st));
  }
  const int4* lists = S->bins.as<int4>();
  const int64_t gcsc = (int64_t)S->nlong + (S->nmed + 3) / 4 + (S->nshort + 31) / 32;
  if (gcsc > 0)
    hipLaunchKernelGGL(k_csc_pass, dim3((unsigned)gcsc), dim3(256), 0, st, S->rows(), S->cvals(),
                       lists, S->d, S->nshort, S->nmed, S->nlong, s, ypart, done);
  if (ev1 != nullptr) NYS_TRY_HIP(hipEventRecord(ev1, st));
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status sparse_sketch(const nys_sparse_s* S, const double* D, double c, const double* Om, int m,
                         double* Y, double* ws, hipStream_t st) {
  const int64_t n = S->n, d = S->d;
  double* Orm = ws;                  // d x m
  double* T = ws + d * m;            // n x m
  double* Yrm = T + n * m;           // d x m
  const unsigned cchunks = (unsigned)((m + 255) / 256);
  hipLaunchKernelGGL(k_cm_to_rm, dim3(nb256(d * m)), dim3(256), 0, st, Om, d, m, Orm);
  // column blocks of 64 per lane group actually used (one 256-column chunk
  // per blockIdx.y; NH = 4 once m exceeds 192)
  const int nh = m >= 256 ? 4 : (m + 63) / 64;
#define NYS_SPMM(NH)                                                                           \
  do {                                                                                         \
    if (n > 0)                                                                                 \
      hipLaunchKernelGGL(k_csr_spmm<NH>, dim3((unsigned)((n + 3) / 4), cchunks), dim3(256), 0,  \
                         st, S->rowptr, S->colidx, S->val, n, m, Orm, D, T);                   \
    hipLaunchKernelGGL(k_csc_spmm<NH>, dim3((unsigned)((d + 3) / 4), cchunks), dim3(256), 0,    \
                       st, S->colptr(), S->rows(), S->cvals(), d, m, T, Yrm);                  \
  } while (0)
  if (nh == 1) NYS_SPMM(1);
  else if (nh == 2) NYS_SPMM(2);
  else if (nh == 3) NYS_SPMM(3);
  else NYS_SPMM(4);
#undef NYS_SPMM
  hipLaunchKernelGGL(k_rm_to_cm, dim3(nb256(d * m)), dim3(256), 0, st, Yrm, d, m, c, Om, Y);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

}  // namespace nys

namespace nys {
// device bytes nys_sparse_create holds at once (CSC copy, s vector, column
// bins, and the transient per-block column counts)
// the three column lists (d triples each) and their lengths
size_t sparse_bins_bytes(int64_t d) { return sizeof(int4) * (size_t)(3 * d + 1); }

size_t sparse_handle_bytes(int64_t n, int64_t d, int64_t nnz) {
  const int64_t rpb = std::max<int64_t>(1, (n + kTBlocks - 1) / kTBlocks);
  const int64_t nblk = std::max<int64_t>(1, (n + rpb - 1) / rpb);
  return (sizeof(int) * (size_t)(d + 1 + 2 * nnz) + 256) +
         sizeof(double) * (size_t)std::max<int64_t>(n, 1) +
         sizeof(int) * ((size_t)nblk * d + 1) + sparse_bins_bytes(d) + 4 * 256;
}
}  // namespace nys

using namespace nys;

extern "C" {

nys_status nys_sparse_create(nys_ctx ctx, int64_t n, int64_t d, int64_t nnz, const int* rowptr,
                             const int* colidx, const float* val, nys_sparse* out) {
  if (ctx == nullptr || out == nullptr || n < 0 || d < 1 || nnz < 0 ||
      nnz > ((int64_t)1 << 31) - 1 || n > ((int64_t)1 << 31) - 2 ||
      d > ((int64_t)1 << 31) - 2 || rowptr == nullptr ||
      (nnz > 0 && (colidx == nullptr || val == nullptr)))
    return NYS_ERR_INVALID;
  *out = nullptr;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  hipStream_t st = ctx->stream;
  // rowptr must describe nnz entries: check its ends on the host
  int ends[2] = {0, 0};
  NYS_TRY_HIP(hipMemcpyAsync(&ends[0], rowptr, sizeof(int), hipMemcpyDeviceToHost, st));
  NYS_TRY_HIP(hipMemcpyAsync(&ends[1], rowptr + n, sizeof(int), hipMemcpyDeviceToHost, st));
  NYS_TRY_HIP(hipStreamSynchronize(st));
  if (ends[0] != 0 || ends[1] != nnz) return NYS_ERR_INVALID;
  nys_sparse_s* S = new (std::nothrow) nys_sparse_s();
  if (S == nullptr) return NYS_ERR_NOMEM;
  S->n = n;
  S->d = d;
  S->nnz = nnz;
  S->device = ctx->device;
  S->num_cu = ctx->num_cu;
  S->rowptr = rowptr;
  S->colidx = colidx;
  S->val = val;
  nys_status s = S->csc.reserve(sizeof(int) * (size_t)(d + 1 + 2 * nnz) + 256);
  if (s == NYS_OK) s = S->s.reserve(sizeof(double) * (size_t)std::max<int64_t>(n, 1));
  nys::DevBuf cnt;
  const int64_t rpb = std::max<int64_t>(1, (n + kTBlocks - 1) / kTBlocks);
  const int nblk = (int)std::max<int64_t>(1, (n + rpb - 1) / rpb);
  // counts of every row block, then one int flagging malformed input
  if (s == NYS_OK) s = cnt.reserve(sizeof(int) * ((size_t)nblk * d + 1));
  int* bad = cnt.ptr ? cnt.as<int>() + (size_t)nblk * d : nullptr;
  if (s == NYS_OK &&
      hipMemsetAsync(cnt.ptr, 0, sizeof(int) * ((size_t)nblk * d + 1), st) != hipSuccess)
    s = NYS_ERR_HIP;
  // validate before any entry is read through rowptr: rows non-decreasing
  // (with the ends checked above, every rowptr value lies in [0, nnz]); then
  // the counts, which flag column indices outside [0, d)
  auto check = [&]() {
    int hbad = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return NYS_ERR_HIP;
    return hbad ? NYS_ERR_INVALID : NYS_OK;
  };
  if (s == NYS_OK && n > 0) {
    hipLaunchKernelGGL(k_tr_check_rows, dim3(nb256(n)), dim3(256), 0, st, rowptr, n, bad);
    s = check();
  }
  if (s == NYS_OK && n > 0 && nnz > 0) {
    hipLaunchKernelGGL(k_tr_count, dim3(64, nblk), dim3(256), 0, st, rowptr, colidx, n, d, rpb,
                       cnt.as<int>(), bad);
    s = check();
  }
  if (s == NYS_OK) {
    hipLaunchKernelGGL(k_tr_colsum, dim3(nb256(d)), dim3(256), 0, st, cnt.as<int>(), d, nblk,
                       S->colptr());
    hipLaunchKernelGGL(k_tr_colscan, dim3(1), dim3(1024), 0, st, S->colptr(), d);
    hipLaunchKernelGGL(k_tr_addbase, dim3(nb256(d)), dim3(256), 0, st, cnt.as<int>(), d, nblk,
                       S->colptr());
    if (n > 0 && nnz > 0)
      hipLaunchKernelGGL(k_tr_fill, dim3(nblk), dim3(64), 0, st, rowptr, colidx, val, n, d, rpb,
                         cnt.as<int>(), S->rows(), S->cvals());
    if (hipGetLastError() != hipSuccess) s = NYS_ERR_HIP;
  }
  // column bins for the A^T pass: three lists of d slots and their lengths
  if (s == NYS_OK) s = S->bins.reserve(sparse_bins_bytes(d));
  if (s == NYS_OK) {
    int4* lists = S->bins.as<int4>();
    int* counts = reinterpret_cast<int*>(lists + 3 * d);
    int hc[3] = {0, 0, 0};
    if (hipMemsetAsync(counts, 0, sizeof(int) * 3, st) != hipSuccess) s = NYS_ERR_HIP;
    if (s == NYS_OK) {
      hipLaunchKernelGGL(k_bin_cols, dim3(1), dim3(1024), 0, st, S->colptr(), d, lists, counts);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(hc, counts, sizeof(int) * 3, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        s = NYS_ERR_HIP;
    }
    S->nshort = hc[0];
    S->nmed = hc[1];
    S->nlong = hc[2];
  }
  cnt.release();
  if (s != NYS_OK) {
    S->csc.release();
    S->s.release();
    S->bins.release();
    delete S;
    return s;
  }
  *out = S;
  return NYS_OK;
}

nys_status nys_sparse_destroy(nys_sparse S) {
  if (S == nullptr) return NYS_ERR_INVALID;
  (void)hipSetDevice(S->device);
  S->csc.release();
  S->s.release();
  S->bins.release();
  delete S;
  return NYS_OK;
}

}  // extern "C"
