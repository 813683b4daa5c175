// Sparse A (CSR) for the NysADMM hot path: the matvec pair A^T (D (A p)) as
// two streaming passes, a row pass over the CSR arrays (t = A p and the mode
// epilogue s = f(t)) and a column pass over a CSC copy (y = A^T s), and the
// sketch A^T (D (A Omega)) as two sparse-times-dense products.  Every sum is
// FP64 in a fixed order, so results are bitwise reproducible.  The CSC copy
// is built once by a deterministic counting transpose: rows are split into
// blocks, each block's column counts are prefix-summed across blocks, and
// each block places its entries row by row (within a row the columns are
// distinct, so no two lanes share a slot).  In the copy every column holds at
// least one entry (an empty column holds the entry (row 0, value 0)), and the
// row index of each column's first entry carries bit 31, so that a pass over
// the entries in storage order finds column j as the j-th flagged entry.
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
constexpr int kColFlag = (int)0x80000000u;   // first entry of a column in the CSC copy

// *bad = 1 unless rowptr is non-decreasing (its ends were checked on the host)
// and every row holds at most kMaxRowLen entries (the row pass addresses a
// row through a buffer resource of 4-byte elements with a 32-bit byte size)
constexpr int kMaxRowLen = 1 << 29;
__global__ __launch_bounds__(256) void k_tr_check_rows(const int* __restrict__ rowptr, int64_t n,
                                                       int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && (rowptr[i + 1] < rowptr[i] || rowptr[i + 1] - rowptr[i] > kMaxRowLen)) *bad = 1;
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
  colptr[j] = s > 0 ? s : 1;   // an empty column keeps one slot for its zero entry
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

// After the fill: flag each column's first entry; an empty column (the last
// block's slot counter still at the column start) gets the entry (row 0,
// value 0) in its one slot.
__global__ __launch_bounds__(256) void k_tr_pad(const int* __restrict__ cnt, int64_t d, int nblk,
                                                const int* __restrict__ colptr,
                                                int* __restrict__ rows, float* __restrict__ cval) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= d) return;
  const int pos = colptr[j];
  if (cnt[(int64_t)(nblk - 1) * d + j] == pos) {
    rows[pos] = kColFlag;
    cval[pos] = 0.0f;
  } else {
    rows[pos] |= kColFlag;
  }
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

// Stage x[0, h) (h <= 16 * 1024) into LDS by a 1024-thread workgroup with
// all sixteen loads of a thread in flight before the stores.
__device__ __forceinline__ void stage16(double* xl, const double* __restrict__ x, int h, int tid) {
  if (h <= 0) return;
  double t[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int i = tid + u * 1024;
    t[u] = x[i < h ? i : h - 1];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int i = tid + u * 1024;
    if (i < h) xl[i] = t[u];
  }
}

// Row pass: t_i = A_i p (one wavefront per row), s_i = f_mode(t_i) into s,
// per-workgroup sum of the mode's q term into qpart.  Persistent workgroups
// of 1024 threads (one per CU): the first kCsrHead entries of p are staged in
// LDS, where the gathers of the popular (low-index) columns of bag-of-words
// data land, and wavefront w of workgroup g takes rows g * 16 + w, then
// every 16 * gridDim.x rows on.  The next row's bounds are loaded before the
// current row's entries; a row is read in batches of 64 * kCsrCh entries
// (lane l takes entries k0 + c * 64 + l) through buffer resources bounded to
// the row (a lane past the row end reads index 0 and value 0), every index
// and value load of a batch issued before its gathers, then the LDS reads
// and, for columns past the head only, the global gathers.  Each lane adds its
// products in entry order; q terms are added in row order, the 16
// wavefronts' sums in wavefront order.
constexpr int kCsrT = 1024;
constexpr int kCsrHead = 16384;
constexpr int kCsrCh = 10;   // entries per lane per batch (rows up to 640 in one batch)
// word 3 of a raw buffer resource (32-bit elements, no swizzle) on gfx950
constexpr int kBufferWord3 = 0x00020000;
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
  stage16(pl, p, head, threadIdx.x);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double q = 0.0;
  const int64_t stride = (int64_t)gridDim.x * (kCsrT / 64);
  int64_t i = (int64_t)blockIdx.x * (kCsrT / 64) + wv;
  int rb = 0, re = 0;
  if (i < n && mode != kModeTOnly) {
    rb = rowptr[i];
    re = rowptr[i + 1];
  }
  for (; i < n; i += stride) {
    int nb = 0, ne = 0;
    if (i + stride < n && mode != kModeTOnly) {
      nb = rowptr[i + stride];
      ne = rowptr[i + stride + 1];
    }
    double acc = 0.0;
    // the row's index and value arrays as buffer resources of exactly its
    // length: a lane past the row end reads 0 (index 0, value 0), so the
    // loads need no clamp and take their offsets from the instruction
    const int rbu = __builtin_amdgcn_readfirstlane(rb);
    const int len = __builtin_amdgcn_readfirstlane(re) - rbu;
    const __amdgpu_buffer_rsrc_t rcol = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(col + rbu), (short)0, len * 4, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rval = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(val + rbu), (short)0, len * 4, kBufferWord3);
    for (int k0 = 0; k0 < len; k0 += 64 * kCsrCh) {
      int jj[kCsrCh];
      float vv[kCsrCh];
#pragma unroll
      for (int c = 0; c < kCsrCh; ++c) {
        const int off = (k0 + c * 64 + lane) * 4;
        jj[c] = __builtin_amdgcn_raw_buffer_load_b32(rcol, off, 0, 0);
        vv[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rval, off, 0, 0));
      }
      double lv[kCsrCh], gv[kCsrCh];
#pragma unroll
      for (int c = 0; c < kCsrCh; ++c) {
        lv[c] = pl[jj[c] < head ? jj[c] : 0];
        gv[c] = 0.0;
        if (jj[c] >= head) gv[c] = p[jj[c]];
      }
#pragma unroll
      for (int c = 0; c < kCsrCh; ++c)
        acc = fma((double)vv[c], (jj[c] < head ? lv[c] : 0.0) + gv[c], acc);
    }
    rb = nb;
    re = ne;
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

// DPP helpers of the column pass (FP64 as two 32-bit halves)
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffull), CTRL, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, RM, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffull), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// One step of a segmented inclusive scan over the 64 lanes: (v, fs) of the
// partner the DPP control selects (row_shr 1/2/4/8 within rows of 16, then
// row_bcast 15 and 31; (0, no flag) where there is none) is added in front
// unless a segment starts at or before this lane within the window.
template <int CTRL, int RM>
__device__ __forceinline__ void seg_step(double& v, int& fs) {
  const double pv = dpp_f64<CTRL, RM>(v);
  const int pf = __builtin_amdgcn_update_dpp(0, fs, CTRL, RM, 0xf, false);
  if (!fs) {
    v = pv + v;
    fs = pf;
  }
}

// Column pass: y_j = sum over column j of A_ij s_i over the CSC copy in
// storage order, with s staged in LDS (its first kCscHead entries).
// Workgroup g (1024 threads, one per CU) owns the entries [B_g, B_{g+1}), a
// column-aligned range chosen at handle creation so that the largest range
// is as small as possible; its wavefront w owns the w-th sixteenth of it
// (wstart[16 g + w] to wstart[16 g + w + 1]), whatever the column
// boundaries, and wbase[16 g + w] is the number of columns starting before
// its first entry, minus one.  A wavefront reads 64 EPL entries per round,
// EPL consecutive ones per lane (16-byte loads from the entry index rounded
// down to a multiple of 4; entries outside its range count as zero), sums them in
// order split at column starts, then combines the lanes by one segmented
// scan: a column that ends inside the wavefront's range is written by the
// lane holding its last entry's successor (or at the range end), its sum
// taken in entry order.  The partial sums of the columns that cross
// wavefront boundaries (the part before a wavefront's first column start,
// the part from its last one) are combined in wavefront order by one thread
// after a barrier.
constexpr int kCscHead = 16384;
constexpr int kCscEpl = 8;      // consecutive entries per lane per round
constexpr int kCscPad = 1024;   // entries past the end of the CSC arrays (a round's loads overrun)
template <int EPL>
__global__ __launch_bounds__(1024) void k_csc_pass(const int* __restrict__ rows,
                                                   const float* __restrict__ cval,
                                                   const int* __restrict__ wstart,
                                                   const int* __restrict__ wbase, int64_t n,
                                                   const double* __restrict__ s,
                                                   double* __restrict__ y,
                                                   const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  __shared__ double sl[kCscHead];
  __shared__ double hd[16], tl[16];
  __shared__ int hf[16], tord[16], topen[16];
  const int g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int hs = (int)(n < kCscHead ? n : kCscHead);
  const bool all_lds = n <= kCscHead;
  stage16(sl, s, hs, tid);
  __syncthreads();
  const int r0 = wstart[g * 16 + w], r1 = wstart[g * 16 + w + 1];
  const int wend = wstart[g * 16 + 16];
  const int base = wbase[g * 16 + w];
  double carry = 0.0;   // partial of the column open at the end of the last round
  int cnt = 0;          // column starts seen so far by the wavefront
  double head = 0.0;    // partial before the wavefront's first column start
  for (int a = r0 & ~3; a < r1; a += 64 * EPL) {
    const int e0 = a + EPL * lane;
    int rw[EPL];
    float cv[EPL];
#pragma unroll
    for (int h = 0; h < EPL / 4; ++h) {
      const int4 rr = *reinterpret_cast<const int4*>(rows + e0 + 4 * h);
      const float4 cc = *reinterpret_cast<const float4*>(cval + e0 + 4 * h);
      rw[4 * h] = rr.x; rw[4 * h + 1] = rr.y; rw[4 * h + 2] = rr.z; rw[4 * h + 3] = rr.w;
      cv[4 * h] = cc.x; cv[4 * h + 1] = cc.y; cv[4 * h + 2] = cc.z; cv[4 * h + 3] = cc.w;
    }
    double x[EPL];
    int fl = 0;   // bit j: entry e0 + j starts a column
#pragma unroll
    for (int j = 0; j < EPL; ++j) {
      const bool valid = e0 + j >= r0 && e0 + j < r1;
      const int row = valid ? (rw[j] & ~kColFlag) : 0;
      double sv;
      if (all_lds) {
        sv = sl[row < hs ? row : 0];
      } else {
        const double lv = sl[row < kCscHead ? row : 0];
        const double gv = s[row < kCscHead ? 0 : row];
        sv = row < kCscHead ? lv : gv;
      }
      x[j] = (valid && row < n) ? (double)cv[j] * sv : 0.0;
      if (valid && (rw[j] & kColFlag)) fl |= 1 << j;
    }
    const int nf = __popc(fl);
    const unsigned long long fm = __ballot(fl != 0);
    // column starts in the lanes below (exclusive prefix over the wavefront)
    int pre = nf;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(pre, off, 64);
      if (lane >= off) pre += o;
    }
    const int fb = cnt + pre - nf;
    // in-lane pass: columns that start and end inside the lane are written
    double hsum = 0.0, run = 0.0;
    int seen = 0;
#pragma unroll
    for (int j = 0; j < EPL; ++j) {
      if (fl & (1 << j)) {
        if (seen == 0) hsum = run;
        else y[base + fb + seen] = run;
        run = 0.0;
        ++seen;
      }
      run += x[j];
    }
    if (!fl) hsum = run;
    double v = fl ? run : hsum;   // from the lane's last column start, or the whole lane
    int fs = fl ? 1 : 0;
    seg_step<0x111, 0xf>(v, fs);
    seg_step<0x112, 0xf>(v, fs);
    seg_step<0x114, 0xf>(v, fs);
    seg_step<0x118, 0xf>(v, fs);
    seg_step<0x142, 0xa>(v, fs);
    seg_step<0x143, 0xc>(v, fs);
    // the column that ends just before this lane's first column start
    const double vprev = dpp_f64<0x138, 0xf>(v);   // wave_shr:1
    const int fsprev = __builtin_amdgcn_update_dpp(0, fs, 0x138, 0xf, 0xf, false);
    const double prev_total = (fsprev ? vprev : carry + vprev) + hsum;
    if (fl && fb > 0) y[base + fb] = prev_total;
    if (cnt == 0 && fm != 0ull) head = readlane_f64(prev_total, __ffsll((long long)fm) - 1);
    const double v63 = readlane_f64(v, 63);
    carry = fm ? v63 : carry + v63;
    cnt = __shfl(fb + nf, 63, 64);
  }
  if (lane == 0) {
    hf[w] = cnt > 0;
    hd[w] = cnt > 0 ? head : carry;
    tl[w] = carry;
    tord[w] = base + cnt;
    topen[w] = cnt > 0 && r1 < wend;
    if (cnt > 0 && r1 >= wend && r1 > r0) y[base + cnt] = carry;
  }
  __syncthreads();
  if (tid == 0) {
    bool open = false;
    double acc = 0.0;
    int ord = -1;
    for (int v = 0; v < 16; ++v) {
      if (!hf[v]) {
        acc += hd[v];
        continue;
      }
      if (open) y[ord] = acc + hd[v];
      open = topen[v] != 0;
      acc = tl[v];
      ord = tord[v];
    }
    if (open) y[ord] = acc;
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
      const double* b = B + (int64_t)(idx[k + u] & ~kColFlag) * m;
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
    const double* b = B + (int64_t)(idx[k] & ~kColFlag) * m;
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
  hipLaunchKernelGGL(k_csc_pass<kCscEpl>, dim3((unsigned)S->cgrid), dim3(1024), 0, st, S->rows(),
                     S->cvals(), S->wstart(), S->wbase(), S->n, s, ypart, done);
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
// CSC slots (rows and values each): every entry, one per empty column, and
// the overrun of the column pass's 16-byte loads; a multiple of 4
static int64_t sparse_csc_cap(int64_t d, int64_t nnz) { return (nnz + d + kCscPad + 3) / 4 * 4; }

// device bytes nys_sparse_create holds at once (CSC copy, s vector, the
// column-pass split, and the transient per-block column counts)
size_t sparse_handle_bytes(int64_t n, int64_t d, int64_t nnz) {
  const int64_t rpb = std::max<int64_t>(1, (n + kTBlocks - 1) / kTBlocks);
  const int64_t nblk = std::max<int64_t>(1, (n + rpb - 1) / rpb);
  const int64_t roff = (d + 1 + 3) / 4 * 4;
  return (sizeof(int) * (size_t)(roff + 2 * sparse_csc_cap(d, nnz)) + 256) +
         sizeof(double) * (size_t)std::max<int64_t>(n, 1) +
         sizeof(int) * ((size_t)nblk * d + 1) + sizeof(int) * (2 * (16 * 1024 + 1)) + 4 * 256;
}

// Column-aligned split of the nnzc CSC entries into at most G ranges with
// the largest range as small as possible (binary search on the capacity T;
// for a given T, ranges are cut greedily at the last column start within
// T); then each range into 16 wavefront ranges of equal size.  cp is the
// CSC colptr (d + 1 entries, strictly increasing: no column is empty).
static void sparse_split(const std::vector<int>& cp, int G, std::vector<int>& wstart,
                         std::vector<int>& wbase) {
  const int64_t d = (int64_t)cp.size() - 1;
  const int64_t nnzc = cp[d];
  auto cut = [&](int64_t T, std::vector<int64_t>* out) {
    int64_t b = 0;
    int parts = 0;
    while (b < nnzc) {
      if (parts == G) return false;
      const auto it = std::upper_bound(cp.begin(), cp.end(), (int64_t)std::min<int64_t>(b + T, nnzc));
      const int64_t nb = *(it - 1);
      if (nb <= b) return false;   // a column longer than T
      if (out != nullptr) out->push_back(nb);
      b = nb;
      ++parts;
    }
    return true;
  };
  int64_t longest = 0;
  for (int64_t j = 0; j < d; ++j) longest = std::max<int64_t>(longest, cp[j + 1] - cp[j]);
  int64_t lo = std::max<int64_t>(longest, (nnzc + G - 1) / G), hi = std::max<int64_t>(nnzc, 1);
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (cut(mid, nullptr)) hi = mid;
    else lo = mid + 1;
  }
  std::vector<int64_t> B{0};
  cut(lo, &B);
  while ((int)B.size() < G + 1) B.push_back(nnzc);
  wstart.assign((size_t)16 * G + 1, 0);
  wbase.assign((size_t)16 * G + 1, 0);
  for (int g = 0; g < G; ++g) {
    const int64_t L = B[g + 1] - B[g];
    for (int w = 0; w < 16; ++w) wstart[(size_t)16 * g + w] = (int)(B[g] + L * w / 16);
  }
  wstart[(size_t)16 * G] = (int)nnzc;
  for (size_t i = 0; i < wstart.size(); ++i)
    wbase[i] = (int)(std::lower_bound(cp.begin(), cp.begin() + d, wstart[i]) - cp.begin()) - 1;
}
}  // namespace nys

using namespace nys;

extern "C" {

nys_status nys_sparse_create(nys_ctx ctx, int64_t n, int64_t d, int64_t nnz, const int* rowptr,
                             const int* colidx, const float* val, nys_sparse* out) {
  if (ctx == nullptr || out == nullptr || n < 0 || d < 1 || nnz < 0 ||
      n > ((int64_t)1 << 31) - 2 || d > ((int64_t)1 << 31) - 2 ||
      sparse_csc_cap(d, nnz) > ((int64_t)1 << 31) - 1 || rowptr == nullptr ||
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
  S->cap = sparse_csc_cap(d, nnz);
  nys_status s = S->csc.reserve(sizeof(int) * (size_t)(S->row_off() + 2 * S->cap) + 256);
  // row indices and values start zeroed (the slots past colptr[d] stay so)
  if (s == NYS_OK && hipMemsetAsync(S->rows(), 0, sizeof(int) * (size_t)(2 * S->cap), st) !=
                         hipSuccess)
    s = NYS_ERR_HIP;
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
    hipLaunchKernelGGL(k_tr_pad, dim3(nb256(d)), dim3(256), 0, st, cnt.as<int>(), d, nblk,
                       S->colptr(), S->rows(), S->cvals());
    if (hipGetLastError() != hipSuccess) s = NYS_ERR_HIP;
  }
  // the column pass's split, from the CSC colptr on the host
  if (s == NYS_OK) {
    std::vector<int> cp((size_t)d + 1);
    if (hipMemcpyAsync(cp.data(), S->colptr(), sizeof(int) * (size_t)(d + 1),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      s = NYS_ERR_HIP;
    if (s == NYS_OK) {
      S->nnzc = cp[(size_t)d];
      S->cgrid = std::max(1, S->num_cu);
      std::vector<int> ws, wb;
      sparse_split(cp, S->cgrid, ws, wb);
      s = S->part.reserve(sizeof(int) * (ws.size() + wb.size()));
      if (s == NYS_OK &&
          (hipMemcpyAsync(S->part.as<int>(), ws.data(), sizeof(int) * ws.size(),
                          hipMemcpyHostToDevice, st) != hipSuccess ||
           hipMemcpyAsync(S->part.as<int>() + ws.size(), wb.data(), sizeof(int) * wb.size(),
                          hipMemcpyHostToDevice, st) != hipSuccess ||
           hipStreamSynchronize(st) != hipSuccess))
        s = NYS_ERR_HIP;
    }
  }
  cnt.release();
  if (s != NYS_OK) {
    S->csc.release();
    S->s.release();
    S->part.release();
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
  S->part.release();
  delete S;
  return NYS_OK;
}

}  // extern "C"
