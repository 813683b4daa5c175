// FP64 kernels of the Nystrom core (Algorithm RandNysAppx after the sketch):
// tiled FP64 GEMM, in-place upper Cholesky, upper triangular inverse, power
// iteration for ||Y||_2, two-sided block Jacobi eigensolver, eigenpair sort.
// All of them are small (r <= 1024) and latency bound; they run once per
// sketch, never inside the PCG loop.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace nys {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ------------------------------------------------------------ FP64 GEMM
// C(m,n) = alpha sum_k A(m,k) w_k B(k,n) + beta C(m,n), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn], C(m,n) = C[m*scm + n*scn], w_k = wk[k] or 1.
// FP64 matrix cores (16x16x4 FP64 MFMA, FP32 operands widened on load): a
// workgroup computes a 64 x 64 tile, wavefront w the 32 x 32 quarter
// (w >> 1, w & 1) as 2 x 2 MFMA blocks, K in steps of 16 through LDS with the
// next step's operands loaded into registers while the current step's MFMAs
// run.  With gridDim.z > 1 each z handles a K chunk and writes the raw sum to
// C + z*split_stride (layout m*N + n); k_split_reduce finishes.
typedef double d4 __attribute__((ext_vector_type(4)));

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_gemm64(int M, int N, int K, int kchunk,
                                               const TA* __restrict__ A, int64_t sam, int64_t sak,
                                               const TB* __restrict__ B, int64_t sbk, int64_t sbn,
                                               double* __restrict__ C, int64_t scm, int64_t scn,
                                               int64_t split_stride, double alpha, double beta,
                                               const double* __restrict__ wk) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = 32 * (wv >> 1), wn = 32 * (wv & 1);
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (d4)0.0;
  // consecutive threads take consecutive elements along whichever index has
  // unit stride (k for the Gram-type products X^T Y of column-major X, Y;
  // m or n otherwise), so every load instruction reads whole cache lines
  const bool ak = (sak == 1 && sam != 1), bk = (sbk == 1 && sbn != 1);
  double an[4], bn[4];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + e * 256;
      const int mm = ak ? (idx >> 4) : (idx & 63), ka = ak ? (idx & 15) : (idx >> 6);
      const int nn = bk ? (idx >> 4) : (idx & 63), kb2 = bk ? (idx & 15) : (idx >> 6);
      const int gka = k0 + ka, gkb = k0 + kb2;
      an[e] = (m0 + mm < M && gka < ke) ? (double)A[(int64_t)(m0 + mm) * sam + (int64_t)gka * sak]
                                        : 0.0;
      bn[e] = (n0 + nn < N && gkb < ke)
                  ? (double)B[(int64_t)gkb * sbk + (int64_t)(n0 + nn) * sbn] * (wk ? wk[gkb] : 1.0)
                  : 0.0;
    }
  };
  auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + e * 256;
      const int mm = ak ? (idx >> 4) : (idx & 63), ka = ak ? (idx & 15) : (idx >> 6);
      const int nn = bk ? (idx >> 4) : (idx & 63), kb2 = bk ? (idx & 15) : (idx >> 6);
      As[ka][mm] = an[e];
      Bs[kb2][nn] = bn[e];
    }
  };
  const int fi = lane & 15, fk = lane >> 4;   // MFMA operand: row/column fi, k fk
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += 16) {
    store();
    __syncthreads();
    if (k0 + 16 < ke) load(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + fk][wm + 16 * i + fi];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + fk][wn + 16 * j + fi];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // FP64 16x16 result layout: lane (fk, fi) holds rows fk + 4 v of column fi,
  // so acc[i][j][v] = C(m0 + wm + 16 i + fk + 4 v, n0 + wn + 16 j + fi)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm + 16 * i + fk + 4 * v, gn = n0 + wn + 16 * j + fi;
        if (gm < M && gn < N) {
          if (gridDim.z > 1) {
            C[blockIdx.z * split_stride + (int64_t)gm * N + gn] = acc[i][j][v];
          } else {
            double* c = C + (int64_t)gm * scm + (int64_t)gn * scn;
            *c = (beta == 0.0) ? alpha * acc[i][j][v] : fma(alpha, acc[i][j][v], beta * *c);
          }
        }
      }
}

// C = alpha * sum_z ws[z] + beta C over the S split-K partials.  A workgroup
// covers 16 outputs with 16 groups of lanes; group g adds the partials
// z = g, g + 16, ... with eight loads in flight, the groups are combined in
// LDS in a fixed order (for few outputs S is large: up to 1024).
constexpr int kSrOut = 16;
__global__ __launch_bounds__(256) void k_split_reduce(int M, int N, int S,
                                                      const double* __restrict__ ws,
                                                      double* __restrict__ C, int64_t scm,
                                                      int64_t scn, double alpha, double beta) {
  constexpr int G = 256 / kSrOut;
  __shared__ double part[G][kSrOut];
  const int o = threadIdx.x % kSrOut, g = threadIdx.x / kSrOut;
  const int64_t idx = (int64_t)blockIdx.x * kSrOut + o;
  const int64_t tot = (int64_t)M * N;
  double a[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) a[t] = 0.0;
  if (idx < tot) {
    int z = g;
    for (; z + 7 * G < S; z += 8 * G) {
#pragma unroll
      for (int t = 0; t < 8; ++t) a[t] += ws[(int64_t)(z + t * G) * tot + idx];
    }
    for (; z < S; z += G) a[0] += ws[(int64_t)z * tot + idx];
  }
  part[g][o] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  if (g == 0 && idx < tot) {
    double s = 0.0;
#pragma unroll
    for (int h = 0; h < G; ++h) s += part[h][o];
    const int m = (int)(idx / N), n = (int)(idx % N);
    double* c = C + (int64_t)m * scm + (int64_t)n * scn;
    *c = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * *c);
  }
}

// 1/sqrt(x) and 1/x for positive normal x: the hardware estimate refined by
// two Newton steps (y <- y (3 - x y^2) / 2, y <- y (2 - x y)), within a few
// ulp: the rotation needs no correctly rounded result, and this chain is a
// fraction of the length of the library's sqrt and division
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// pivot of a Cholesky step: sqrt(d) and 1/sqrt(d) (d > 0); the Newton-refined
// estimate for normal d, the library's square root and division otherwise
__device__ __forceinline__ void chol_pivot(double dii, double* piv, double* rinv) {
  if (dii > 1e-280 && dii < 1e280) {
    *rinv = rsq_nr(dii);
    *piv = dii * *rinv;
  } else {
    *piv = sqrt(fabs(dii));
    *rinv = 1.0 / *piv;
  }
}

// P <- C^-T P for the upper-triangular b x b block C (rdiag = 1 / diag(C)),
// P b x nc, right-looking: at step i every thread of column c forms
// x = P[i][c] / C[i][i] and its row group (NT / WC groups) takes x C[i][j]
// off the rows j > i it owns; one barrier per step.  The finished row i is
// stored one step later (nobody reads it then), by row group 0.
template <int CB, int WC, int NT>
__device__ __forceinline__ void right_looking_solve(double (&C)[CB][CB + 1],
                                                    double (&P)[CB][WC + 1],
                                                    const double* rdiag, int b, int nc, int tid) {
  constexpr int NG = NT / WC;
  const int c = tid % WC, jr = tid / WC;
  double prev = 0.0;
  for (int i = 0; i < b; ++i) {
    double x = 0.0;
    if (c < nc) {
      x = P[i][c] * rdiag[i];
      if (jr == 0 && i > 0) P[i - 1][c] = prev;
      for (int j = i + 1 + jr; j < b; j += NG) P[j][c] = fma(-C[i][j], x, P[j][c]);
    }
    prev = x;
    __syncthreads();
  }
  if (c < nc && jr == 0 && b > 0) P[b - 1][c] = prev;
}

// Order the wavefront's own LDS accesses around this point (a barrier for a
// single wavefront: its LDS operations complete in issue order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x from lane l of the wavefront (l wave-uniform)
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// e-th tile (I, J), I <= J, of the upper triangle of an n x n grid of tiles,
// row-major
__device__ __forceinline__ void upper_tile(int e, int n, int* I, int* J) {
  int a = 0;
  while (e >= n - a) {
    e -= n - a;
    ++a;
  }
  *I = a;
  *J = a + e;
}

// Upper Cholesky factor C (C^T C = M) in place, row-major with leading
// dimension ld; only the upper triangle of M is read, and the strict lower
// triangle receives C^T (M[j][i] = C[i][j]), so that column l of C is
// contiguous in row l.  One workgroup of 512 threads, right-looking by
// blocks of kCB rows, four barriers per block: the diagonal block is factored
// in the registers of the first wavefront (lane j holds column j; the entries
// C[i][p] of the rank-1 updates are read from their lanes), the block row of
// C is formed by forward substitution against it (one thread per column, all
// columns at once), and the trailing upper triangle takes the rank-kCB update
// as 16 x 16 tiles on the FP64 matrix cores.  *fail = 1 on a non-positive or
// non-finite pivot.
constexpr int kCB = 32;
constexpr int kCholOneWg = 256;
constexpr int kCholT = 512;   // threads of k_chol_upper

__global__ __launch_bounds__(kCholT) void k_chol_upper(double* __restrict__ M, int r, int ld,
                                                     int* __restrict__ fail) {
  __shared__ double C[kCB][kCB + 1];
  __shared__ double P[kCB][kCholOneWg + 1];
  __shared__ double rdiag[kCB];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) bad = 0;
  for (int kb = 0; kb < r; kb += kCB) {
    const int b = (r - kb < kCB) ? r - kb : kCB;
    const int nrest = r - kb - b;
    for (int e = tid; e < b * b; e += kCholT) {
      const int i = e / b, j = e % b;
      C[i][j] = (j >= i) ? M[(int64_t)(kb + i) * ld + kb + j] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      // lane j (mod 32) holds column j, padded to 32 x 32 with the identity
      // beyond b; entries below the diagonal are carried but never read
      const int j = lane & (kCB - 1);
      double col[kCB];
#pragma unroll
      for (int p = 0; p < kCB; ++p)
        col[p] = (p < b && j < b && p <= j) ? C[p][j] : (p == j ? 1.0 : 0.0);
      bool ok = true;
      double rj = 1.0;
#pragma unroll
      for (int i = 0; i < kCB; ++i) {
        const double dii = readlane_f64(col[i], i);
        ok = ok && (dii > 0.0) && isfinite(dii);
        double piv, rinv;
        chol_pivot(dii, &piv, &rinv);
        col[i] = (j == i) ? piv : col[i] * rinv;
        if (j == i) rj = rinv;
#pragma unroll
        for (int p = 0; p < kCB; ++p)
          if (p > i) col[p] = fma(-readlane_f64(col[i], p), col[i], col[p]);
      }
      if (lane < b) {
#pragma unroll
        for (int p = 0; p < kCB; ++p)
          if (p <= j) C[p][j] = col[p];
        rdiag[j] = rj;
      }
      if (!ok && lane == 0) bad = 1;
    }
    __syncthreads();
    if (bad) break;
    for (int e = tid; e < b * b; e += kCholT) {
      const int i = e / b, j = e % b;
      if (j >= i) {
        M[(int64_t)(kb + i) * ld + kb + j] = C[i][j];
        if (j > i) M[(int64_t)(kb + j) * ld + kb + i] = C[i][j];
      }
    }
    // block row X = C_kk^-T M[kb:kb+b, kb+b:]: thread c owns column c
    if (tid < nrest) {
      const int c = tid;
      double x[kCB];
#pragma unroll
      for (int i = 0; i < kCB; ++i) x[i] = (i < b) ? M[(int64_t)(kb + i) * ld + kb + b + c] : 0.0;
#pragma unroll
      for (int i = 0; i < kCB; ++i) {
        if (i < b) {
          double s = x[i];
#pragma unroll
          for (int l = 0; l < i; ++l) s = fma(-C[l][i], x[l], s);
          x[i] = s * rdiag[i];
          P[i][c] = x[i];
          M[(int64_t)(kb + i) * ld + kb + b + c] = x[i];
          M[(int64_t)(kb + b + c) * ld + kb + i] = x[i];
        }
      }
    }
    __syncthreads();
    // trailing upper triangle: M[p][q] -= sum_i X[i][p] X[i][q], p <= q, by
    // 16 x 16 tiles (FP64 MFMA 16x16x4: lane (fk, fi) supplies X[k0 + fk][.. + fi]
    // of both operands and holds rows fk + 4 v of column fi).  nrest > 0
    // implies b = kCB.  Columns of P at or beyond nrest hold stale values;
    // they only reach outputs outside the trailing block, which are not
    // written.  Diagonal tiles also write their lower half, which the lower
    // triangle's C^T entries of later blocks overwrite.
    if (nrest > 0) {
      const int nt = (nrest + 15) >> 4;
      const int fi = lane & 15, fk = lane >> 4;
      for (int u = wv; u < nt * (nt + 1) / 2; u += kCholT / 64) {
        int I, J;
        upper_tile(u, nt, &I, &J);
        d4 acc = (d4)0.0;
#pragma unroll
        for (int k0 = 0; k0 < kCB; k0 += 4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(P[k0 + fk][16 * I + fi],
                                                     P[k0 + fk][16 * J + fi], acc, 0, 0, 0);
        const int qq = 16 * J + fi;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int pp = 16 * I + fk + 4 * v;
          if (pp < nrest && qq < nrest) {
            double* m = M + (int64_t)(kb + b + pp) * ld + kb + b + qq;
            *m -= acc[v];
          }
        }
      }
    }
    __syncthreads();
  }
  if (bad && tid == 0) *fail = 1;
}

// ---- blocked Cholesky for r > kCholOneWg (same contract as k_chol_upper)
constexpr int kLB = 64;

// Diagonal block M[kb:kb+b, kb:kb+b] <- its upper Cholesky factor (LDS).
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ M, int ld, int kb, int b,
                                                   int* __restrict__ fail) {
  __shared__ double C[kLB][kLB + 1];
  __shared__ double rowv[kLB];
  __shared__ int bad;
  if (*fail) return;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    C[i][j] = (j >= i) ? M[(int64_t)(kb + i) * ld + kb + j] : 0.0;
  }
  __syncthreads();
  // thread column q = tid % kLB, rows p = tid / kLB + 4 k of the b x b block
  const int tq = tid % kLB;
  for (int i = 0; i < b; ++i) {
    if (tid >= i && tid < b) {
      const double dii = C[i][i];
      if (tid == i && (!(dii > 0.0) || !isfinite(dii))) bad = 1;
      double piv, rinv;
      chol_pivot(dii, &piv, &rinv);
      rowv[tid] = (tid == i) ? piv : C[i][tid] * rinv;
    }
    __syncthreads();
    if (bad) break;
    if (tid >= i && tid < b) C[i][tid] = rowv[tid];
    if (tq < b) {
      const double rq = rowv[tq];
      for (int pp = tid / kLB; pp <= tq; pp += 256 / kLB)
        if (pp > i) C[pp][tq] -= rowv[pp] * rq;
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) *fail = 1;
    return;
  }
  for (int e = tid; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    if (j >= i) M[(int64_t)(kb + i) * ld + kb + j] = C[i][j];
  }
}

// Block row X = C_kk^-T M[kb:kb+b, kb+b:]: a workgroup per kLB columns, one
// column per thread, forward substitution against C_kk in LDS.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ M, int ld, int kb, int b,
                                                    int nrest, int* __restrict__ fail) {
  __shared__ double C[kLB][kLB + 1];
  __shared__ double P[kLB][kLB + 1];
  __shared__ double rdiag[kLB];
  if (*fail) return;
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * kLB;
  const int nc = min(kLB, nrest - c0);
  for (int e = tid; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    C[i][j] = (j >= i) ? M[(int64_t)(kb + i) * ld + kb + j] : 0.0;
  }
  for (int e = tid; e < b * nc; e += 256) {
    const int i = e / nc, jj = e % nc;
    P[i][jj] = M[(int64_t)(kb + i) * ld + kb + b + c0 + jj];
  }
  __syncthreads();
  if (tid < b) rdiag[tid] = 1.0 / C[tid][tid];
  __syncthreads();
  right_looking_solve<kLB, kLB, 256>(C, P, rdiag, b, nc, tid);
  __syncthreads();
  for (int e = tid; e < b * nc; e += 256) {
    const int i = e / nc, jj = e % nc;
    M[(int64_t)(kb + i) * ld + kb + b + c0 + jj] = P[i][jj];
  }
}

// Trailing update M[p][q] -= sum_i X[i][p] X[i][q] on the upper triangle:
// one workgroup per kLB x kLB tile (ti <= tj), X's two column blocks in LDS.
__global__ __launch_bounds__(256) void k_chol_trail(double* __restrict__ M, int ld, int kb, int b,
                                                    int nrest, int tc, int* __restrict__ fail) {
  __shared__ double Xp[kLB][kLB + 1];
  __shared__ double Xq[kLB][kLB + 1];
  if (*fail) return;
  // tile index -> (ti, tj) with ti <= tj, row-major over the upper triangle
  int t = blockIdx.x, ti = 0;
  while (t >= tc - ti) {
    t -= tc - ti;
    ++ti;
  }
  const int tj = ti + t;
  const int tid = threadIdx.x;
  const int p0 = ti * kLB, q0 = tj * kLB;
  const int np = min(kLB, nrest - p0), nq = min(kLB, nrest - q0);
  const int64_t c = kb + b;   // first trailing index
  for (int e = tid; e < b * kLB; e += 256) {
    const int i = e / kLB, jj = e % kLB;
    Xp[i][jj] = jj < np ? M[(int64_t)(kb + i) * ld + c + p0 + jj] : 0.0;
    Xq[i][jj] = jj < nq ? M[(int64_t)(kb + i) * ld + c + q0 + jj] : 0.0;
  }
  __syncthreads();
  // 16 outputs per thread: rows pr = tid / 16 + 16 a, columns qc = tid % 16 + 16 e
  const int pr0 = tid >> 4, qc0 = tid & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int pp = pr0 + 16 * a;
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
      const int qq = qc0 + 16 * e2;
      if (pp >= np || qq >= nq) continue;
      if (ti == tj && qq < pp) continue;   // upper triangle only
      double sacc = 0.0;
      for (int i = 0; i < b; ++i) sacc = fma(Xp[i][pp], Xq[i][qq], sacc);
      M[(c + p0 + pp) * ld + c + q0 + qq] -= sacc;
    }
  }
}

// strict lower triangle <- the transpose of the upper factor
__global__ void k_chol_mirror_lower(double* __restrict__ M, int r, int ld,
                                    const int* __restrict__ fail) {
  if (*fail) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e / r), j = (int)(e % r);
  if (i > j) M[(int64_t)i * ld + j] = M[(int64_t)j * ld + i];
}

// Z = C^-1 for the upper triangular C (r x r, row-major, ld) in the layout
// chol_upper leaves (strict lower triangle = C^T, so column l of C is row l).
// One wavefront per column k, right-looking back substitution: the partial
// sums s_i = sum_{l' > l} C(i, l') z_l' of the rows i < l still open stay in
// registers (row i in lane i % 64, slot i / 64).  At step l (k down to 0) the
// owner of row l forms z_l = ([l == k] - s_l) / C(l, l), every lane reads it
// (readlane), and the open rows add C(i, l) z_l; column l of C is fetched D
// steps ahead into a register ring.
template <int NS, int D>
__global__ __launch_bounds__(256) void k_trinv_upper(const double* __restrict__ Cm, int r, int ld,
                                                     double* __restrict__ Z, int ldz) {
  __shared__ double rd[64 * NS];
  for (int i = threadIdx.x; i < r; i += 256) rd[i] = 1.0 / Cm[(int64_t)i * ld + i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 4 + wv;
  if (k >= r) return;
  for (int i = k + 1 + lane; i < r; i += 64) Z[(int64_t)i * ldz + k] = 0.0;
  double s[NS], ring[D][NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) s[j] = 0.0;
  auto fetch = [&](int l, double (&dst)[NS]) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int i = lane + 64 * j;
      dst[j] = (l > 0 && i < l) ? Cm[(int64_t)l * ld + i] : 0.0;
    }
  };
#pragma unroll
  for (int u = 0; u < D; ++u) fetch(k - u, ring[u]);
  for (int l0 = k; l0 >= 0; l0 -= D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int l = l0 - u;
      if (l < 0) break;
      const int js = l >> 6, ol = l & 63;
      double t = s[0];
#pragma unroll
      for (int j = 1; j < NS; ++j) t = (js == j) ? s[j] : t;
      const int lo = __builtin_amdgcn_readlane(__double2loint(t), ol);
      const int hi = __builtin_amdgcn_readlane(__double2hiint(t), ol);
      const double z = ((l == k ? 1.0 : 0.0) - __hiloint2double(hi, lo)) * rd[l];
      if (lane == 0) Z[(int64_t)l * ldz + k] = z;
#pragma unroll
      for (int j = 0; j < NS; ++j) s[j] = fma(ring[u][j], z, s[j]);
      fetch(l - D, ring[u]);
    }
  }
}

// Largest eigenvalue of the symmetric psd r x r matrix G by power iteration
// (x <- G x / ||G x||), Rayleigh quotient written to *out (the iterations
// taken to out[1]).  y = G x is summed by np groups of threads, each over a
// contiguous range of k (np = 1024 / r rounded up to 64), the group sums
// added in a fixed order.
__global__ __launch_bounds__(1024) void k_power_iter(const double* __restrict__ G, int r, int ld,
                                                     int iters, double* __restrict__ out) {
  __shared__ double x[1024];
  __shared__ double part[1024];
  __shared__ double red[16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int r64 = (r + 63) / 64 * 64;
  const int np = 1024 / r64;   // 1 .. 16
  const int i = t % r64, g = t / r64;
  const int kper = (r + np - 1) / np;
  const int kb = g * kper, ke = min(r, kb + kper);
  if (t < r) x[t] = 1.0 / sqrt((double)r) * (1.0 + 1e-3 * (double)(t % 7));
  __syncthreads();
  double lam = 0.0;
  int stable = 0, it = 0;
  for (; it <= iters; ++it) {
    if (g < np && i < r) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
      int k = kb;
      for (; k + 3 < ke; k += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = fma(G[(int64_t)(k + u) * ld + i], x[k + u], a[u]);
      }
      for (; k < ke; ++k) a[0] = fma(G[(int64_t)k * ld + i], x[k], a[0]);
      part[t] = (a[0] + a[1]) + (a[2] + a[3]);
    }
    __syncthreads();
    double y = 0.0;
    if (t < r)
      for (int h = 0; h < np; ++h) y += part[h * r64 + t];
    // Rayleigh quotient x^T G x (x normalised) and ||y||^2
    double xy = (t < r) ? x[t] * y : 0.0, yy = y * y;
    xy = wave_sum(xy);
    yy = wave_sum(yy);
    if (lane == 0) red[wv] = xy;
    __syncthreads();
    double sxy = 0.0;
    for (int w = 0; w < 16; ++w) sxy += red[w];
    __syncthreads();
    if (lane == 0) red[wv] = yy;
    __syncthreads();
    double syy = 0.0;
    for (int w = 0; w < 16; ++w) syy += red[w];
    const double lam_prev = lam;
    lam = sxy;
    if (syy <= 0.0 || !isfinite(syy)) {
      lam = 0.0;
      break;
    }
    // only the binade of ||Y||_2 enters the shift: stop once the Rayleigh
    // quotient has settled to 1e-13 for 4 consecutive iterations
    stable = (it > 0 && fabs(lam - lam_prev) <= 1e-13 * lam) ? stable + 1 : 0;
    if (stable >= 4) break;
    if (t < r) x[t] = y / sqrt(syy);
    __syncthreads();
  }
  if (t == 0) {
    out[0] = lam;
    out[1] = (double)it;
  }
}

// ------------------------------------------------------------ Jacobi
// Two-sided block Jacobi on the symmetric R x R matrix H (R a multiple of 32,
// row-major), blocks of 16 indices, block pairs chosen round-robin (nb - 1
// rounds of nb / 2 disjoint pairs per sweep).  Within a visit of the pair
// block (a, b) only the pairs (i in a, j in b) are rotated, 16 at a time:
// step s pairs index k of a with index (k + s) mod 16 of b, so every cross
// pair is rotated once per visit.  The pairs inside a block are rotated in the
// first round of each sweep (a cyclic round-robin over the 16 indices of each
// block of the pair, before the cross steps).  Every off-diagonal pair is
// therefore rotated once per sweep, in about R sequential steps, half of what
// a full cyclic sweep of each 32 x 32 pair block per round would take.
//
// A round is one launch: nb / 2 workgroups solve the pair blocks of round t
// (forming each 32 x 32 pair block from H_{t-1} and the rotations Q^{t-1} of
// the previous round, so that they need not wait for the full update), and
// the remaining workgroups form H_t = Q^{t-1 T} H_{t-1} Q^{t-1} tile by tile
// and accumulate V <- V Q^{t-1}.  The last round's update is a launch of its
// own, followed by the convergence check.
constexpr int kJB = 16;        // block size
constexpr int kJP = 2 * kJB;   // pair block size
constexpr int kJT = 256;       // threads of every Jacobi workgroup
constexpr int kJE = kJP * kJP / kJT;   // tile elements per thread
constexpr int kJU = kJB * (kJB + 1) / 2;   // upper 2x2 blocks of a step

// Round-robin pairing of nb blocks (nb even): round t, pair k -> (a, b).
__device__ __forceinline__ void rr_pair(int nb, int t, int k, int* a, int* b) {
  auto pos = [&](int p) { return p == 0 ? 0 : ((p - 1 + t) % (nb - 1)) + 1; };
  *a = pos(k);
  *b = pos(nb - 1 - k);
}

// The pair k of round t that holds block x, and whether x is its second member.
__device__ __forceinline__ void rr_locate(int nb, int t, int x, int* k, int* h) {
  int p = 0;
  if (x != 0) p = ((x - 1 - t) % (nb - 1) + (nb - 1)) % (nb - 1) + 1;
  if (p < nb / 2) {
    *k = p;
    *h = 0;
  } else {
    *k = nb - 1 - p;
    *h = 1;
  }
}

// counters[s]: pair blocks that rotated in sweep s; counters[64 + s]: 1 if
// the matrix after sweep s still fails the rotation criterion somewhere.
// Sweep s (with its check) is skipped when sweep s - 1 left the matrix
// passing; its check flag then stays 0, so every later sweep is skipped too.
__device__ __forceinline__ bool jacobi_skip(const int* counters, int sweep) {
  return sweep > 0 && counters[64 + sweep - 1] == 0;
}

// index of the i-th member (0..31) of pair block (a, b)
__device__ __forceinline__ int pair_index(int a, int b, int i) {
  return i < kJB ? a * kJB + i : b * kJB + (i - kJB);
}

// A rotation is applied when |a_pq| > max(tol sqrt(|a_pp a_qq|), tol * trace(H))
// (tol: 1e-15 for FP64 factors, looser where the sketch itself is FP32):
// the relative test gives small eigenvalues their accuracy, the absolute floor
// stops rotations that only chase the rounding of the tile updates.  Compared
// in squares (no square root).
__device__ __forceinline__ bool jac_rotates(double apq, double app, double aqq, double tol,
                                            double floor_abs) {
  return apq != 0.0 && apq * apq > fmax(tol * tol * fabs(app * aqq), floor_abs * floor_abs);
}

// The rotation (c, s) of positions p < q that zeroes a_pq, with the inner
// angle |phi| <= pi / 4: theta = (a_qq - a_pp) / 2, h = sqrt(theta^2 + a_pq^2),
// cos 2 phi = |theta| / h, c^2 = (1 + cos 2 phi) / 2 and s = sign(theta) a_pq /
// (2 h c).  c^2 has no cancellation, and c^2 + s^2 = 1 to rounding because
// sin^2 2 phi = 1 - cos^2 2 phi.  s = 0 means no rotation.
__device__ __forceinline__ double2 jac_rotation(double apq, double app, double aqq, double tol,
                                                double floor_abs, bool* rotated) {
  if (!jac_rotates(apq, app, aqq, tol, floor_abs)) return make_double2(1.0, 0.0);
  *rotated = true;
  const double theta = 0.5 * (aqq - app);
  const double h2 = fma(theta, theta, apq * apq);
  double c, s;
  if (h2 > 1e-280 && h2 < 1e280) {
    const double rh = rsq_nr(h2);
    const double c2 = fma(0.5 * fabs(theta), rh, 0.5);
    const double rc = rsq_nr(c2);
    c = c2 * rc;
    s = 0.5 * apq * rh * rc;
  } else {   // squares near the ends of the range: the tangent form, no squaring
    const double tau = theta / apq;
    const double t = copysign(1.0 / (fabs(tau) + sqrt(1.0 + tau * tau)), apq);
    c = 1.0 / sqrt(fma(t, t, 1.0));
    s = t * c;
  }
  return make_double2(c, theta < 0.0 ? -s : s);
}

// (x00 x01; x10 x11) <- J_a^T X J_b for the rotations ra (rows) and rb (columns)
__device__ __forceinline__ void blk_rotate(double2 ra, double2 rb, double& x00, double& x01,
                                           double& x10, double& x11) {
  if (ra.y != 0.0) {
    const double c = ra.x, s = ra.y;
    const double y00 = c * x00 - s * x10, y01 = c * x01 - s * x11;
    const double y10 = s * x00 + c * x10, y11 = s * x01 + c * x11;
    x00 = y00; x01 = y01; x10 = y10; x11 = y11;
  }
  if (rb.y != 0.0) {
    const double c = rb.x, s = rb.y;
    const double y00 = c * x00 - s * x01, y01 = s * x00 + c * x01;
    const double y10 = c * x10 - s * x11, y11 = s * x10 + c * x11;
    x00 = y00; x01 = y01; x10 = y10; x11 = y11;
  }
}

// The same with no test: a rotation (1, 0) leaves finite entries unchanged
// bit for bit (c x - s y = x and s x + c y = y with c = 1, s = 0), so the
// cross steps apply every rotation without diverging on which ones are idle.
__device__ __forceinline__ void blk_rotate_all(double2 ra, double2 rb, double& x00, double& x01,
                                               double& x10, double& x11) {
  {
    const double c = ra.x, s = ra.y;
    const double y00 = c * x00 - s * x10, y01 = c * x01 - s * x11;
    const double y10 = s * x00 + c * x10, y11 = s * x01 + c * x11;
    x00 = y00; x01 = y01; x10 = y10; x11 = y11;
  }
  {
    const double c = rb.x, s = rb.y;
    const double y00 = c * x00 - s * x01, y01 = s * x00 + c * x01;
    const double y10 = c * x10 - s * x11, y11 = s * x10 + c * x11;
    x00 = y00; x01 = y01; x10 = y10; x11 = y11;
  }
}

__device__ __forceinline__ int rr16(int x, int st) { return x == 0 ? 0 : ((x - 1 + st) % 15) + 1; }

// Positions p < q of rotation k (0..15) at step st of a visit.  INTRA steps:
// rotations 0..7 pair positions of the first block (round-robin over its 16
// indices), 8..15 those of the second.  Cross steps: k with 16 + (k + st) % 16.
template <bool INTRA>
__device__ __forceinline__ void step_pair(int k, int st, int* p, int* q) {
  if (INTRA) {
    const int blk = k >> 3, kk = k & 7;
    int x = rr16(kk, st), y = rr16(15 - kk, st);
    if (x > y) {
      const int t = x;
      x = y;
      y = t;
    }
    *p = kJB * blk + x;
    *q = kJB * blk + y;
  } else {
    *p = k;
    *q = kJB + ((k + st) & (kJB - 1));
  }
}

// The 2x2 block of rotations (ka, kb), ka <= kb, of the step, and its mirror.
// S stays exactly symmetric: the block and its transpose get the same values,
// and the rotated pair's off-diagonal entry is set to zero.
template <bool INTRA>
__device__ __forceinline__ void upd_block(double (&S)[kJP][kJP + 1], const double2* C, int st,
                                          int ka, int kb) {
  const double2 ra = C[ka], rb = C[kb];
  if (ra.y == 0.0 && rb.y == 0.0) return;
  int p, q, p2, q2;
  step_pair<INTRA>(ka, st, &p, &q);
  step_pair<INTRA>(kb, st, &p2, &q2);
  double x00 = S[p][p2], x01 = S[p][q2], x10 = S[q][p2], x11 = S[q][q2];
  blk_rotate(ra, rb, x00, x01, x10, x11);
  if (ka == kb) {
    S[p][p] = x00;
    S[q][q] = x11;
    S[p][q] = 0.0;
    S[q][p] = 0.0;
  } else {
    S[p][p2] = x00; S[p][q2] = x01; S[q][p2] = x10; S[q][q2] = x11;
    S[p2][p] = x00; S[q2][p] = x01; S[p2][q] = x10; S[q2][q] = x11;
  }
}

// upd_block for a cross step's off-diagonal block (ka < kb), every rotation
// applied (see blk_rotate_all)
__device__ __forceinline__ void upd_block_cross(double (&S)[kJP][kJP + 1], const double2* C,
                                                int st, int ka, int kb) {
  const double2 ra = C[ka], rb = C[kb];
  int p, q, p2, q2;
  step_pair<false>(ka, st, &p, &q);
  step_pair<false>(kb, st, &p2, &q2);
  double x00 = S[p][p2], x01 = S[p][q2], x10 = S[q][p2], x11 = S[q][q2];
  blk_rotate_all(ra, rb, x00, x01, x10, x11);
  S[p][p2] = x00; S[p][q2] = x01; S[q][p2] = x10; S[q][q2] = x11;
  S[p2][p] = x00; S[q2][p] = x01; S[p2][q] = x10; S[q2][q] = x11;
}

// Q <- Q J over the 16 rotations of the step: two (row, rotation) pairs per thread
template <bool INTRA>
__device__ __forceinline__ void upd_q(double (&Q)[kJP][kJP + 1], const double2* C, int st,
                                      int tid) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + kJT * h;
    const int i = e >> 4, k = e & (kJB - 1);
    const double2 r = C[k];
    if (r.y != 0.0) {
      int p, q;
      step_pair<INTRA>(k, st, &p, &q);
      const double qp = Q[i][p], qv = Q[i][q];
      Q[i][p] = r.x * qp - r.y * qv;
      Q[i][q] = r.y * qp + r.x * qv;
    }
  }
}
static_assert(kJP * kJB == 2 * kJT, "two (row, rotation) pairs per thread");

// The same over the threads t = 0 .. 191 of wavefronts 1-3 (pairs t, t + 192,
// t + 384): every load of the step is issued before the first store (the
// pairs touch disjoint entries of Q).
constexpr int kJQT = kJT - 64;
constexpr int kJQN = (kJP * kJB + kJQT - 1) / kJQT;
__device__ __forceinline__ void upd_q_cross(double (&Q)[kJP][kJP + 1], const double2* C, int st,
                                            int t) {
  double2 r[kJQN];
  double qp[kJQN], qv[kJQN];
  int row[kJQN], pp[kJQN], qq[kJQN];
#pragma unroll
  for (int h = 0; h < kJQN; ++h) {
    const int e = t + kJQT * h;
    const int k = e & (kJB - 1);
    row[h] = e >> 4;
    step_pair<false>(k, st, &pp[h], &qq[h]);
    r[h] = (e < kJP * kJB) ? C[k] : make_double2(1.0, 0.0);
  }
  // every rotation applied (see blk_rotate_all); only the pairs past the 512
  // of the step are left out
#pragma unroll
  for (int h = 0; h < kJQN; ++h) {
    if (t + kJQT * h < kJP * kJB) {
      qp[h] = Q[row[h]][pp[h]];
      qv[h] = Q[row[h]][qq[h]];
    }
  }
#pragma unroll
  for (int h = 0; h < kJQN; ++h) {
    if (t + kJQT * h < kJP * kJB) {
      Q[row[h]][pp[h]] = r[h].x * qp[h] - r[h].y * qv[h];
      Q[row[h]][qq[h]] = r[h].y * qp[h] + r[h].x * qv[h];
    }
  }
}

// e-th upper 2x2 block (ka <= kb), row-major over the upper triangle
__device__ __forceinline__ void upper_block(int e, int* ka, int* kb) {
  int a = 0;
  while (e >= kJB - a) {
    e -= kJB - a;
    ++a;
  }
  *ka = a;
  *kb = a + e;
}
// e-th upper block that is neither diagonal nor (a, a + 1) nor (0, 15): the
// 104 blocks the rotation lanes do not own in the cross steps
constexpr int kJOther = kJU - 2 * kJB;
__device__ __forceinline__ void other_block(int e, int* ka, int* kb) {
  *ka = *kb = 0;
  for (int a = 0; a < kJB; ++a) {
    const int lo = a + 2, hi = (a == 0) ? kJB - 2 : kJB - 1;
    const int n = hi >= lo ? hi - lo + 1 : 0;
    if (e < n) {
      *ka = a;
      *kb = lo + e;
      return;
    }
    e -= n;
  }
}

// The 16 x 16 tile (ti, tj) of X Y (X^T Y when XT) for 32 x 32 operands in
// LDS on the FP64 matrix cores: lane (fk, fi) supplies X(16 ti + fi, k0 + fk)
// and Y(k0 + fk, 16 tj + fi) and holds rows 16 ti + fk + 4 v of column
// 16 tj + fi of the product in acc[v].  Wavefront w takes tile (w >> 1, w & 1).
static_assert(kJP == 32 && kJT == 256, "tile_mfma: four wavefronts, one 16 x 16 tile each");
template <bool XT>
__device__ __forceinline__ d4 tile_mfma(const double (&X)[kJP][kJP + 1],
                                        const double (&Y)[kJP][kJP + 1], int ti, int tj, int fi,
                                        int fk) {
  d4 acc = (d4)0.0;
#pragma unroll
  for (int k0 = 0; k0 < kJP; k0 += 4) {
    const double a = XT ? X[k0 + fk][16 * ti + fi] : X[16 * ti + fi][k0 + fk];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Y[k0 + fk][16 * tj + fi], acc, 0, 0, 0);
  }
  return acc;
}

// Update workgroup v of round t: v < np^2 forms tile (P, Q) of
// Hout = Q_P^T Hin[P, Q] Q_Q; the others take V[rows, P] <- V[rows, P] Q_P.
__device__ __forceinline__ void jacobi_update(const double* __restrict__ Hin,
                                              double* __restrict__ Hout, double* __restrict__ V,
                                              int R, int t, const double* __restrict__ Qbuf,
                                              int v, double (&T)[kJP][kJP + 1],
                                              double (&W)[kJP][kJP + 1]) {
  const int tid = threadIdx.x;
  const int nb = R / kJB;
  const int np = nb / 2;
  const int lane = tid & 63, wv = tid >> 6;
  const int ti = wv >> 1, tj = wv & 1, fi = lane & 15, fk = lane >> 4;
  if (v < np * np) {
    const int P = v / np, Qi = v % np;
    int pa, pb, qa, qb;
    rr_pair(nb, t, P, &pa, &pb);
    rr_pair(nb, t, Qi, &qa, &qb);
    const double* QP = Qbuf + (int64_t)P * kJP * kJP;
    const double* QQ = Qbuf + (int64_t)Qi * kJP * kJP;
#pragma unroll
    for (int h = 0; h < kJE; ++h) {
      const int e = tid + h * kJT;
      const int i = e / kJP, j = e % kJP;
      T[i][j] = Hin[(int64_t)pair_index(pa, pb, i) * R + pair_index(qa, qb, j)];
      W[i][j] = QQ[e];
    }
    __syncthreads();
    d4 o = tile_mfma<false>(T, W, ti, tj, fi, fk);   // X = T Q_Q
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) T[16 * ti + fk + 4 * q][16 * tj + fi] = o[q];
#pragma unroll
    for (int h = 0; h < kJE; ++h) {
      const int e = tid + h * kJT;
      W[e / kJP][e % kJP] = QP[e];
    }
    __syncthreads();
    o = tile_mfma<true>(W, T, ti, tj, fi, fk);        // Q_P^T X
#pragma unroll
    for (int q = 0; q < 4; ++q)
      Hout[(int64_t)pair_index(pa, pb, 16 * ti + fk + 4 * q) * R +
           pair_index(qa, qb, 16 * tj + fi)] = o[q];
  } else {
    const int w = v - np * np;
    const int P = w % np, rc = w / np;
    int pa, pb;
    rr_pair(nb, t, P, &pa, &pb);
    const double* QP = Qbuf + (int64_t)P * kJP * kJP;
#pragma unroll
    for (int h = 0; h < kJE; ++h) {
      const int e = tid + h * kJT;
      const int i = e / kJP, j = e % kJP;
      T[i][j] = V[(int64_t)(rc * kJP + i) * R + pair_index(pa, pb, j)];
      W[i][j] = QP[e];
    }
    __syncthreads();
    const d4 o = tile_mfma<false>(T, W, ti, tj, fi, fk);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      V[(int64_t)(rc * kJP + 16 * ti + fk + 4 * q) * R + pair_index(pa, pb, 16 * tj + fi)] = o[q];
  }
}

// S <- the pair block (a, b) of H_t = Q^{t-1 T} H_{t-1} Q^{t-1}, from H_{t-1}
// (Hin) and the previous round's rotations: with block a in pair P1 of round
// t - 1 (half h1) and b in P2 (half h2), M_i the 16 columns of Q_{P_i} that
// belong to the block, S_aa = M1^T H[P1, P1] M1, S_bb = M2^T H[P2, P2] M2 and
// S_ab = M1^T H[P1, P2] M2.  S_aa and S_bb are made exactly symmetric (upper
// triangle kept).
struct PairForm {
  double T[3][kJP][kJP + 1];
  double M[2][kJP][kJB + 1];
  double X[3][kJP][kJB + 1];
};
__device__ __forceinline__ void form_pair(const double* __restrict__ Hin,
                                          const double* __restrict__ Qprev, int R, int t, int a,
                                          int b, PairForm& F, double (&S)[kJP][kJP + 1]) {
  const int tid = threadIdx.x;
  const int nb = R / kJB;
  int P[2], hf[2];
  rr_locate(nb, t - 1, a, &P[0], &hf[0]);
  rr_locate(nb, t - 1, b, &P[1], &hf[1]);
  int m0[2], m1[2];
  rr_pair(nb, t - 1, P[0], &m0[0], &m1[0]);
  rr_pair(nb, t - 1, P[1], &m0[1], &m1[1]);
  // tiles (P1, P1), (P2, P2), (P1, P2) and the two column blocks of Q
#pragma unroll
  for (int h = 0; h < kJE; ++h) {
    const int e = tid + h * kJT;
    const int i = e / kJP, j = e % kJP;
    const int r0 = pair_index(m0[0], m1[0], i), r1 = pair_index(m0[1], m1[1], i);
    const int c0 = pair_index(m0[0], m1[0], j), c1 = pair_index(m0[1], m1[1], j);
    F.T[0][i][j] = Hin[(int64_t)r0 * R + c0];
    F.T[1][i][j] = Hin[(int64_t)r1 * R + c1];
    F.T[2][i][j] = Hin[(int64_t)r0 * R + c1];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + h * kJT;   // 512 = 32 x 16 per block
    const int i = e >> 4, c = e & 15;
    F.M[0][i][c] = Qprev[(int64_t)P[0] * kJP * kJP + i * kJP + kJB * hf[0] + c];
    F.M[1][i][c] = Qprev[(int64_t)P[1] * kJP * kJP + i * kJP + kJB * hf[1] + c];
  }
  __syncthreads();
  // FP64 MFMA 16x16x4: lane (fk, fi) = (lane >> 4, lane & 15) supplies
  // A(fi, k0 + fk) and B(k0 + fk, fi) and holds D(fk + 4 v, fi) in acc[v].
  // X0 = T0 M1, X1 = T1 M2, X2 = T2 M2: six 16 x 16 tiles (matrix tt >> 1,
  // row half tt & 1), K = 32; wavefronts 0, 1 take two, 2, 3 one.
  const int lane = tid & 63, wv = tid >> 6;
  const int fi = lane & 15, fk = lane >> 4;
  for (int tt = wv; tt < 6; tt += 4) {
    const int which = tt >> 1, rh = tt & 1, mi = which == 0 ? 0 : 1;
    d4 acc = (d4)0.0;
#pragma unroll
    for (int k0 = 0; k0 < kJP; k0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(F.T[which][kJB * rh + fi][k0 + fk],
                                                 F.M[mi][k0 + fk][fi], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) F.X[which][kJB * rh + fk + 4 * v][fi] = acc[v];
  }
  __syncthreads();
  // S_aa = M1^T X0, S_bb = M2^T X1, S_ab = M1^T X2: one 16 x 16 tile per
  // wavefront 0..2
  if (wv < 3) {
    const int h = wv, mi = h == 1 ? 1 : 0;
    d4 acc = (d4)0.0;
#pragma unroll
    for (int k0 = 0; k0 < kJP; k0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(F.M[mi][k0 + fk][fi], F.X[h][k0 + fk][fi], acc,
                                                 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = fk + 4 * v, j = fi;
      const double sv = acc[v];
      if (h == 0) {
        if (i <= j) { S[i][j] = sv; S[j][i] = sv; }
      } else if (h == 1) {
        if (i <= j) { S[kJB + i][kJB + j] = sv; S[kJB + j][kJB + i] = sv; }
      } else {
        S[i][kJB + j] = sv;
        S[kJB + j][i] = sv;
      }
    }
  }
}

// One round of the sweep.  Workgroups 0 .. nb/2 - 1 solve the pair blocks of
// round t and write Qcur; with FIRST (round 0) they take the pair block from
// Hin directly and rotate the intra-block pairs first, otherwise they form it
// from Hin = H_{t-1} and Qprev, and the further workgroups write
// Hout = H_t and update V with Qprev.
//
// In the cross steps the rotation lanes (0..15) own the diagonal block of
// their rotation and the block (k, k + 1) (lane 15: (0, 15)); after applying
// the step they hold every entry that the next step's rotation k needs
// (a_kk, a_kq and, from lane k + 1, a_qq), so the next rotation is formed
// before the barrier and a step takes one barrier.  The other 104 blocks and
// the columns of Q are updated by wavefronts 1-3, so the rotation lanes'
// chain (block update, next rotation) is the only work of wavefront 0.
template <bool FIRST>
__global__ __launch_bounds__(kJT) void k_jacobi_round(const double* __restrict__ Hin,
                                                      double* __restrict__ Hout,
                                                      double* __restrict__ V, int R, int round,
                                                      const double* __restrict__ Qprev,
                                                      double* __restrict__ Qcur,
                                                      int* __restrict__ counters, int sweep,
                                                      const double* __restrict__ gnorm,
                                                      double tol) {
  if (jacobi_skip(counters, sweep)) return;
  // S and Q live in the first two T tiles of F: those are dead once the
  // pair block is formed (and never used in round 0), which keeps the launch
  // at 47 KB of LDS (three workgroups per CU at large r)
  __shared__ double2 cs[2][kJB];
  __shared__ PairForm F;
  double (&S)[kJP][kJP + 1] = F.T[0];
  double (&Q)[kJP][kJP + 1] = F.T[1];
  const int tid = threadIdx.x;
  const int nb = R / kJB;
  const int np = nb / 2;
  if (!FIRST && (int)blockIdx.x >= np) {
    jacobi_update(Hin, Hout, V, R, round - 1, Qprev, blockIdx.x - np, F.T[0], F.T[1]);
    return;
  }
  const double floor_abs = tol * (*gnorm);
  int a, b;
  rr_pair(nb, round, blockIdx.x, &a, &b);
  if (FIRST) {
#pragma unroll
    for (int h = 0; h < kJE; ++h) {
      const int e = tid + h * kJT;
      const int i = e / kJP, j = e % kJP;
      // upper triangle of the pair block, mirrored (H is symmetric up to rounding)
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      S[i][j] = Hin[(int64_t)pair_index(a, b, lo) * R + pair_index(a, b, hi)];
    }
  } else {
    form_pair(Hin, Qprev, R, round, a, b, F, S);
  }
#pragma unroll
  for (int h = 0; h < kJE; ++h) {
    const int e = tid + h * kJT;
    Q[e / kJP][e % kJP] = (e / kJP == e % kJP) ? 1.0 : 0.0;
  }
  bool rotated = false;
  __syncthreads();
  if (FIRST) {
    int gka = 0, gkb = 0;
    const bool gblk = tid < kJU;
    if (gblk) upper_block(tid, &gka, &gkb);
    for (int st = 0; st < kJB - 1; ++st) {
      if (tid < kJB) {
        int p, q;
        step_pair<true>(tid, st, &p, &q);
        cs[0][tid] = jac_rotation(S[p][q], S[p][p], S[q][q], tol, floor_abs, &rotated);
      }
      __syncthreads();
      if (gblk) upd_block<true>(S, cs[0], st, gka, gkb);
      upd_q<true>(Q, cs[0], st, tid);
      __syncthreads();
    }
  }
  // cross steps
  int oka = 0, okb = 0;
  const bool oblk = tid >= 64 && tid < 64 + kJOther;
  if (oblk) other_block(tid - 64, &oka, &okb);
  double app = 0.0, apq = 0.0, aqq = 0.0;
  if (tid < kJB) {
    app = S[tid][tid];
    apq = S[tid][kJB + tid];
    aqq = S[kJB + tid][kJB + tid];
    cs[0][tid] = jac_rotation(apq, app, aqq, tol, floor_abs, &rotated);
  }
  __syncthreads();
  for (int st = 0; st < kJB; ++st) {
    const double2* C = cs[st & 1];
    if (tid < kJB) {
      const int k = tid, k1 = (k + 1) & (kJB - 1);
      const int ka = (k < kJB - 1) ? k : 0, kb = (k < kJB - 1) ? k1 : kJB - 1;
      const int p = ka, q = kJB + ((ka + st) & (kJB - 1));
      const int p2 = kb, q2 = kJB + ((kb + st) & (kJB - 1));
      double x00 = S[p][p2], x01 = S[p][q2], x10 = S[q][p2], x11 = S[q][q2];
      const double2 rk = C[k], ra = C[ka], rb = C[kb];
      // the diagonal block of rotation k, from the registers; every rotation
      // applied (see blk_rotate_all), the rotated pair's entry set to 0
      double d00 = app, d01 = apq, d10 = apq, d11 = aqq;
      const int qk = kJB + ((k + st) & (kJB - 1));
      blk_rotate_all(rk, rk, d00, d01, d10, d11);
      const double dz = (rk.y != 0.0) ? 0.0 : apq;
      S[k][k] = d00;
      S[qk][qk] = d11;
      S[k][qk] = dz;
      S[qk][k] = dz;
      blk_rotate_all(ra, rb, x00, x01, x10, x11);
      S[p][p2] = x00; S[p][q2] = x01; S[q][p2] = x10; S[q][q2] = x11;
      S[p2][p] = x00; S[q2][p] = x01; S[p2][q] = x10; S[q2][q] = x11;
      const double nx11 = __shfl(d11, k1, 64);
      if (st + 1 < kJB) {
        app = d00;
        aqq = nx11;
        apq = (k < kJB - 1) ? x01 : x10;
        cs[(st + 1) & 1][k] = jac_rotation(apq, app, aqq, tol, floor_abs, &rotated);
      }
    } else if (tid >= 64) {
      // wavefronts 1-3: the other blocks, then Q (wavefront 0 carries the
      // rotation lanes' dependent chain alone)
      if (oblk) upd_block_cross(S, C, st, oka, okb);
      upd_q_cross(Q, C, st, tid - 64);
    }
    __syncthreads();
  }
  double* Qo = Qcur + (int64_t)blockIdx.x * kJP * kJP;
#pragma unroll
  for (int h = 0; h < kJE; ++h) {
    const int e = tid + h * kJT;
    Qo[e] = Q[e / kJP][e % kJP];
  }
  // only the first kJB threads (all in the first wavefront) compute rotations
  if (__any(rotated) && tid == 0) atomicAdd(&counters[sweep], 1);
}

// The update of the last round of a sweep (no solve follows in its launch).
__global__ __launch_bounds__(kJT) void k_jacobi_update(const double* __restrict__ Hin,
                                                       double* __restrict__ Hout,
                                                       double* __restrict__ V, int R, int round,
                                                       const double* __restrict__ Qbuf,
                                                       const int* __restrict__ counters,
                                                       int sweep) {
  if (jacobi_skip(counters, sweep)) return;
  __shared__ double T[kJP][kJP + 1];
  __shared__ double W[kJP][kJP + 1];
  jacobi_update(Hin, Hout, V, R, round, Qbuf, blockIdx.x, T, W);
}

// *out = trace of the R x R matrix (one workgroup)
// flag = 1 if some off-diagonal pair of G fails the rotation criterion of
// the pair solves (a further sweep would rotate); 0 stays otherwise.  The
// updated G is symmetric only up to the rounding of the tile products, and a
// pair block reads whichever of G(i,j), G(j,i) its local order puts above the
// diagonal, so the pair counts as converged when either entry passes.
__global__ __launch_bounds__(256) void k_jacobi_check(const double* __restrict__ G, int R,
                                                     const double* __restrict__ gnorm,
                                                     int* __restrict__ counters, int sweep,
                                                     double tol) {
  if (jacobi_skip(counters, sweep)) return;
  int* flag = counters + 64 + sweep;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)R * R) return;
  const int i = (int)(e / R), j = (int)(e % R);
  if (j <= i) return;
  const double floor_abs = tol * (*gnorm);
  const double apq = fmin(fabs(G[e]), fabs(G[(int64_t)j * R + i]));
  const double app = G[(int64_t)i * R + i], aqq = G[(int64_t)j * R + j];
  if (jac_rotates(apq, app, aqq, tol, floor_abs)) *flag = 1;
}

// The check flag of sweep s, with the sequence number the host waits for, as
// one 8-byte store into pinned host memory.
__global__ void k_jacobi_report(const int* __restrict__ counters, int sweep,
                                unsigned long long* __restrict__ slot, unsigned seq) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    *slot = ((unsigned long long)seq << 32) | (unsigned)counters[64 + sweep];
}

__global__ __launch_bounds__(256) void k_trace(const double* __restrict__ G, int R,
                                               double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < R; i += 256) s += fabs(G[(int64_t)i * R + i]);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void k_eye(double* __restrict__ V, int R) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (int64_t)R * R) V[e] = (e / R == e % R) ? 1.0 : 0.0;
}

// V (R x R row-major) = the column-major r x r basis B0, identity on the padding
__global__ void k_pad_basis(const double* __restrict__ B0, int r, double* __restrict__ V, int R) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)R * R) return;
  const int k = (int)(e / R), c = (int)(e % R);
  V[e] = (k < r && c < r) ? B0[(int64_t)c * r + k] : (k == c ? 1.0 : 0.0);
}

// Pad the r x r matrix (ld) into an R x R zero-padded matrix.
__global__ void k_pad(const double* __restrict__ A, int r, int ld, double* __restrict__ P, int R) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)R * R) return;
  const int i = (int)(e / R), j = (int)(e % R);
  P[e] = (i < r && j < r) ? A[(int64_t)i * ld + j] : 0.0;
}

// Descending order of diag(G) (R entries); perm[k] = index of the k-th largest,
// sig2[k] its value.  Ties keep index order.
__global__ __launch_bounds__(1024) void k_eig_sort(const double* __restrict__ G, int R,
                                                   int* __restrict__ perm,
                                                   double* __restrict__ sig2) {
  const int i = threadIdx.x;
  if (i >= R) return;
  const double v = G[(int64_t)i * R + i];
  int rank = 0;
  for (int j = 0; j < R; ++j) {
    const double w = G[(int64_t)j * R + j];
    rank += (w > v) || (w == v && j < i);
  }
  perm[rank] = i;
  sig2[rank] = v;
}

// W(k, c) = V(k, perm[c]) / sqrt(sig2[c]) for k < r, c < r  (row-major r x r, ldw)
__global__ void k_eig_vectors(const double* __restrict__ V, int R, const int* __restrict__ perm,
                              const double* __restrict__ sig2, int r, double* __restrict__ W,
                              int ldw) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int k = (int)(e / r), c = (int)(e % r);
  W[(int64_t)k * ldw + c] = V[(int64_t)k * R + perm[c]] / sqrt(sig2[c]);
}

}  // namespace

nys_status gemm64(hipStream_t st, int M, int N, int K, const void* A, bool a_f32, int64_t sam,
                  int64_t sak, const void* B, bool b_f32, int64_t sbk, int64_t sbn, double* C,
                  int64_t scm, int64_t scn, double alpha, double beta, double* split_ws,
                  size_t split_ws_elems, const double* wk) {
  if (M <= 0 || N <= 0) return NYS_OK;
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  // split K (chunks of >= 128) until about four workgroups per CU are busy
  int S = 1;
  if (K > 256 && split_ws != nullptr) {
    S = std::min((K + 127) / 128, std::max(1, 1024 / (tm * tn)));
    while (S > 1 && (size_t)S * M * N > split_ws_elems) --S;
  }
  int kchunk = (K + S - 1) / S;
  kchunk = (kchunk + 15) / 16 * 16;
  S = std::max(1, (K + kchunk - 1) / kchunk);
  dim3 grid(tn, tm, S);
  double* out = S > 1 ? split_ws : C;
  const int64_t sstride = (int64_t)M * N;
#define NYS_GEMM(TA, TB)                                                                     \
  hipLaunchKernelGGL((k_gemm64<TA, TB>), grid, dim3(256), 0, st, M, N, K, kchunk,            \
                     static_cast<const TA*>(A), sam, sak, static_cast<const TB*>(B), sbk, sbn, \
                     out, scm, scn, sstride, alpha, beta, wk)
  if (a_f32 && b_f32) NYS_GEMM(float, float);
  else if (a_f32) NYS_GEMM(float, double);
  else if (b_f32) NYS_GEMM(double, float);
  else NYS_GEMM(double, double);
#undef NYS_GEMM
  if (hipGetLastError() != hipSuccess) return NYS_ERR_HIP;
  if (S > 1) {
    const int64_t tot = (int64_t)M * N;
    hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((tot + kSrOut - 1) / kSrOut)), dim3(256), 0,
                       st, M, N, S, split_ws, C, scm, scn, alpha, beta);
    if (hipGetLastError() != hipSuccess) return NYS_ERR_HIP;
  }
  return NYS_OK;
}

nys_status chol_upper(hipStream_t st, double* M, int r, int ld, int* fail) {
  if (r > 1024) return NYS_ERR_INVALID;
  if (r <= kCholOneWg) {
    hipLaunchKernelGGL(k_chol_upper, dim3(1), dim3(kCholT), 0, st, M, r, ld, fail);
    return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
  }
  // blocked right-looking form for larger r: per block row, the diagonal
  // block (one workgroup), the block row (a workgroup per kLB columns) and the
  // trailing update (a workgroup per kLB x kLB tile of the upper triangle)
  for (int kb = 0; kb < r; kb += kLB) {
    const int b = std::min(kLB, r - kb);
    const int nrest = r - kb - b;
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, M, ld, kb, b, fail);
    if (nrest > 0) {
      const int tc = (nrest + kLB - 1) / kLB;
      hipLaunchKernelGGL(k_chol_panel, dim3(tc), dim3(256), 0, st, M, ld, kb, b, nrest, fail);
      hipLaunchKernelGGL(k_chol_trail, dim3(tc * (tc + 1) / 2), dim3(256), 0, st, M, ld, kb, b,
                         nrest, tc, fail);
    }
  }
  hipLaunchKernelGGL(k_chol_mirror_lower, dim3((unsigned)(((int64_t)r * r + 255) / 256)), dim3(256),
                     0, st, M, r, ld, fail);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status trinv_upper(hipStream_t st, const double* Cm, int r, int ld, double* Z, int ldz) {
  if (r > 1024) return NYS_ERR_INVALID;
  const dim3 grid((r + 3) / 4);
  if (r <= 256)
    hipLaunchKernelGGL((k_trinv_upper<4, 16>), grid, dim3(256), 0, st, Cm, r, ld, Z, ldz);
  else if (r <= 512)
    hipLaunchKernelGGL((k_trinv_upper<8, 8>), grid, dim3(256), 0, st, Cm, r, ld, Z, ldz);
  else
    hipLaunchKernelGGL((k_trinv_upper<16, 4>), grid, dim3(256), 0, st, Cm, r, ld, Z, ldz);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status power_iter(hipStream_t st, const double* G, int r, int ld, int iters, double* out) {
  if (r > 1024) return NYS_ERR_INVALID;
  hipLaunchKernelGGL(k_power_iter, dim3(1), dim3(1024), 0, st, G, r, ld, iters, out);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

int jacobi_pad(int r) { return std::max(kJP, (r + kJP - 1) / kJP * kJP); }

size_t jacobi_ws_doubles(int r) {
  const int R = jacobi_pad(r);
  const int np = R / kJP;
  return 2 * (size_t)R * R + (size_t)R * R + 2 * (size_t)np * kJP * kJP + 2 * (size_t)R + 128;
}

// Eigendecomposition of the symmetric r x r matrix G (row-major, ld) by block
// Jacobi.  Outputs: sig2 (r, descending) and W (r x r row-major, ldw) with
// W(:, c) = v_c / sqrt(sig2_c).  ws must hold jacobi_ws_doubles(r) doubles;
// counters (>= max_sweeps ints) and host_flag are scratch.  Returns
// NYS_ERR_NOT_CONVERGED if a sweep still rotated after max_sweeps.
// Wait until the device has written sequence number seq into the slot; once
// the slot has stayed unwritten for a few milliseconds the stream is queried
// (PollPace) so that a failed or drained stream ends the wait with an error.
nys_status wait_jacobi_slot(hipStream_t st, const volatile unsigned long long* slot, unsigned seq,
                            int* val) {
  PollPace pace;
  for (long n = 1;; ++n) {
    unsigned long long v = *slot;
    if ((unsigned)(v >> 32) == seq) {
      *val = (int)(unsigned)(v & 0xffffffffu);
      return NYS_OK;
    }
    if (pace.due(n)) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        v = *slot;
        if ((unsigned)(v >> 32) != seq) return NYS_ERR_HIP;
        *val = (int)(unsigned)(v & 0xffffffffu);
        return NYS_OK;
      }
      if (e != hipErrorNotReady) return NYS_ERR_HIP;
    }
    __builtin_ia32_pause();
  }
}

nys_status jacobi_eig(hipStream_t st, const double* G, int r, int ld, double* ws, int* counters,
                      int max_sweeps, void* host_pinned, void* host_pinned_dev, int* poll_seq,
                      double* sig2, double* W, int ldw, int* sweeps_out, const double* V0,
                      double tol) {
  const int R = jacobi_pad(r);
  const int nb = R / kJB;
  const int np = nb / 2;
  double* G0 = ws;
  double* G1 = G0 + (size_t)R * R;
  double* V = G1 + (size_t)R * R;
  double* Qr[2] = {V + (size_t)R * R, V + (size_t)R * R + (size_t)np * kJP * kJP};
  double* s2 = Qr[1] + (size_t)np * kJP * kJP;
  int* perm = reinterpret_cast<int*>(s2 + R);
  double* gnorm = s2 + 2 * R;   // perm occupies R ints = R/2 doubles
  const int64_t RR = (int64_t)R * R;
  if (max_sweeps < 1 || max_sweeps > 60) return NYS_ERR_INVALID;
  hipLaunchKernelGGL(k_pad, dim3((unsigned)((RR + 255) / 256)), dim3(256), 0, st, G, r, ld, G0, R);
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, st, G0, R, gnorm);
  if (V0 != nullptr)
    hipLaunchKernelGGL(k_pad_basis, dim3((unsigned)((RR + 255) / 256)), dim3(256), 0, st, V0, r,
                       V, R);
  else
    hipLaunchKernelGGL(k_eye, dim3((unsigned)((RR + 255) / 256)), dim3(256), 0, st, V, R);
  if (hipMemsetAsync(counters, 0, sizeof(int) * 128, st) != hipSuccess) return NYS_ERR_HIP;
  // Sweeps are enqueued one ahead of the host's reading of their check flag
  // (written by the device into pinned memory), so the GPU does not idle on a
  // host round trip between sweeps; a sweep enqueued after convergence returns
  // at once.  after[s] is the buffer that holds the matrix after sweep s.
  auto* slots_h = reinterpret_cast<volatile unsigned long long*>(
      static_cast<char*>(host_pinned) + kJacSlotOffset);
  auto* slots_d =
      reinterpret_cast<unsigned long long*>(static_cast<char*>(host_pinned_dev) + kJacSlotOffset);
  double* after[60];
  unsigned seqs[60];
  constexpr int kAhead = 2;
  int enq = 0, sweeps = 0;
  bool converged = false;
  for (int s = 0; s < max_sweeps; ++s) {
    while (enq < max_sweeps && enq - s < kAhead) {
      // round t's launch solves round t and applies round t - 1 (G0 = H_{t-1}
      // in, G1 = H_t out); the last round's update is a launch of its own
      const unsigned nupd = (unsigned)(np * np + np * (R / kJP));
      hipLaunchKernelGGL(k_jacobi_round<true>, dim3(np), dim3(kJT), 0, st, G0, G1, V, R, 0,
                         Qr[1], Qr[0], counters, enq, gnorm, tol);
      for (int t = 1; t < nb - 1; ++t) {
        hipLaunchKernelGGL(k_jacobi_round<false>, dim3(np + nupd), dim3(kJT), 0, st, G0, G1, V,
                           R, t, Qr[(t - 1) & 1], Qr[t & 1], counters, enq, gnorm, tol);
        std::swap(G0, G1);
      }
      hipLaunchKernelGGL(k_jacobi_update, dim3(nupd), dim3(kJT), 0, st, G0, G1, V, R, nb - 2,
                         Qr[(nb - 2) & 1], counters, enq);
      std::swap(G0, G1);
      after[enq] = G0;
      // converged when every off-diagonal pair passes the rotation criterion,
      // i.e. when the next sweep would not rotate
      hipLaunchKernelGGL(k_jacobi_check, dim3((unsigned)((RR + 255) / 256)), dim3(256), 0, st,
                         G0, R, gnorm, counters, enq, tol);
      // sequence numbers are unique per context: stale slot contents never match
      *poll_seq = (*poll_seq % 1000000000) + 1;
      seqs[enq] = (unsigned)*poll_seq;
      hipLaunchKernelGGL(k_jacobi_report, dim3(1), dim3(64), 0, st, counters, enq,
                         slots_d + (enq % 4), seqs[enq]);
      if (hipGetLastError() != hipSuccess) return NYS_ERR_HIP;
      ++enq;
    }
    int flag = 1;
    NYS_TRY(wait_jacobi_slot(st, slots_h + (s % 4), seqs[s], &flag));
    ++sweeps;
    if (flag == 0) {
      converged = true;
      G0 = after[s];
      break;
    }
  }
  if (!converged) return NYS_ERR_NOT_CONVERGED;
  hipLaunchKernelGGL(k_eig_sort, dim3(1), dim3(1024), 0, st, G0, R, perm, s2);
  if (hipMemcpyAsync(sig2, s2, sizeof(double) * r, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return NYS_ERR_HIP;
  const int64_t rr = (int64_t)r * r;
  hipLaunchKernelGGL(k_eig_vectors, dim3((unsigned)((rr + 255) / 256)), dim3(256), 0, st, V, R,
                     perm, s2, r, W, ldw);
  if (sweeps_out) *sweeps_out = sweeps;
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

}  // namespace nys
