// Device building blocks of the fused matvec pair, shared by the single-
// problem kernel (gemv.hip) and the batched path (batched.hip).
#pragma once

#include "internal.h"

namespace nys {
namespace gram {

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


// First column of chunk m of thread tid.  Rows that are 16-byte aligned are
// read chunk-interleaved across the workgroup (consecutive threads, then the
// next chunk); unaligned rows give each wave a contiguous block of CPL chunks,
// so that re-aligning a chunk only needs the next lane of the same wave
// (except at the end of the wave's block).
template <typename T, int CPL, bool ALIGNED, int NT>
__device__ __forceinline__ int col0(int tid, int m) {
  constexpr int VN = Chunk<T>::N;
  if (ALIGNED) return (tid + m * NT) * VN;
  return (((tid >> 6) * CPL + m) * 64 + (tid & 63)) * VN;
}

// Offset (in elements) of a row start from the previous 16-byte boundary.
template <typename T>
__device__ __forceinline__ int row_offset(const T* arow) {
  return (int)((reinterpret_cast<uintptr_t>(arow) / sizeof(T)) % Chunk<T>::N);
}

template <typename T>
struct Extra {
  static constexpr int N = Chunk<T>::N - 1;   // elements the last lane of a wave fetches
};

// Issue the loads of R rows (and of their epilogue inputs aux[row]).
// Aligned rows: one 16-byte load per chunk.
// Unaligned rows: each lane loads the 16-byte block at row_start - o + col
// (o = row_offset), which always holds at least one element of the row, and
// lane 63 also loads the Extra<T>::N elements after its last chunk; the blocks
// are shifted into column order by realign_group once they have arrived.
template <typename T, int CPL, int R, bool ALIGNED, int NT>
__device__ __forceinline__ void load_group(
    typename Chunk<T>::V (&a)[R][CPL], T (&ex)[R][Extra<T>::N], double (&av)[R],
    const T* __restrict__ A, const double* __restrict__ aux, int64_t row, int64_t r1, int d,
    int64_t ld, int tid) {
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int64_t rr = row + i;
    const bool ok = rr < r1;
    const T* arow = A + rr * ld;
    // the per-row input of the epilogue (D, or b) travels with the row
    av[i] = (aux != nullptr && ok) ? aux[rr] : 0.0;
    if (ALIGNED) {
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        const int c0 = col0<T, CPL, ALIGNED, NT>(tid, m);
        V val = (V)(T)0;
        if (ok && c0 < d) {
          if (c0 + VN <= d) {
            val = __builtin_nontemporal_load(reinterpret_cast<const V*>(arow + c0));
          } else {
#pragma unroll
            for (int v = 0; v < VN; ++v) val[v] = (c0 + v < d) ? arow[c0 + v] : (T)0;
          }
        }
        a[i][m] = val;
      }
    } else {
      const int o = row_offset(arow);
      const T* base = arow - o;
#pragma unroll
      for (int m = 0; m < CPL; ++m) {
        const int c0 = col0<T, CPL, ALIGNED, NT>(tid, m);
        V val = (V)(T)0;
        // the block holds row columns c0 - o .. c0 - o + VN - 1
        if (ok && c0 < d + o) val = __builtin_nontemporal_load(reinterpret_cast<const V*>(base + c0));
        a[i][m] = val;
      }
      const int cl = col0<T, CPL, ALIGNED, NT>(tid, CPL - 1);
#pragma unroll
      for (int k = 0; k < Extra<T>::N; ++k) {
        const int c = cl + 1 + k;
        ex[i][k] = (ok && (tid & 63) == 63 && c < d) ? arow[c] : (T)0;
      }
    }
  }
}

// Shift the blocks of unaligned rows into column order: column c0 + v is
// component v + o of the lane's block, or component v + o - VN of the next
// lane's block (the next chunk's lane 0 for lane 63, or the prefetched extra
// elements at the end of the wave's block).  Columns >= d become 0.
template <typename T, int CPL, int R, bool ALIGNED, int NT>
__device__ __forceinline__ void realign_group(typename Chunk<T>::V (&a)[R][CPL],
                                              const T (&ex)[R][Extra<T>::N],
                                              const T* __restrict__ A, int64_t row, int d,
                                              int64_t ld, int tid) {
  if (ALIGNED) return;
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
  const int lane = tid & 63;
  const int src = (lane + 1) & 63;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int o = row_offset(A + (row + i) * ld);
    if (o == 0) continue;   // uniform across the wave
#pragma unroll
    for (int m = 0; m < CPL; ++m) {
      const V cur = a[i][m];
      // lane 0 hands its next-chunk block to lane 63; others hand their own
      V give = cur;
      if (m + 1 < CPL && lane == 0) give = a[i][m + 1];
      V nb;
#pragma unroll
      for (int v = 0; v < VN; ++v) nb[v] = __shfl(give[v], src, 64);
      if (m == CPL - 1 && lane == 63) {
        // next block components k < o are columns c0 + VN - o + k = cl + 1 + (VN - o + k - 1)
#pragma unroll
        for (int k = 0; k < VN - 1; ++k) {
          T val = (T)0;
#pragma unroll
          for (int j = 0; j < Extra<T>::N; ++j)
            if (j == VN - o + k - 1) val = ex[i][j];
          if (k < o) nb[k] = val;
        }
      }
      const int c0 = col0<T, CPL, ALIGNED, NT>(tid, m);
      V out;
#pragma unroll
      for (int v = 0; v < VN; ++v) {
        T val = (T)0;
#pragma unroll
        for (int sft = 1; sft < VN; ++sft)
          if (sft == o) val = (v + sft < VN) ? cur[(v + sft) % VN] : nb[(v + sft) % VN];
        out[v] = (c0 + v < d) ? val : (T)0;
      }
      a[i][m] = out;
    }
  }
}

// Row dots of one group, cross-wave reduction, epilogue, and the A^T update.
template <typename T, int WAVES, int CPL, int R>
__device__ __forceinline__ void process_group(
    typename Chunk<T>::V (&a)[R][CPL], const double (&av)[R], int64_t row, int64_t r1, int mode,
    const double (&pr)[CPL][Chunk<T>::N], double (&yr)[CPL][Chunk<T>::N], double& q,
    const double* __restrict__ aux, double* __restrict__ auxout, double (*red)[R][WAVES],
    int& buf, int tid) {
  constexpr int VN = Chunk<T>::N;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const bool tonly = (mode == kModeTOnly);
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
    // converts the stored row again instead of keeping twice the registers
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
        double sacc = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) sacc += red[buf][i][w];
        t[i] = sacc;
      }
      buf ^= 1;
    }
  }
  double sv[R];
  if (mode == kModeLogit || mode == kModeLogGrad) {
    // transcendental epilogue: lane i evaluates row i, the results are
    // broadcast (one evaluation per wave instead of R in sequence)
    double ti = 0.0, bi = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (lane == i) {
        ti = t[i];
        bi = av[i];
      }
    const bool mine = lane < R && row + lane < r1;
    double sl = 0.0, ql = 0.0;
    if (mine) {
      const double sg = sigm(ti);
      const double lossl = log1p(exp(-fabs(ti))) + fmax(ti, 0.0) - bi * ti;
      if (mode == kModeLogit) {
        const double w = sg * sigm(-ti);
        sl = w * ti + bi - sg;
        if (auxout != nullptr && wv == 0) auxout[row + lane] = w;
      } else {
        sl = sg - bi;
      }
      ql = lossl;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      sv[i] = __shfl(sl, i, 64);
      q += __shfl(ql, i, 64);
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double sacc = 0.0;
      if (row + i < r1) {
        const double ti = tonly ? 0.0 : t[i];
        if (mode == kModeHess) {
          sacc = (aux != nullptr ? av[i] : 1.0) * ti;
          q = fma(sacc, ti, q);
        } else if (mode == kModeLsGrad) {
          sacc = ti - av[i];
          q = fma(sacc, sacc, q);
        } else {  // kModeTOnly
          sacc = av[i];
        }
      }
      sv[i] = sacc;
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int m = 0; m < CPL; ++m)
#pragma unroll
      for (int v = 0; v < VN; ++v) yr[m][v] = fma(sv[i], (double)a[i][m][v], yr[m][v]);
}

// Row dots only (y = A p over one block of columns, A explicit and
// symmetric in the kernel SVM): t_i = A_i p is written to out[row + i] and
// q += pr_i t_i, with pr_i = p at the row index (loaded with the row as av).
template <typename T, int WAVES, int CPL, int R>
__device__ __forceinline__ void rowdot_group(const typename Chunk<T>::V (&a)[R][CPL],
                                             const double (&av)[R], int64_t row, int64_t r1,
                                             const double (&pr)[CPL][Chunk<T>::N], double& q,
                                             double* __restrict__ out, double (*red)[R][WAVES],
                                             int& buf, int tid) {
  constexpr int VN = Chunk<T>::N;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  double t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < CPL; ++m)
#pragma unroll
      for (int v = 0; v < VN; ++v) acc = fma((double)a[i][m][v], pr[m][v], acc);
    t[i] = wave_sum(acc);
  }
  if (WAVES > 1) {
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < R; ++i) red[buf][i][wv] = t[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double sacc = 0.0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) sacc += red[buf][i][w];
      t[i] = sacc;
    }
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (row + i < r1) {
      q = fma(av[i], t[i], q);
      if (tid == i) out[row + i] = t[i];
    }
  }
}

}  // namespace gram
}  // namespace nys
