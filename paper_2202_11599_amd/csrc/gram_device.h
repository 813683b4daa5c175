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


template <typename T, int CPL, int R, bool ALIGNED, int NT>
__device__ __forceinline__ void load_group(
    typename Chunk<T>::V (&a)[R][CPL], const T* __restrict__ A, int64_t row, int64_t r1, int d,
    int64_t ld, int tid) {
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
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
}

// Row dots of one group, cross-wave reduction, epilogue, and the A^T update.
template <typename T, int WAVES, int CPL, int R>
__device__ __forceinline__ void process_group(
    typename Chunk<T>::V (&a)[R][CPL], int64_t row, int64_t r1, int mode,
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

}  // namespace gram
}  // namespace nys
