// Randomized Nystrom sketch (Algorithm RandNysAppx, block step of Algorithm
// AdaptiveRandNysAppx) and its FP64 core.
//
//   omega (Gaussian, d x m)  --CholeskyQR2 (FP64)-->  Omega block
//   T = A Omega               (n x m, MFMA for FP32/BF16, FP64 tiles otherwise)
//   Y = A^T (D o T) + c Omega (d x m, split-K MFMA + FP64 reduction)
//   core (FP64): nu from ||Y||_2, Cholesky of Omega^T Y_nu, B = Y_nu C^-1,
//   G = B^T B = V Sigma^2 V^T (block Jacobi), U = B V Sigma^-1,
//   Lambda = max(0, Sigma^2 - nu).
//
// In the FP32/BF16 forms the GEMMs use Omega rounded to that precision, and the
// core uses that rounded Omega (upcast) as the test matrix, so Y is a sketch of
// exactly the matrix the GEMMs multiplied.  Their core matrix Omega^T H Omega
// is formed as T^T D T + c Omega^T Omega in FP64 from the FP32 T, which equals
// Omega^T Y in exact arithmetic and stays positive definite whatever rounding
// the A^T pass carried.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <type_traits>
#include <cstdio>
#include <cstdlib>

#include "internal.h"

namespace nys {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f8 __attribute__((ext_vector_type(8)));

constexpr int kBK = 32;     // K step of the MFMA kernels
constexpr int kOPad = 40;   // LDS row pitch (elements) of the Omega / A^T tiles

__device__ __forceinline__ bf16x8 to_bf16(const f8& x) {
  bf16x8 r;
#pragma unroll
  for (int v = 0; v < 8; ++v) r[v] = (__bf16)x[v];
  return r;
}

// Load 8 consecutive floats p[0..7] (elements at or past `valid` are 0).
__device__ __forceinline__ f8 load8(const float* p, int valid, bool vec) {
  f8 r;
  if (vec && valid >= 8) {
    const f4 a = *reinterpret_cast<const f4*>(p);
    const f4 b = *reinterpret_cast<const f4*>(p + 4);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      r[v] = a[v];
      r[v + 4] = b[v];
    }
  } else {
#pragma unroll
    for (int v = 0; v < 8; ++v) r[v] = v < valid ? p[v] : 0.0f;
  }
  return r;
}

// T(:, col0 + c) = A Omega_lp(:, c), c < ncols, for rows row0 <= i < n (a
// launch may cover a range of rows).  A workgroup of NW wavefronts
// (blockDim = 64 NW) covers 16 RB NW rows from row0; wavefront w owns RB
// consecutive 16-row blocks (RB = 2 for at most 5 column blocks, so that a K
// step holds enough MFMA work, else 1) and all NB column blocks (16 NB
// columns from 16 NB blockIdx.y).  The Omega tile (16 NB x 32 per K step) goes
// through double-buffered LDS and is shared by the NW wavefronts; each
// wavefront reads its A rows straight from memory in MFMA operand order,
// the next step's rows and Omega tile loaded while the current step's MFMAs
// run (one barrier per step).  Omega_lp is (rows = columns of Omega) x ldo
// with zero padding up to ldo (a multiple of 32) and up to 16 NB rows.
constexpr int kSkMaxChunks = 4;   // 16-byte Omega chunks staged per thread
// column blocks from which the sketch passes read the next block's LDS operand
// during the current block's products (with fewer, measured slower)
constexpr int kSkPipeNB = 6;
constexpr int kSk1MaxW = 13;      // wavefronts per workgroup of a single first-pass launch, at most
constexpr int sk1_row_blocks(int NB) { return NB <= 5 ? 2 : 1; }
// wavefronts per first-pass workgroup, at most: 16 (four per SIMD, at most
// 128 registers per lane) up to 13 column blocks, 12 for the widest tiles
// (more registers: three per SIMD); the two-block form launches at most 8
constexpr int sk1_max_waves(int NB) {
  return sk1_row_blocks(NB) == 2 ? 8 : (NB >= 14 ? 12 : 16);
}
// wavefronts per first-pass workgroup, at least: the Omega tile is staged
// in kSkMaxChunks 16-byte chunks per thread
constexpr int sk1_min_waves(int NB, bool bf) {
  return (16 * NB * (bf ? 4 : 8) + 64 * kSkMaxChunks - 1) / (64 * kSkMaxChunks) > 4
             ? (16 * NB * (bf ? 4 : 8) + 64 * kSkMaxChunks - 1) / (64 * kSkMaxChunks)
             : 4;
}
constexpr int sk2_col_blocks(int) { return 2; }
template <bool BF, int NB>
__global__ __launch_bounds__(64 * sk1_max_waves(NB)) void k_sk1(const float* __restrict__ A, int64_t n, int d,
                                              int64_t ld, int vec, const void* __restrict__ Olp,
                                              int ldo, float* __restrict__ T, int64_t ldt,
                                              int col0, int ncols, int64_t row0) {
  constexpr int NP = 16 * NB;
  constexpr int RB = sk1_row_blocks(NB);
  constexpr int TILE = NP * kOPad * (BF ? 2 : 4);
  __shared__ __attribute__((aligned(32))) char smem[2 * TILE];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nthr = blockDim.x;
  const int q = lane >> 4, m = lane & 15;
  const int64_t m0 = row0 + ((int64_t)blockIdx.x * (nthr >> 6) + wv) * 16 * RB;
  const int n0 = blockIdx.y * NP;
  f4 acc[RB][NB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = (f4)0.0f;
  constexpr int NCH = BF ? NP * 4 : NP * 8;   // 16-byte chunks of one Omega tile
  // staged chunks as separate values (an indexed array would go to scratch);
  // the host launches at least NCH / (64 kSkMaxChunks) wavefronts
  uint4 ob0, ob1, ob2, ob3;
  auto chunk = [&](int c) __attribute__((always_inline)) -> uint4& {
    return c == 0 ? ob0 : c == 1 ? ob1 : c == 2 ? ob2 : ob3;
  };
  auto load_omega = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < kSkMaxChunks; ++c) {
      const int e = tid + nthr * c;
      if (e < NCH) {
        if (BF) {
          const int nn = e >> 2, kk = (e & 3) * 8;
          chunk(c) = *reinterpret_cast<const uint4*>(static_cast<const __bf16*>(Olp) +
                                                     (int64_t)(n0 + nn) * ldo + k0 + kk);
        } else {
          const int nn = e >> 3, kk = (e & 7) * 4;
          chunk(c) = *reinterpret_cast<const uint4*>(static_cast<const float*>(Olp) +
                                                     (int64_t)(n0 + nn) * ldo + k0 + kk);
        }
      }
    }
  };
  auto store_omega = [&](char* buf) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < kSkMaxChunks; ++c) {
      const int e = tid + nthr * c;
      if (e < NCH) {
        if (BF) {
          const int nn = e >> 2, kk = (e & 3) * 8;
          *reinterpret_cast<uint4*>(reinterpret_cast<__bf16*>(buf) + nn * kOPad + kk) = chunk(c);
        } else {
          const int nn = e >> 3, kk = (e & 7) * 4;
          *reinterpret_cast<uint4*>(reinterpret_cast<float*>(buf) + nn * kOPad + kk) = chunk(c);
        }
      }
    }
  };
  f8 an[RB];
  auto load_a = [&](int k0) __attribute__((always_inline)) {
    const int kk = k0 + 8 * q;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t row = m0 + 16 * rb + m;
      an[rb] = (row < n && kk < d) ? load8(A + row * ld + kk, d - kk, vec) : (f8)0.0f;
    }
  };
  load_omega(0);
  load_a(0);
  store_omega(smem);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < d; k0 += kBK) {
    f8 af[RB];
    bf16x8 ab[RB];   // BF16: converted before the next step's loads are issued
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if constexpr (BF) ab[rb] = to_bf16(an[rb]);
      else af[rb] = an[rb];
    }
    const bool more = k0 + kBK < d;
    if (more) {
      load_omega(k0 + kBK);
      load_a(k0 + kBK);
    }
    const char* buf = smem + cur * TILE;
    // the Omega operand of column block nb + 1 is read from LDS while block
    // nb's products run; from kSkPipeNB column blocks on, group barriers keep
    // the scheduler from sinking each read to its products (DS reads = 0x100,
    // MFMA = 0x8)
    if constexpr (BF) {
      const __bf16* Os = reinterpret_cast<const __bf16*>(buf) + m * kOPad + 8 * q;
      bf16x8 bv = *reinterpret_cast<const bf16x8*>(Os);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf16x8 bn = bv;
        if (nb + 1 < NB) bn = *reinterpret_cast<const bf16x8*>(Os + (nb + 1) * 16 * kOPad);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          acc[rb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab[rb], bv, acc[rb][nb], 0, 0, 0);
        bv = bn;
      }
      if constexpr (NB >= kSkPipeNB) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
#pragma unroll
        for (int nb = 0; nb + 1 < NB; ++nb) {
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, RB, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, RB, 0);
      }
    } else {
      const float* Os = reinterpret_cast<const float*>(buf) + m * kOPad + 8 * q;
      f8 bv = *reinterpret_cast<const f8*>(Os);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        f8 bn = bv;
        if (nb + 1 < NB) bn = *reinterpret_cast<const f8*>(Os + (nb + 1) * 16 * kOPad);
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            acc[rb][nb] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(af[rb][s], bv[s], acc[rb][nb], 0, 0, 0);
        bv = bn;
      }
      if constexpr (NB >= kSkPipeNB) {
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
        for (int nb = 0; nb + 1 < NB; ++nb) {
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 8 * RB, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 8 * RB, 0);
      }
    }
    if (more) store_omega(smem + (cur ^ 1) * TILE);
    __syncthreads();
    cur ^= 1;
  }
  // 16x16 FP32 result layout: lane (q, m) holds rows 4 q + v of column m
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = n0 + nb * 16 + m;
      if (c >= ncols) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = m0 + 16 * rb + 4 * q + v;
        if (r < n) T[(int64_t)(col0 + c) * ldt + r] = acc[rb][nb][v];
      }
    }
}

// Ypart[s][c][j] = sum_{i in slice s} A[i][j] D[i] T[i][c]  (j < d, c < ncols).
// A workgroup of kSk2W wavefronts covers 16 JB kSk2W columns j of A and all
// NB sketch column blocks; wavefront w owns JB = 2 consecutive 16-column
// blocks of A (four per wavefront at small NB measured no faster).  Per K step
// of 32 rows i, (D o T) for the NB blocks is staged in double-buffered LDS
// (column-major, as T is stored; for BF16 as hi and lo parts, so only A is
// rounded to BF16) and shared by the wavefronts, while each wavefront reads
// its A^T operand straight from memory: lane (q, m) takes A[i0 + 8q + s][j]
// for s < 8, 64 contiguous bytes per 16 lanes, so A needs no transpose.
constexpr int kSk2W = 8;
constexpr int kTPad = 40;   // LDS pitch (elements) of a staged T column (16-byte rows)
template <bool BF, int NB>
__global__ __launch_bounds__(64 * kSk2W) void k_sk2(const float* __restrict__ A, int64_t n, int d,
                                                    int64_t ld, const double* __restrict__ D,
                                                    const float* __restrict__ T, int64_t ldt,
                                                    int col0, int ncols, int64_t slice,
                                                    float* __restrict__ Yp, int ldy) {
  constexpr int NP = 16 * NB;
  constexpr int JB = sk2_col_blocks(NB);
  constexpr int TILE = NP * kTPad * 4;   // one buffer: FP32 (D o T), or bf16 hi + lo
  constexpr int NT = 64 * kSk2W;
  __shared__ __attribute__((aligned(32))) char smem[2 * TILE];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int q = lane >> 4, m = lane & 15;
  const int j0 = blockIdx.x * 16 * JB * kSk2W + 16 * JB * wv;
  const int64_t i_beg = (int64_t)blockIdx.y * slice;
  const int64_t i_end = (i_beg + slice < n) ? i_beg + slice : n;
  f4 acc[JB][NB];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[jb][nb] = (f4)0.0f;
  // (D o T) tile: NP columns x 32 rows, thread tid stages 4 consecutive rows
  // of one column per item: items e = tid + NT u, column e >> 3, rows 4 (e & 7)
  constexpr int NIT = (NP * 8 + NT - 1) / NT;
  f4 tv[NIT];
  auto load_t = [&](int64_t i0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int e = tid + NT * u;
      const int c = e >> 3, rr = (e & 7) * 4;
      f4 x = (f4)0.0f;
      if (e < NP * 8 && c < ncols) {
        const int64_t ib = i0 + rr;
        const float* src = T + (int64_t)(col0 + c) * ldt + ib;
        if (ib + 3 < i_end) {
          x = *reinterpret_cast<const f4*>(src);   // ldt and ib are multiples of 4
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (ib + v < i_end) x[v] = src[v];
        }
        if (D != nullptr) {
#pragma unroll
          for (int v = 0; v < 4; ++v) x[v] *= (ib + v < i_end) ? (float)D[ib + v] : 0.0f;
        }
      }
      tv[u] = x;
    }
  };
  auto store_t = [&](char* buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int e = tid + NT * u;
      if (e < NP * 8) {
        const int c = e >> 3, rr = (e & 7) * 4;
        if (BF) {
          __bf16* hi = reinterpret_cast<__bf16*>(buf);
          __bf16* lo = hi + NP * kTPad;
          bf16x4 h, l;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            h[v] = (__bf16)tv[u][v];
            l[v] = (__bf16)(tv[u][v] - (float)h[v]);
          }
          *reinterpret_cast<bf16x4*>(hi + c * kTPad + rr) = h;
          *reinterpret_cast<bf16x4*>(lo + c * kTPad + rr) = l;
        } else {
          *reinterpret_cast<f4*>(reinterpret_cast<float*>(buf) + c * kTPad + rr) = tv[u];
        }
      }
    }
  };
  // A^T operand: lane (q, m), j block jb: A[i0 + 8q + s][j0 + 16 jb + m], s < 8
  f8 an[JB];
  auto load_a = [&](int64_t i0) __attribute__((always_inline)) {
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
      const int j = j0 + 16 * jb + m;
      const int64_t ib = i0 + 8 * q;
#pragma unroll
      for (int s = 0; s < 8; ++s)
        an[jb][s] = (j < d && ib + s < i_end) ? A[(ib + s) * ld + j] : 0.0f;
    }
  };
  if (i_beg < i_end) {
    load_t(i_beg);
    load_a(i_beg);
    store_t(smem);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t i0 = i_beg; i0 < i_end; i0 += kBK) {
    f8 a[JB];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) a[jb] = an[jb];
    const bool more = i0 + kBK < i_end;
    if (more) {
      load_t(i0 + kBK);
      load_a(i0 + kBK);
    }
    const char* buf = smem + cur * TILE;
    if constexpr (BF) {
      bf16x8 b[JB];
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) b[jb] = to_bf16(a[jb]);
      const __bf16* hi = reinterpret_cast<const __bf16*>(buf);
      const __bf16* lo = hi + NP * kTPad;
      // block nb + 1's operands are read while block nb's products run
      const int off0 = m * kTPad + 8 * q;
      bf16x8 th = *reinterpret_cast<const bf16x8*>(hi + off0);
      bf16x8 tl = *reinterpret_cast<const bf16x8*>(lo + off0);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf16x8 nh = th, nl = tl;
        if (nb + 1 < NB) {
          nh = *reinterpret_cast<const bf16x8*>(hi + off0 + (nb + 1) * 16 * kTPad);
          nl = *reinterpret_cast<const bf16x8*>(lo + off0 + (nb + 1) * 16 * kTPad);
        }
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          acc[jb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[jb], th, acc[jb][nb], 0, 0, 0);
          acc[jb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[jb], tl, acc[jb][nb], 0, 0, 0);
        }
        th = nh;
        tl = nl;
      }
      if constexpr (NB >= kSkPipeNB) {
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
        for (int nb = 0; nb + 1 < NB; ++nb) {
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 2 * JB, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 2 * JB, 0);
      }
    } else {
      // the (D o T) operand of block nb + 1 is read from LDS while block nb's
      // products run (two wavefronts per SIMD hide little latency otherwise)
      const float* Ts = reinterpret_cast<const float*>(buf) + m * kTPad + 8 * q;
      f8 bv = *reinterpret_cast<const f8*>(Ts);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        f8 bn = bv;
        if (nb + 1 < NB) bn = *reinterpret_cast<const f8*>(Ts + (nb + 1) * 16 * kTPad);
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
            acc[jb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[jb][s], bv[s], acc[jb][nb], 0, 0, 0);
        bv = bn;
      }
      // keep that order from kSkPipeNB column blocks on: the scheduler
      // otherwise sinks each read to its products (DS reads = 0x100, MFMA = 0x8)
      if constexpr (NB >= kSkPipeNB) {
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
        for (int nb = 0; nb + 1 < NB; ++nb) {
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 8 * JB, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 8 * JB, 0);
      }
    }
    if (more) store_t(smem + (cur ^ 1) * TILE);
    __syncthreads();
    cur ^= 1;
  }
  float* Ys = Yp + (int64_t)blockIdx.y * ncols * ldy;
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = nb * 16 + m;
      if (c >= ncols) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + 16 * jb + 4 * q + v;
        if (j < d) Ys[(int64_t)c * ldy + j] = acc[jb][nb][v];
      }
    }
}

// Mb(i, r0 + j) = sum_k T(k, i) D_k T(k, r0 + j), i < r1, j < m: the FP64
// core matrix T^T D T of the FP32/BF16 forms (FP32 T; each product is exact
// in FP64).  Workgroup g sums the rows k of one contiguous slice on the FP64
// matrix cores: the slice's T rows, 32 at a time and all r1 (+ padding)
// columns, are staged in double-buffered LDS in T's own column-major order,
// and wavefront w owns the output blocks w, w + kGtW, ... of the list of
// 16 x 16 blocks (row-major; only blocks bi <= bj when the product is the
// square r0 = 0, m = r1 one).  Partial sums go to Wp[g][block][16 x 16];
// k_gram_t_reduce adds them in slice order.
typedef double d4g __attribute__((ext_vector_type(4)));
constexpr int kGtW = 8;        // wavefronts per workgroup
constexpr int kGtMaxB = 12;    // output blocks per wavefront, at most
constexpr int kGtMaxC = 272;   // staged columns: r1 + padding
constexpr int kGtPad = 36;     // LDS pitch (floats) of a staged column

__device__ __forceinline__ void gram_block(int b, int RB, int CB, bool sym, int* bi, int* bj) {
  if (!sym) {
    *bi = b / CB;
    *bj = b % CB;
    return;
  }
  int i = 0;
  while (b >= RB - i) {
    b -= RB - i;
    ++i;
  }
  *bi = i;
  *bj = i + b;
}

__global__ __launch_bounds__(64 * kGtW) void k_gram_t(const float* __restrict__ T, int64_t ldt,
                                                      int64_t n, const double* __restrict__ D,
                                                      int r1, int r0, int m, int sym,
                                                      int64_t slice, double* __restrict__ Wp) {
  __shared__ __attribute__((aligned(16))) float Ts[2][kGtMaxC][kGtPad];
  __shared__ double Ds[2][32];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int fi = lane & 15, fk = lane >> 4;
  const int RB = (r1 + 15) / 16, CB = (m + 15) / 16;
  const int nblk = sym ? RB * (RB + 1) / 2 : RB * CB;
  const int ncol = max(16 * RB, r0 + 16 * CB);   // staged columns (zero past r1)
  int bi[kGtMaxB], bj[kGtMaxB];
#pragma unroll
  for (int t = 0; t < kGtMaxB; ++t) {
    const int b = wv + kGtW * t;
    int x = 0, y = 0;
    if (b < nblk) gram_block(b, RB, CB, sym != 0, &x, &y);
    // wavefront-uniform: keep them in scalar registers
    bi[t] = __builtin_amdgcn_readfirstlane(x);
    bj[t] = __builtin_amdgcn_readfirstlane(y);
  }
  d4g acc[kGtMaxB];
#pragma unroll
  for (int t = 0; t < kGtMaxB; ++t) acc[t] = (d4g)0.0;
  const int64_t kb = (int64_t)blockIdx.x * slice;
  const int64_t ke = (kb + slice < n) ? kb + slice : n;
  // staging items: (column c, 4-row group g4), 8 per column
  constexpr int NIT = (kGtMaxC * 8 + 64 * kGtW - 1) / (64 * kGtW);
  f4 tv[NIT];
  double dv = 1.0;
  auto load = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int e = tid + 64 * kGtW * u;
      const int c = e >> 3, g4 = (e & 7) * 4;
      f4 x = (f4)0.0f;
      if (c < r1 && e < ncol * 8) {
        const int64_t k = k0 + g4;
        const float* src = T + (int64_t)c * ldt + k;
        if (k + 3 < ke) {
          x = *reinterpret_cast<const f4*>(src);   // ldt and k are multiples of 4
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (k + v < ke) x[v] = src[v];
        }
      }
      tv[u] = x;
    }
    if (tid < 32) dv = (D != nullptr && k0 + tid < ke) ? D[k0 + tid] : 1.0;
  };
  auto store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int e = tid + 64 * kGtW * u;
      const int c = e >> 3, g4 = (e & 7) * 4;
      if (e < ncol * 8) *reinterpret_cast<f4*>(&Ts[buf][c][g4]) = tv[u];
    }
    if (tid < 32) Ds[buf][tid] = dv;
  };
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += 32) {
    const bool more = k0 + 32 < ke;
    if (more) load(k0 + 32);
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4) {
      const double w = Ds[cur][kk + fk];
#pragma unroll
      for (int t = 0; t < kGtMaxB; ++t) {
        if (wv + kGtW * t < nblk) {
          const double a = (double)Ts[cur][16 * bi[t] + fi][kk + fk] * w;
          const double b = (double)Ts[cur][r0 + 16 * bj[t] + fi][kk + fk];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
      }
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  // FP64 16x16 result layout: lane (fk, fi) holds rows fk + 4 v of column fi
#pragma unroll
  for (int t = 0; t < kGtMaxB; ++t) {
    const int b = wv + kGtW * t;
    if (b < nblk) {
      double* o = Wp + ((int64_t)blockIdx.x * nblk + b) * 256;
#pragma unroll
      for (int v = 0; v < 4; ++v) o[(fk + 4 * v) * 16 + fi] = acc[t][v];
    }
  }
}

// Mb[i * ldm + r0 + j] = sum over the G slices of the partial blocks (slice
// order); with sym the lower triangle reads the transposed upper block.
__global__ void k_gram_t_reduce(const double* __restrict__ Wp, int G, int r1, int r0, int m,
                                int sym, double* __restrict__ Mb, int ldm) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r1 * m) return;
  const int i = (int)(e / m), j = (int)(e % m);
  const int RB = (r1 + 15) / 16, CB = (m + 15) / 16;
  const int nblk = sym ? RB * (RB + 1) / 2 : RB * CB;
  int bi = i >> 4, bj = j >> 4, ii = i & 15, jj = j & 15;
  if (sym && bi > bj) {
    const int t = bi; bi = bj; bj = t;
    const int u = ii; ii = jj; jj = u;
  }
  const int b = sym ? bi * RB - bi * (bi - 1) / 2 + (bj - bi) : bi * CB + bj;
  // eight interleaved partial sums (slices g = u mod 8), combined in a fixed
  // order: eight loads in flight, the same result on every call
  const double* src = Wp + (int64_t)b * 256 + ii * 16 + jj;
  const int64_t step = (int64_t)nblk * 256;
  double a[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u] = 0.0;
  int g = 0;
  for (; g + 7 < G; g += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += src[(int64_t)(g + u) * step];
  }
  for (; g < G; ++g) a[0] += src[(int64_t)g * step];
  Mb[(int64_t)i * ldm + r0 + j] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Launch shape of k_gram_t: usable when ceil(blocks / kGtW) <= kGtMaxB and
// the staged columns fit; returns the partial-buffer bytes (0 = not usable).
struct GramTShape {
  int G, nblk;
  int64_t slice;
  size_t wp_b;
};
GramTShape gram_t_shape(int64_t n, int r1, int r0, int m, int num_cu) {
  GramTShape g{0, 0, 0, 0};
  const bool sym = (r0 == 0 && m == r1);
  const int RB = (r1 + 15) / 16, CB = (m + 15) / 16;
  const int nblk = sym ? RB * (RB + 1) / 2 : RB * CB;
  const int ncol = std::max(16 * RB, r0 + 16 * CB);
  if ((nblk + kGtW - 1) / kGtW > kGtMaxB || ncol > kGtMaxC) return g;
  g.nblk = nblk;
  g.G = (int)std::max<int64_t>(1, std::min<int64_t>(num_cu, (n + 31) / 32));
  g.slice = ((n + g.G - 1) / g.G + 31) / 32 * 32;
  g.G = (int)((n + g.slice - 1) / g.slice);
  g.wp_b = align_up(sizeof(double) * (size_t)g.G * nblk * 256);
  return g;
}

// Y(:, col0 + c) = sum_s Ypart[s][c] + coef * Omega(:, col0 + c)   (FP64)
__global__ void k_sk2_reduce(const float* __restrict__ Yp, int S, int ncols, int ldy, int d,
                             const double* __restrict__ Om, double coef, double* __restrict__ Y,
                             int col0) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)ncols * d) return;
  const int c = (int)(e / d), j = (int)(e % d);
  double s = 0.0;
  for (int z = 0; z < S; ++z) s += (double)Yp[((int64_t)z * ncols + c) * ldy + j];
  const int64_t o = (int64_t)(col0 + c) * d + j;
  Y[o] = s + coef * Om[o];
}

// *out = max over i, j of |G(i, j) - [i == j]| for the r x r row-major G
// (one workgroup; NaN propagates as a failure)
__global__ __launch_bounds__(1024) void k_orth_err(const double* __restrict__ G, int r,
                                                   double* __restrict__ out) {
  __shared__ double sh[16];
  double m = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)r * r; e += 1024) {
    const int64_t i = e / r, j = e % r;
    const double v = fabs(G[e] - (i == j ? 1.0 : 0.0));
    m = (v > m || v != v) ? v : m;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = (o > m || o != o) ? o : m;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int k = 1; k < 16; ++k) t = (sh[k] > t || sh[k] != sh[k]) ? sh[k] : t;
    *out = t;
  }
}

// Y(:, c) = T(:, c) + coef * Omega(:, c) in FP64, c < m (T: FP32, pitch ldt)
__global__ void k_sym_y(const float* __restrict__ T, int64_t ldt, int d, int m,
                        const double* __restrict__ Om, double coef, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)m * d) return;
  const int c = (int)(e / d), j = (int)(e % d);
  Y[e] = (double)T[(int64_t)c * ldt + j] + coef * Om[e];
}

// Round the FP64 Omega block to the sketch precision: the low-precision copy
// (rows = columns, pitch ldo, zero padded to nrows_pad x ldo) and the FP64
// value of the rounded entries written back into Omega.
template <bool BF>
__global__ void k_round_omega(double* __restrict__ Om, int d, int m, void* __restrict__ lp,
                              int ldo, int nrows_pad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nrows_pad * ldo) return;
  const int c = (int)(e / ldo), j = (int)(e % ldo);
  double v = 0.0;
  if (c < m && j < d) v = Om[(int64_t)c * d + j];
  if (BF) {
    const __bf16 b = (__bf16)(float)v;
    static_cast<__bf16*>(lp)[e] = b;
    if (c < m && j < d) Om[(int64_t)c * d + j] = (double)(float)b;
  } else {
    const float f = (float)v;
    static_cast<float*>(lp)[e] = f;
    if (c < m && j < d) Om[(int64_t)c * d + j] = (double)f;
  }
}

// y = x + a * z elementwise (n entries)
__global__ void k_axpy(int64_t n, const double* __restrict__ x, double a,
                       const double* __restrict__ z, double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) y[e] = x[e] + a * z[e];
}

// M = 0.5 (X + X^T) + nu * Gam  (r x r, row-major)
__global__ void k_shift_sym(const double* __restrict__ X, const double* __restrict__ Gam,
                            double nu, int r, double* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e / r), j = (int)(e % r);
  M[e] = 0.5 * (X[(int64_t)i * r + j] + X[(int64_t)j * r + i]) + nu * Gam[e];
}

// M = G - mu I (r x r)
__global__ void k_sub_diag(const double* __restrict__ G, int r, double mu,
                           double* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e / r), j = (int)(e % r);
  M[e] = G[e] - (i == j ? mu : 0.0);
}

// mirror the upper-left block's new columns: M[c][i] = M[i][c] for c >= c0
__global__ void k_mirror_cols(double* __restrict__ M, int ld, int c0, int r) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * (r - c0)) return;
  const int i = (int)(e / (r - c0)), c = c0 + (int)(e % (r - c0));
  if (i < c0) M[(int64_t)c * ld + i] = M[(int64_t)i * ld + c];
}

__global__ void k_lambda(const double* __restrict__ sig2, double nu, int r,
                         double* __restrict__ lam) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < r) lam[i] = fmax(0.0, sig2[i] - nu);
}

__global__ void k_to_f32(const double* __restrict__ x, int64_t n, float* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) y[e] = (float)x[e];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

struct CoreWs {
  double *GY, *GO, *M, *Cinv, *Bm, *G, *W, *sig2, *jac, *split, *scal;
  int* ints;
  size_t split_elems;
};

size_t core_split_elems(int64_t d, int r) {
  return std::max<size_t>((size_t)16 * r * r, (size_t)4 * d * std::min(r, 64));
}

size_t core_ws_bytes_of(int64_t d, int r) {
  const size_t rr = align_up(sizeof(double) * (size_t)r * r);
  const size_t dr = align_up(sizeof(double) * (size_t)d * r);
  const size_t jac = align_up(sizeof(double) * jacobi_ws_doubles(r));
  const size_t split = align_up(sizeof(double) * core_split_elems(d, r));
  return 6 * rr + dr + jac + split + align_up(sizeof(double) * 1024) + 4096 + 4096;
}

nys_status core_workspace(nys_ctx ctx, int64_t d, int r, CoreWs* w) {
  const size_t rr = align_up(sizeof(double) * (size_t)r * r);
  const size_t dr = align_up(sizeof(double) * (size_t)d * r);
  const size_t jac = align_up(sizeof(double) * jacobi_ws_doubles(r));
  w->split_elems = core_split_elems(d, r);
  const size_t split = align_up(sizeof(double) * w->split_elems);
  NYS_TRY(ctx->core_ws.reserve(core_ws_bytes_of(d, r)));
  char* p = static_cast<char*>(ctx->core_ws.ptr);
  auto take = [&](size_t b) { char* q = p; p += b; return reinterpret_cast<double*>(q); };
  w->GY = take(rr);
  w->GO = take(rr);
  w->M = take(rr);
  w->Cinv = take(rr);
  w->G = take(rr);
  w->W = take(rr);
  w->Bm = take(dr);
  w->jac = take(jac);
  w->split = take(split);
  w->sig2 = take(align_up(sizeof(double) * 1024));
  w->scal = take(4096);
  w->ints = reinterpret_cast<int*>(take(4096));
  return NYS_OK;
}

nys_status read_back(nys_ctx ctx, const void* dev, size_t bytes, void* host) {
  // through the pinned area below the polling slots, in pieces if needed
  const char* src = static_cast<const char*>(dev);
  char* dst = static_cast<char*>(host);
  while (bytes > 0) {
    const size_t n = bytes < kPollOffset ? bytes : kPollOffset;
    NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, src, n, hipMemcpyDeviceToHost, ctx->stream));
    NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
    std::memcpy(dst, ctx->host_pinned, n);
    src += n;
    dst += n;
    bytes -= n;
  }
  return NYS_OK;
}

double eps_of(double x, int mbits) {
  int e = 0;
  (void)std::frexp(x, &e);   // x = f 2^e, f in [0.5, 1)
  return std::ldexp(1.0, e - 1 - mbits);
}

// Thin QR of a block by CholeskyQR (Gram -> Cholesky -> Q = X R^-1), in
// place on Om (d x m, column-major).  After each pass the Gram of the result
// is formed and max |Q^T Q - I| read back; a second pass runs only when it
// exceeds 1e-14 m.  A Gaussian block with d well above m has condition number
// near (1 + sqrt(m/d)) / (1 - sqrt(m/d)) (below 3 for d >= 4m), so one pass
// leaves Q orthonormal to about 1e-15 and the second pass (CholeskyQR2) is
// needed only for nearly square or ill-conditioned blocks.  The Nystrom
// approximation depends on range(Omega) only; the shifted core uses the
// computed Omega^T Omega, not the identity.  *err_out (optional): the final
// max |Q^T Q - I|.  tmp: d x m scratch (w.Bm when NULL)
nys_status orthonormalize(nys_ctx ctx, double* Om, int64_t d, int m, const CoreWs& w,
                          double* tmp = nullptr, double* err_out = nullptr) {
  hipStream_t st = ctx->stream;
  if (tmp == nullptr) tmp = w.Bm;
  // the Cholesky failure flag in ints[0] (never reset between the passes:
  // after a failed factorisation the remaining kernels run on meaningless
  // values, their indexing does not depend on them, and the result is
  // discarded) and the orthogonality error as a double at ints[2..3], read
  // back together
  double* err_dev = reinterpret_cast<double*>(w.ints + 2);
  NYS_TRY_HIP(hipMemsetAsync(w.ints, 0, sizeof(int), st));
  NYS_TRY(gemm64(st, m, m, (int)d, Om, false, d, 1, Om, false, 1, d, w.M, m, 1, 1.0, 0.0,
                 w.split, w.split_elems));
  double err = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    NYS_TRY(chol_upper(st, w.M, m, m, w.ints));
    NYS_TRY(trinv_upper(st, w.M, m, m, w.Cinv, m));
    // Bm = Om Rinv  (d x m col-major), then copy back
    NYS_TRY(gemm64(st, (int)d, m, m, Om, false, 1, d, w.Cinv, false, m, 1, tmp, 1, d, 1.0, 0.0,
                   w.split, w.split_elems));
    NYS_TRY_HIP(hipMemcpyAsync(Om, tmp, sizeof(double) * d * m, hipMemcpyDeviceToDevice, st));
    // Q^T Q: the acceptance test, and the next pass's Gram
    NYS_TRY(gemm64(st, m, m, (int)d, Om, false, d, 1, Om, false, 1, d, w.M, m, 1, 1.0, 0.0,
                   w.split, w.split_elems));
    hipLaunchKernelGGL(k_orth_err, dim3(1), dim3(1024), 0, st, w.M, m, err_dev);
    unsigned char hb[16];
    NYS_TRY(read_back(ctx, w.ints, sizeof(hb), hb));
    int fail = 0;
    std::memcpy(&fail, hb, sizeof(int));
    std::memcpy(&err, hb + 8, sizeof(double));
    if (fail) return NYS_ERR_NOT_SPD;   // block without full column rank
    if (err <= 1e-14 * m) break;
  }
  if (err_out) *err_out = err;
  return NYS_OK;
}

// The FP64 core of Algorithm RandNysAppx on the factor's current sketch.
// test_mu >= 0: stop after forming G = B^T B when G - (nu + test_mu) I is
// positive definite (its Cholesky succeeds), i.e. when every retained
// eigenvalue max(0, sigma^2 - nu) exceeds test_mu; *above = 1 and the factor's
// U and lambda are left unset.  Otherwise (or test_mu < 0) the
// eigendecomposition is completed and *above = 0.
nys_status nys_core(nys_ctx ctx, nys_factor F, double test_mu, int* above) {
  if (above) *above = 0;
  hipStream_t st = ctx->stream;
  const int64_t d = F->d;
  const int r = F->r;
  CoreWs w;
  NYS_TRY(core_workspace(ctx, d, r, &w));
  const double* Y = F->Y.as<double>();
  const double* Om = F->Omega.as<double>();
  // ||Y||_2 = sqrt(lambda_max(Y^T Y))
  NYS_TRY(gemm64(st, r, r, (int)d, Y, false, d, 1, Y, false, 1, d, w.GY, r, 1, 1.0, 0.0, w.split,
                 w.split_elems));
  NYS_TRY(power_iter(st, w.GY, r, r, 300, w.scal));
  // Omega^T Omega
  NYS_TRY(gemm64(st, r, r, (int)d, Om, false, d, 1, Om, false, 1, d, w.GO, r, 1, 1.0, 0.0,
                 w.split, w.split_elems));
  // base core matrix Omega^T Y (FP64 form; also for an explicit symmetric
  // matrix) or the stored T^T D T + c Omega^T Omega
  const double* base;
  if (F->prec == NYS_F64 || F->sym || F->sparse) {
    NYS_TRY(gemm64(st, r, r, (int)d, Om, false, d, 1, Y, false, 1, d, w.G, r, 1, 1.0, 0.0,
                   w.split, w.split_elems));
    base = w.G;
  } else {
    base = F->Mbase.as<double>();
  }
  double lmax = 0.0;
  NYS_TRY(read_back(ctx, w.scal, sizeof(double), &lmax));
  if (!(lmax > 0.0) || !std::isfinite(lmax)) return NYS_ERR_NONFINITE;
  double nu = std::sqrt((double)d) * eps_of(std::sqrt(lmax), F->mantissa_bits);
  int attempt = 0;
  for (;; ++attempt) {
    hipLaunchKernelGGL(k_shift_sym, dim3(blocks((int64_t)r * r)), dim3(256), 0, st, base, w.GO,
                       nu, r, w.M);
    NYS_TRY_HIP(hipMemsetAsync(w.ints, 0, sizeof(int), st));
    NYS_TRY(chol_upper(st, w.M, r, r, w.ints));
    int fail = 0;
    NYS_TRY(read_back(ctx, w.ints, sizeof(int), &fail));
    if (!fail) break;
    if (attempt == 3) return NYS_ERR_NOT_SPD;
    nu *= 10.0;
  }
  NYS_TRY(trinv_upper(st, w.M, r, r, w.Cinv, r));
  // B = (Y + nu Omega) C^-1 : two GEMMs into Bm (d x r col-major)
  NYS_TRY(gemm64(st, (int)d, r, r, Y, false, 1, d, w.Cinv, false, r, 1, w.Bm, 1, d, 1.0, 0.0,
                 w.split, w.split_elems));
  NYS_TRY(gemm64(st, (int)d, r, r, Om, false, 1, d, w.Cinv, false, r, 1, w.Bm, 1, d, nu, 1.0,
                 w.split, w.split_elems));
  // G = B^T B, eigendecomposition G = V Sigma^2 V^T
  NYS_TRY(gemm64(st, r, r, (int)d, w.Bm, false, d, 1, w.Bm, false, 1, d, w.G, r, 1, 1.0, 0.0,
                 w.split, w.split_elems));
  if (test_mu >= 0.0) {
    // inertia of G - (nu + test_mu) I through one Cholesky attempt
    hipLaunchKernelGGL(k_sub_diag, dim3(blocks((int64_t)r * r)), dim3(256), 0, st, w.G, r,
                       nu + test_mu, w.M);
    NYS_TRY_HIP(hipMemsetAsync(w.ints, 0, sizeof(int), st));
    NYS_TRY(chol_upper(st, w.M, r, r, w.ints));
    int fail = 0;
    NYS_TRY(read_back(ctx, w.ints, sizeof(int), &fail));
    if (!fail) {
      F->nu = nu;
      if (above) *above = 1;
      return NYS_OK;
    }
  }
  int sweeps = 0;
  // Rebuild with the previous factor's U at hand: V0 = orthonormalised
  // B^T U_prev spans nearly the eigenvectors of G when the operator moved
  // little (the logistic weights between refreshes), so the eigensolver
  // starts from G' = V0^T G V0, nearly diagonal, and needs a few sweeps
  // instead of about ten.  The result is G's eigendecomposition either way;
  // if V0 is not of full rank the solver starts from the identity.
  const double* V0 = nullptr;
  const double* Gj = w.G;
  if (F->basis_hint != nullptr) {
    double* Vb = w.GO;   // r x r column-major (free after the shifted Cholesky)
    NYS_TRY(gemm64(st, r, r, (int)d, w.Bm, false, d, 1, F->basis_hint, false, 1, d, Vb, 1, r,
                   1.0, 0.0, w.split, w.split_elems));
    double err = 0.0;
    nys_status so = orthonormalize(ctx, Vb, r, r, w, w.W, &err);
    // CholeskyQR is exact to rounding only for a well-conditioned V0:
    // accept the basis when max |V0^T V0 - I| <= 1e-13 r
    if (so == NYS_OK && !(err <= 1e-13 * r)) so = NYS_ERR_NOT_SPD;
    if (so == NYS_OK) {
      // G' = V0^T (G V0): T1 (column-major) in GY, G' (row-major) in M
      NYS_TRY(gemm64(st, r, r, r, w.G, false, r, 1, Vb, false, 1, r, w.GY, 1, r, 1.0, 0.0,
                     w.split, w.split_elems));
      NYS_TRY(gemm64(st, r, r, r, Vb, false, r, 1, w.GY, false, 1, r, w.M, r, 1, 1.0, 0.0,
                     w.split, w.split_elems));
      V0 = Vb;
      Gj = w.M;
    } else if (so != NYS_ERR_NOT_SPD) {
      return so;
    }
  }
  NYS_TRY(jacobi_eig(st, Gj, r, r, w.jac, w.ints + 16, 40, ctx->host_pinned,
                     ctx->host_pinned_dev, &ctx->poll_seq, w.sig2, w.W, r, &sweeps, V0));
  if (getenv("NYSADMM_VERBOSE"))
    fprintf(stderr, "[nysadmm] eigensolver r=%d sweeps=%d start=%s\n", r, sweeps,
            V0 != nullptr ? "previous-basis" : (F->basis_hint != nullptr ? "identity-fallback"
                                                                          : "identity"));
  // U = B V Sigma^-1
  NYS_TRY(F->U.reserve(sizeof(double) * d * r));
  NYS_TRY(gemm64(st, (int)d, r, r, w.Bm, false, 1, d, w.W, false, r, 1, F->U.as<double>(), 1, d,
                 1.0, 0.0, w.split, w.split_elems));
  NYS_TRY(F->lam.reserve(sizeof(double) * r));
  hipLaunchKernelGGL(k_lambda, dim3(blocks(r)), dim3(256), 0, st, w.sig2, nu, r,
                     F->lam.as<double>());
  F->lam_host.resize(r);
  NYS_TRY(read_back(ctx, F->lam.ptr, sizeof(double) * r, F->lam_host.data()));
  for (double v : F->lam_host)
    if (!std::isfinite(v)) return NYS_ERR_NONFINITE;
  F->nu = nu;
  F->use_u32 = (F->prec != NYS_F64);
  if (F->use_u32) {
    NYS_TRY(F->U32.reserve(sizeof(float) * d * r));
    hipLaunchKernelGGL(k_to_f32, dim3(blocks(d * r)), dim3(256), 0, st, F->U.as<double>(), d * r,
                       F->U32.as<float>());
  }
  NYS_TRY_HIP(hipGetLastError());
  return NYS_OK;
}

nys_status grow(nys::DevBuf& b, size_t old_bytes, size_t new_bytes, hipStream_t st) {
  if (b.bytes >= new_bytes && b.ptr != nullptr) return NYS_OK;
  nys::DevBuf nb;
  NYS_TRY(nb.reserve(new_bytes));
  if (old_bytes > 0 && b.ptr != nullptr)
    NYS_TRY_HIP(hipMemcpyAsync(nb.ptr, b.ptr, old_bytes, hipMemcpyDeviceToDevice, st));
  b.release();   // reused only after the queued copy has run
  b = nb;
  return NYS_OK;
}

#define NYS_NB_SWITCH(NB, X) \
  switch (NB) {                 \
    case 1: X(1); break;        \
    case 2: X(2); break;        \
    case 3: X(3); break;        \
    case 4: X(4); break;        \
    case 5: X(5); break;        \
    case 6: X(6); break;        \
    case 7: X(7); break;        \
    case 8: X(8); break;        \
    case 9: X(9); break;        \
    case 10: X(10); break;      \
    case 11: X(11); break;      \
    case 12: X(12); break;      \
    case 13: X(13); break;      \
    case 14: X(14); break;      \
    case 15: X(15); break;      \
    default: X(16); break;      \
  }

// Rows [row0, row1) of T, workgroups of NW wavefronts.
template <bool BF>
nys_status launch_sk1_rows(int NB, int NW, const nys_dense& A, int vec, const void* Olp, int ldo,
                           float* T, int64_t ldt, int col0, int ncols, int npass, int64_t row0,
                           int64_t row1, hipStream_t st) {
  if (row1 <= row0) return NYS_OK;
  const int rows = 16 * NW * sk1_row_blocks(NB);
  dim3 grid((unsigned)((row1 - row0 + rows - 1) / rows), npass);
  const float* a = static_cast<const float*>(A.data);
#define NYS_SK1(N)                                                                              \
  hipLaunchKernelGGL((k_sk1<BF, N>), grid, dim3(64 * NW), 0, st, a, row1, (int)A.d, A.ld, vec, \
                     Olp, ldo, T, ldt, col0, ncols, row0)
  NYS_NB_SWITCH(NB, NYS_SK1)
#undef NYS_SK1
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

// T = A Omega_lp over all rows: the first launch takes rows [0, rows1) with NW
// wavefronts per workgroup, a second one the rest with NW2.
template <bool BF>
nys_status launch_sk1(int NB, int NW, int64_t rows1, int NW2, const nys_dense& A, int vec,
                      const void* Olp, int ldo, float* T, int64_t ldt, int col0, int ncols,
                      int npass, hipStream_t st) {
  const int64_t r1 = std::min<int64_t>(rows1, A.n);
  NYS_TRY(launch_sk1_rows<BF>(NB, NW, A, vec, Olp, ldo, T, ldt, col0, ncols, npass, 0, r1, st));
  return launch_sk1_rows<BF>(NB, NW2, A, vec, Olp, ldo, T, ldt, col0, ncols, npass, r1, A.n, st);
}

template <bool BF>
nys_status launch_sk2(int NB, const nys_dense& A, const double* D, const float* T, int64_t ldt,
                      int col0, int ncols, int64_t slice, int S, float* Yp, int ldy,
                      hipStream_t st) {
  const int cols = 16 * kSk2W * sk2_col_blocks(NB);
  dim3 grid((unsigned)((A.d + cols - 1) / cols), S);
  const float* a = static_cast<const float*>(A.data);
#define NYS_SK2(N)                                                                              \
  hipLaunchKernelGGL((k_sk2<BF, N>), grid, dim3(64 * kSk2W), 0, st, a, A.n, (int)A.d, A.ld, D,  \
                     T, ldt, col0, ncols, slice, Yp, ldy)
  NYS_NB_SWITCH(NB, NYS_SK2)
#undef NYS_SK2
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

// Launch shape and temporaries of the FP32/BF16-MFMA sketch of m columns.
struct Sk32Shape {
  int ldo, NB, NP, npass, nrows_pad, ldy, S, NW, NW2;
  int64_t rows1;   // rows of the first-pass launch with NW wavefronts; NW2 takes the rest
  int64_t ldt, slice;
  size_t olp_b, yp_b;
};
// Wavefronts per workgroup of the first pass: each takes a 16-row block, and
// the count is chosen so that the last round of workgroups fills the device
// as fully as possible (rounds = ceil(workgroups / resident workgroups)).
int sk1_waves(int64_t n, int NB, bool bf, int num_cu) {
  const int rb = sk1_row_blocks(NB);
  const int64_t nblk = (n + 16 * rb - 1) / (16 * rb);
  const size_t lds = 2 * (size_t)16 * NB * kOPad * (bf ? 2 : 4);
  const int by_lds = std::max<int>(1, (int)((160 * 1024) / lds));
  const int lo = sk1_min_waves(NB, bf);
  const int hi = rb == 2 ? 8 : (NB >= 14 ? 12 : kSk1MaxW);
  const int waves_cu = (rb == 2 || NB >= 14) ? 12 : 16;       // 3 or 4 resident per SIMD
  int best = hi;
  double best_eff = -1.0;
  for (int nw = std::min(lo, hi); nw <= hi; ++nw) {
    const int per_cu = std::max(1, std::min(by_lds, waves_cu / nw));
    const int64_t slots = (int64_t)per_cu * num_cu;
    const int64_t tiles = (nblk + nw - 1) / nw;
    const int64_t rounds = (tiles + slots - 1) / slots;
    const double eff = (double)tiles / (double)(rounds * slots);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = nw;
    }
  }
  return best;
}

// Launch plan of the first pass (T = A Omega), from measured rates on
// 100000 x 4000:
//  * FP32, one 16-row block per wavefront (more than 5 column blocks): the
//    matrix cores bound it, so every SIMD should hold the same number of
//    wavefronts until the rows run out.  Full rounds of 16-wavefront
//    workgroups (one per CU, four per SIMD), then the remaining blocks in
//    one more launch spread over at most one workgroup per CU (at most three
//    wavefronts per SIMD).  One launch leaves 13-wavefront workgroups with
//    four wavefronts on one SIMD and three on the others, or a second round
//    of 16-wavefront workgroups on half of the CUs: 1.81 ms against 1.65 ms
//    at 208 columns, 1.16 against 1.08 at 112.
//  * BF16, one block per wavefront: bound by the latency of the A loads;
//    seven-wavefront workgroups (two per CU) measured fastest (0.53 ms against
//    0.56 at 208 columns, 0.41 against 0.47 at 112).
//  * two blocks per wavefront (at most 5 column blocks): one launch with the
//    workgroup size of sk1_waves.
void sk1_plan(int64_t n, int NB, bool bf, int num_cu, int* nw1, int64_t* rows1, int* nw2) {
  const int rb = sk1_row_blocks(NB);
  *rows1 = n;
  *nw1 = *nw2 = sk1_waves(n, NB, bf, num_cu);
  if (rb != 1) return;
  const int lo = sk1_min_waves(NB, bf);
  if (bf) {
    *nw1 = *nw2 = std::max(lo, 7);
    return;
  }
  const int full = sk1_max_waves(NB) == 16 ? 16 : 12;   // four (three) per SIMD
  const int64_t nblk = (n + 15) / 16;
  const int64_t per_round = (int64_t)full * num_cu;
  const int64_t k_full = nblk / per_round;
  if (k_full == 0) return;
  const int64_t rem = nblk - k_full * per_round;
  *nw1 = full;
  *nw2 = full;
  if (rem == 0) return;
  *rows1 = k_full * per_round * 16;
  *nw2 = (int)std::max<int64_t>(lo, (rem + num_cu - 1) / num_cu);
}
Sk32Shape sk32_shape(int64_t n, int64_t d, int m, int num_cu, bool bf) {
  Sk32Shape s;
  s.ldo = (int)((d + 31) / 32 * 32);
  s.NB = std::min(16, (m + 15) / 16);
  s.NP = 16 * s.NB;
  s.npass = (m + s.NP - 1) / s.NP;
  s.nrows_pad = s.npass * s.NP;
  s.ldt = (n + 7) / 8 * 8;
  s.ldy = (int)((d + 3) / 4 * 4);
  sk1_plan(n, s.NB, bf, num_cu, &s.NW, &s.rows1, &s.NW2);
  // split-K over rows of A for the second pass: one resident workgroup per CU
  // (the accumulators of 32 columns x 16 NB per wavefront), S slices so that
  // the j tiles x slices fill the device once
  const int jcols = 16 * kSk2W * sk2_col_blocks(s.NB);
  const int jt = (int)((d + jcols - 1) / jcols);
  s.S = std::max(1, std::min<int>((int)((n + 255) / 256), num_cu / jt));
  s.slice = (n + s.S - 1) / s.S;
  s.slice = (s.slice + kBK - 1) / kBK * kBK;
  s.S = (int)((n + s.slice - 1) / s.slice);
  s.olp_b = align_up((size_t)s.nrows_pad * s.ldo * (bf ? 2 : 4));
  s.yp_b = align_up(sizeof(float) * (size_t)s.S * m * s.ldy);
  return s;
}

// Sketch one block of m new columns into F (columns r_old .. r_old+m-1).
nys_status sketch_block(nys_ctx ctx, const nys_dense& A, const double* D, double c,
                        const double* omega, int m, nys_factor F) {
  hipStream_t st = ctx->stream;
  const int64_t n = A.n, d = A.d;
  const int r0 = F->r, r1 = F->r + m;
  // capacity
  if (r1 > F->cap) {
    const int cap = std::min<int64_t>(std::max(r1, 2 * F->cap), d - 1);
    NYS_TRY(grow(F->Omega, sizeof(double) * d * r0, sizeof(double) * d * cap, st));
    NYS_TRY(grow(F->Y, sizeof(double) * d * r0, sizeof(double) * d * cap, st));
    if (F->prec != NYS_F64 && !F->sparse) {
      const int64_t ldt = (n + 7) / 8 * 8;
      NYS_TRY(grow(F->T, sizeof(float) * ldt * r0, sizeof(float) * ldt * cap, st));
      // Mbase is cap x cap, row-major with ld = cap: re-pitch on growth
      nys::DevBuf nb;
      NYS_TRY(nb.reserve(sizeof(double) * (size_t)cap * cap));
      if (r0 > 0)
        NYS_TRY_HIP(hipMemcpy2DAsync(nb.ptr, sizeof(double) * cap, F->Mbase.ptr,
                                     sizeof(double) * F->cap, sizeof(double) * r0, r0,
                                     hipMemcpyDeviceToDevice, st));
      F->Mbase.release();
      F->Mbase = nb;
    }
    F->cap = cap;
  }
  double* Om = F->Omega.as<double>() + d * r0;
  NYS_TRY_HIP(hipMemcpyAsync(Om, omega, sizeof(double) * d * m, hipMemcpyDeviceToDevice, st));
  CoreWs w;
  NYS_TRY(core_workspace(ctx, d, std::max(r1, m), &w));
  NYS_TRY(orthonormalize(ctx, Om, d, m, w));
  double* Y = F->Y.as<double>();
  const bool a32 = (A.dtype == NYS_F32);
  if (const nys_sparse_s* SP = as_sparse(A)) {
    // sparse A: Y = A^T (D (A Omega)) + c Omega by two sparse-times-dense passes
    NYS_TRY(ctx->gemm_ws.reserve(sizeof(double) * (size_t)(n + 2 * d) * m + 256));
    NYS_TRY(sparse_sketch(SP, D, c, Om, m, Y + d * r0, ctx->gemm_ws.as<double>(), st));
  } else if (F->sym && F->prec == NYS_F64) {
    // explicit symmetric H = A + c I (kernel SVM): Y = A Omega + c Omega, FP64 sums
    NYS_TRY_HIP(hipMemcpyAsync(Y + d * r0, Om, sizeof(double) * d * m, hipMemcpyDeviceToDevice, st));
    NYS_TRY(gemm64(st, (int)n, m, (int)d, A.data, a32, A.ld, 1, Om, false, 1, d, Y + d * r0, 1, d,
                   1.0, c, w.split, w.split_elems));
  } else if (F->sym) {
    // the same in FP32: Omega rounded to FP32 (the rounded values written
    // back, so the core sees the Omega the products used), Y = A Omega by the
    // FP32-MFMA tiles of the first sketch pass, then Y + c Omega in FP64
    const Sk32Shape sh = sk32_shape(n, d, m, ctx->num_cu, false);
    const int ldo = sh.ldo, NB = sh.NB, npass = sh.npass, nrows_pad = sh.nrows_pad;
    const int64_t ldt = sh.ldt;
    NYS_TRY(ctx->gemm_ws.reserve(align_up((size_t)nrows_pad * ldo * 4)));
    void* Olp = ctx->gemm_ws.ptr;
    hipLaunchKernelGGL(k_round_omega<false>, dim3(blocks((int64_t)nrows_pad * ldo)), dim3(256), 0,
                       st, Om, (int)d, m, Olp, ldo, nrows_pad);
    const int vec = (((uintptr_t)A.data % 16) == 0 && (A.ld % 4) == 0) ? 1 : 0;
    float* T = F->T.as<float>();
    NYS_TRY(launch_sk1<false>(NB, sh.NW, sh.rows1, sh.NW2, A, vec, Olp, ldo, T, ldt, r0, m, npass, st));
    hipLaunchKernelGGL(k_sym_y, dim3(blocks((int64_t)m * d)), dim3(256), 0, st, T + ldt * r0, ldt,
                       (int)d, m, Om, c, Y + d * r0);
  } else if (F->prec == NYS_F64) {
    // T = A Omega (n x m, column-major) in FP64 tiles, Y = A^T (D o T) + c Omega
    NYS_TRY(ctx->gemm_ws.reserve(sizeof(double) * n * m + 256));
    double* T = ctx->gemm_ws.as<double>();
    NYS_TRY(gemm64(st, (int)n, m, (int)d, A.data, a32, A.ld, 1, Om, false, 1, d, T, 1, n, 1.0, 0.0,
                   w.split, w.split_elems));
    NYS_TRY_HIP(hipMemcpyAsync(Y + d * r0, Om, sizeof(double) * d * m, hipMemcpyDeviceToDevice, st));
    NYS_TRY(gemm64(st, (int)d, m, (int)n, A.data, a32, 1, A.ld, T, false, 1, n, Y + d * r0, 1, d,
                   1.0, c, w.split, w.split_elems, D));
  } else {
    if (!a32) return NYS_ERR_INVALID;
    const bool bf = (F->prec == NYS_BF16);
    const Sk32Shape sh = sk32_shape(n, d, m, ctx->num_cu, bf);
    const int ldo = sh.ldo, NB = sh.NB, NP = sh.NP, npass = sh.npass, nrows_pad = sh.nrows_pad;
    const int64_t ldt = sh.ldt;
    const int ldy = sh.ldy, S = sh.S;
    const int64_t slice = sh.slice;
    const size_t olp_b = sh.olp_b;
    NYS_TRY(ctx->gemm_ws.reserve(sh.olp_b + sh.yp_b));
    void* Olp = ctx->gemm_ws.ptr;
    float* Yp = reinterpret_cast<float*>(static_cast<char*>(ctx->gemm_ws.ptr) + olp_b);
    if (bf)
      hipLaunchKernelGGL(k_round_omega<true>, dim3(blocks((int64_t)nrows_pad * ldo)), dim3(256), 0,
                         st, Om, (int)d, m, Olp, ldo, nrows_pad);
    else
      hipLaunchKernelGGL(k_round_omega<false>, dim3(blocks((int64_t)nrows_pad * ldo)), dim3(256),
                         0, st, Om, (int)d, m, Olp, ldo, nrows_pad);
    const int vec = (((uintptr_t)A.data % 16) == 0 && (A.ld % 4) == 0) ? 1 : 0;
    float* T = F->T.as<float>();
    if (bf)
      NYS_TRY(launch_sk1<true>(NB, sh.NW, sh.rows1, sh.NW2, A, vec, Olp, ldo, T, ldt, r0, m, npass, st));
    else
      NYS_TRY(launch_sk1<false>(NB, sh.NW, sh.rows1, sh.NW2, A, vec, Olp, ldo, T, ldt, r0, m, npass, st));
    for (int p = 0; p < npass; ++p) {
      const int cols = std::min(NP, m - p * NP);
      if (bf)
        NYS_TRY(launch_sk2<true>(NB, A, D, T, ldt, r0 + p * NP, cols, slice, S, Yp, ldy, st));
      else
        NYS_TRY(launch_sk2<false>(NB, A, D, T, ldt, r0 + p * NP, cols, slice, S, Yp, ldy, st));
      hipLaunchKernelGGL(k_sk2_reduce, dim3(blocks((int64_t)cols * d)), dim3(256), 0, st, Yp, S,
                         cols, ldy, (int)d, F->Omega.as<double>(), c, Y, r0 + p * NP);
    }
    // new columns of the core matrix: Mbase[:, r0:r1] = T^T D T[:, r0:r1] + c Omega^T Omega_new
    double* Mb = F->Mbase.as<double>();
    const int ldm = F->cap;
    const GramTShape gs = gram_t_shape(n, r1, r0, m, ctx->num_cu);
    if (gs.wp_b > 0) {
      // the partials reuse the temporaries after the Y reduction (stream order)
      NYS_TRY(ctx->gemm_ws.reserve(std::max(sh.olp_b + sh.yp_b, gs.wp_b)));
      double* Wp = ctx->gemm_ws.as<double>();
      const int sym = (r0 == 0 && m == r1) ? 1 : 0;
      hipLaunchKernelGGL(k_gram_t, dim3(gs.G), dim3(64 * kGtW), 0, st, T, ldt, n, D, r1, r0, m,
                         sym, gs.slice, Wp);
      hipLaunchKernelGGL(k_gram_t_reduce, dim3(blocks((int64_t)r1 * m)), dim3(256), 0, st, Wp,
                         gs.G, r1, r0, m, sym, Mb, ldm);
    } else {
      NYS_TRY(gemm64(st, r1, m, (int)n, T, true, ldt, 1, T + ldt * r0, true, 1, ldt, Mb + r0, ldm,
                     1, 1.0, 0.0, w.split, w.split_elems, D));
    }
    if (c != 0.0)
      NYS_TRY(gemm64(st, r1, m, (int)d, F->Omega.ptr, false, d, 1, Om, false, 1, d, Mb + r0, ldm,
                     1, c, 1.0, w.split, w.split_elems));
    hipLaunchKernelGGL(k_mirror_cols, dim3(blocks((int64_t)r1 * m)), dim3(256), 0, st, Mb, ldm, r0,
                       r1);
  }
  NYS_TRY_HIP(hipGetLastError());
  F->r = r1;
  return NYS_OK;
}

}  // namespace

// Mbase with ld = cap is repacked to ld = r for the core.
nys_status sketch_and_core(nys_ctx ctx, const nys_dense& A, const double* D, double c,
                           const double* omega, int m, nys_factor F, double test_mu = -1.0,
                           int* above = nullptr) {
  NYS_TRY(sketch_block(ctx, A, D, c, omega, m, F));
  if (F->prec != NYS_F64 && !F->sym && !F->sparse && F->cap != F->r) {
    // compact Mbase (cap pitch) into core order (r pitch) in gemm_ws
    nys::DevBuf& Mb = F->Mbase;
    nys::DevBuf tmp;
    NYS_TRY(tmp.reserve(sizeof(double) * (size_t)F->r * F->r));
    NYS_TRY_HIP(hipMemcpy2DAsync(tmp.ptr, sizeof(double) * F->r, Mb.ptr, sizeof(double) * F->cap,
                                 sizeof(double) * F->r, F->r, hipMemcpyDeviceToDevice, ctx->stream));
    nys::DevBuf saved = Mb;
    Mb = tmp;
    nys_status s = nys_core(ctx, F, test_mu, above);
    Mb.release();
    Mb = saved;
    return s;
  }
  return nys_core(ctx, F, test_mu, above);
}

// One round of the sketch: extend *F by m columns and rebuild its core.
nys_status sketch_round(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                        const double* omega, int r, nys_dtype prec, nys_factor* F,
                        double test_mu, int* above, bool sym = false,
                        const double* basis_hint = nullptr) {
  if (ctx == nullptr || F == nullptr || omega == nullptr) return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(A));
  if (!(c >= 0.0) || r < 1) return NYS_ERR_INVALID;
  if (prec != NYS_F64 && prec != NYS_F32 && prec != NYS_BF16) return NYS_ERR_INVALID;
  // FP32 / BF16 products need FP32 A; a CSR A takes NYS_F32 to mean FP64
  // products with an FP32 copy of U for the preconditioner
  const bool csr = (A->dtype == NYS_CSR);
  if (prec != NYS_F64 && A->dtype != NYS_F32 && !(csr && prec == NYS_F32))
    return NYS_ERR_INVALID;
  if (A->d > (int64_t)1 << 30 || A->n > ((int64_t)1 << 31) - 1) return NYS_ERR_INVALID;
  const int r_old = (*F != nullptr) ? (*F)->r : 0;
  if (r_old + r >= A->d || r_old + r > 1024) return NYS_ERR_INVALID;
  if (*F != nullptr &&
      ((*F)->d != A->d || (*F)->prec != prec || (*F)->sym != sym || (*F)->sparse != csr))
    return NYS_ERR_INVALID;
  if (sym && (D != nullptr || A->n != A->d || prec == NYS_BF16 || A->dtype == NYS_CSR))
    return NYS_ERR_INVALID;

  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  nys_factor f = *F;
  bool created = false;
  if (f == nullptr) {
    f = new (std::nothrow) nys_factor_s();
    if (f == nullptr) return NYS_ERR_NOMEM;
    f->d = A->d;
    f->device = ctx->device;
    f->prec = prec;
    f->sym = sym;
    f->sparse = csr;
    f->mantissa_bits = (prec == NYS_F64 || csr) ? 52 : 23;
    created = true;
  }
  f->basis_hint = (basis_hint != nullptr && r_old == 0) ? basis_hint : nullptr;
  nys_status s = sketch_and_core(ctx, *A, D, c, omega, r, f, test_mu, above);
  f->basis_hint = nullptr;
  if (s != NYS_OK) {
    if (created) nys_factor_destroy(f);
    return s;
  }
  *F = f;
  return NYS_OK;
}

// Rebuild of a factor with the previous one's U as the eigensolver's start
// basis (same rank and dimension); otherwise as a fresh nys_sketch.
// Upper bounds of the device bytes a sketch call holds in the context (the
// GEMM temporaries of the largest form and the FP64 core workspace) for
// blocks of at most m columns and a total rank of at most r (*tmp), and of
// the buffers of one factor of rank r (capacity at most min(2 r, d - 1)), the
// transient copies made while its capacity grows included (*factor_out).
void sketch_ws_bytes(const nys_dense& A, int m, int r, int num_cu, size_t* tmp,
                     size_t* factor_out) {
  const int64_t n = A.n, d = A.d;
  size_t g = sizeof(double) * (size_t)n * m + 256;                       // FP64 form
  g = std::max(g, sizeof(double) * (size_t)(n + 2 * d) * m + 256);       // sparse form
  if (A.dtype == NYS_F32) {
    const Sk32Shape s = sk32_shape(n, d, m, num_cu, false);               // FP32 >= BF16
    g = std::max(g, s.olp_b + s.yp_b);
    // T^T D T partials of the largest block: the first (square) block of m
    // columns or an appended block of m columns on a rank of at most r
    g = std::max(g, gram_t_shape(n, m, 0, m, num_cu).wp_b);
    if (r > m) g = std::max(g, gram_t_shape(n, r, r - m, m, num_cu).wp_b);
  }
  const int64_t cap = std::min<int64_t>(2 * (int64_t)r, d - 1);
  const int64_t ldt = (n + 7) / 8 * 8;
  const size_t grown = 2 * sizeof(double) * (size_t)(d * cap) +                   // Omega, Y
                       (A.dtype == NYS_F32 ? sizeof(float) * (size_t)(ldt * cap) +   // T
                                                 sizeof(double) * (size_t)(cap * cap)  // Mbase
                                           : 0);
  const size_t factor = 12 * (size_t)d * r + sizeof(double) * (size_t)r +            // U, U32, lambda
                        sizeof(double) * (size_t)r * r + grown;                       // core copy
  *tmp = g + core_ws_bytes_of(d, r);
  *factor_out = factor + grown;   // + one growth transient
}

nys_status sketch_rebuild(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                          const double* omega, int r, nys_dtype prec, nys_factor prev,
                          nys_factor* F) {
  const bool hint = prev != nullptr && prev->r == r && prev->d == A->d && !prev->sym &&
                    prev->lam_host.size() == (size_t)r;
  return sketch_round(ctx, A, D, c, omega, r, prec, F, -1.0, nullptr, false,
                      hint ? prev->U.as<double>() : nullptr);
}

}  // namespace nys

using namespace nys;

extern "C" {

nys_status nys_sketch(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                      const double* omega, int r, nys_dtype prec, nys_factor* F) {
  if (ctx == nullptr || F == nullptr || omega == nullptr) return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(A));
  if (D != nullptr) {
    // the weights are the Hessian of a convex loss, D >= 0 (Section 2.1)
    NYS_TRY_HIP(hipSetDevice(ctx->device));
    nys::CtxScope ctx_scope(ctx);
    NYS_TRY(check_vector(ctx, D, A->n, 0));
  }
  return sketch_round(ctx, A, D, c, omega, r, prec, F, -1.0, nullptr);
}

nys_status nys_sketch_sym(nys_ctx ctx, const nys_dense* K, double c, const double* omega, int r,
                          nys_dtype prec, nys_factor* F) {
  return sketch_round(ctx, K, nullptr, c, omega, r, prec, F, -1.0, nullptr, true);
}

nys_status nys_sketch_adaptive(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                               const double* omega, int s0, int s_max, double rho, double tol,
                               nys_dtype prec, nys_factor* F) {
  if (ctx == nullptr || F == nullptr || *F != nullptr || omega == nullptr) return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(A));
  if (s0 < 1 || s_max < s0 || s_max >= A->d || s_max > 1024 || !(rho > 0.0) || !(tol >= 1.0))
    return NYS_ERR_INVALID;
  if (D != nullptr) {
    NYS_TRY_HIP(hipSetDevice(ctx->device));
    nys::CtxScope ctx_scope(ctx);
    NYS_TRY(check_vector(ctx, D, A->n, 0));
  }
  // kappa = (lambda_s + rho) / rho <= tol  <=>  lambda_s <= (tol - 1) rho, so a
  // round that does not stop is recognised by the inertia of G - (nu + (tol - 1) rho) I
  // and the eigendecomposition is only computed in the final round.
  int s = 0, m = s0;
  nys_factor f = nullptr;
  for (;;) {
    const bool last = s + m >= s_max;
    int above = 0;
    nys_status st = sketch_round(ctx, A, D, c, omega + (int64_t)s * A->d, m, prec, &f,
                                 last ? -1.0 : (tol - 1.0) * rho, &above);
    if (st != NYS_OK) {
      if (f) nys_factor_destroy(f);
      return st;
    }
    s += m;
    if (!above) break;
    m = std::min(s, s_max - s);
  }
  *F = f;
  return NYS_OK;
}

}  // extern "C"
