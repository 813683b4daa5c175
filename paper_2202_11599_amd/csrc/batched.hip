// Batched NysADMM for many independent lasso problems (a regularisation
// path: one A per instance, its gamma changing between calls).  All
// instances advance in lockstep:
//   * the matvec pair of every instance runs in ONE persistent launch per
//     d-bucket, over a list of (instance, row range) tiles; instances whose
//     PCG has converged skip their tiles;
//   * the d-vector kernels run over (instance, block) item lists;
//   * the iteration index lives on the device (PcgDev::k), so a chunk of PCG
//     iterations is captured once into a hipGraph and replayed until every
//     instance has converged;
//   * the launch shape of each bucket (waves, chunks, rows per group, rows per
//     tile, workgroups per CU) is picked by timing candidates on the batch
//     itself the first time it is seen (autotune, cached in the context).
// Per instance the arithmetic is that of the single-problem path: FP64
// products and sums of the stored A, the same PCG recurrences and tests.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>

#include "gram_device.h"
#include "internal.h"

namespace nys {

struct BInst {
  const void* A;
  int64_t n, ld;
  int d, aligned;
  double rho, rho_eff, gamma, tol_rel, tol_abs;
  const void* U;
  int r, u32, active, max_iter;
  const double* lam;
  double lam_s;
  double *x, *z, *u;                    // caller state
  const double* b;                      // response (A^T b pass)
  double *w, *p, *rhs, *cvec, *wy, *atb;
  double *ypart, *qpart;
  int G, ldy;
  double *wwpart, *rrpart, *pppart, *part;
  int nred, nvec, nbp, pad;
  PcgDev* st;
};

struct BTile {
  int inst, slot;
  int64_t r0, r1;
};

struct BItem {
  int inst, blk;
};

namespace {

using namespace gram;

constexpr int kNS = 8;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// vecsel: 0 -> x (PCG init / true residual), 1 -> p (iteration), 2 -> none (A^T b)
template <typename T, int WAVES, int CPL, int R, bool ALIGNED>
__global__ __launch_bounds__(WAVES * 64, (WAVES >= 4 ? 2 : 1)) void k_bgram(
    const BInst* __restrict__ insts, const BTile* __restrict__ tiles, int ntiles, int mode,
    int vecsel, int skip_done) {
  constexpr int NT = WAVES * 64;
  constexpr int VN = Chunk<T>::N;
  typedef typename Chunk<T>::V V;
  __shared__ double red[2][R][WAVES];
  const int tid = threadIdx.x;
  int buf = 0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BTile tl = tiles[t];
    const BInst& I = insts[tl.inst];
    if (!I.active) continue;
    if (skip_done && I.st->done) continue;
    const T* A = static_cast<const T*>(I.A);
    const int d = I.d;
    const double* p = vecsel == 0 ? I.x : (vecsel == 1 ? I.p : nullptr);
    const double* aux = (mode == kModeTOnly) ? I.b : nullptr;
    double pr[CPL][VN], yr[CPL][VN];
#pragma unroll
    for (int m = 0; m < CPL; ++m) {
      const int c0 = col0<T, CPL, ALIGNED, NT>(tid, m);
#pragma unroll
      for (int v = 0; v < VN; ++v) {
        pr[m][v] = (p != nullptr && c0 + v < d) ? p[c0 + v] : 0.0;
        yr[m][v] = 0.0;
      }
    }
    double q = 0.0;
    const int64_t r1 = tl.r1;
    V a0[R][CPL], a1[R][CPL];
    T e0[R][Extra<T>::N], e1[R][Extra<T>::N];
    double v0[R], v1[R];
    load_group<T, CPL, R, ALIGNED, NT>(a0, e0, v0, A, aux, tl.r0, r1, d, I.ld, tid);
    for (int64_t row = tl.r0; row < r1; row += 2 * R) {
      load_group<T, CPL, R, ALIGNED, NT>(a1, e1, v1, A, aux, row + R, r1, d, I.ld, tid);
      realign_group<T, CPL, R, ALIGNED, NT>(a0, e0, A, row, d, I.ld, tid);
      process_group<T, WAVES, CPL, R>(a0, v0, row, r1, mode, pr, yr, q, aux, nullptr, red, buf,
                                      tid);
      if (row + R >= r1) break;
      load_group<T, CPL, R, ALIGNED, NT>(a0, e0, v0, A, aux, row + 2 * R, r1, d, I.ld, tid);
      realign_group<T, CPL, R, ALIGNED, NT>(a1, e1, A, row + R, d, I.ld, tid);
      process_group<T, WAVES, CPL, R>(a1, v1, row + R, r1, mode, pr, yr, q, aux, nullptr, red,
                                      buf, tid);
    }
    double* yp = I.ypart + (int64_t)tl.slot * I.ldy;
#pragma unroll
    for (int m = 0; m < CPL; ++m) {
      const int c0 = col0<T, CPL, ALIGNED, NT>(tid, m);
#pragma unroll
      for (int v = 0; v < VN; ++v)
        if (c0 + v < d) yp[c0 + v] = yr[m][v];
    }
    if (tid == 0) I.qpart[tl.slot] = q;
  }
}

__device__ double bsum1024(const double* __restrict__ a, int n, double* sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double s = 0.0;
  for (int i = tid; i < n; i += 1024) s += a[i];
  s = wave_sum(s);
  __syncthreads();
  if (lane == 0) sh[wv] = s;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < 16; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// op 0 iterate, 1 init (w = rhs - H x), 2 true residual, 3 plain (-> atb),
// 4 init from the carried residual w (no partials: only the norms of w and rhs)
__global__ __launch_bounds__(1024) void k_breduce(const BInst* __restrict__ insts,
                                                  const BItem* __restrict__ items, int op) {
  const BItem it = items[blockIdx.x];
  const BInst& I = insts[it.inst];
  if (!I.active) return;
  if (op == 0 && I.st->done) return;
  constexpr int S = 16;
  __shared__ double part[S][64];
  __shared__ double sh[16];
  const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
  const int64_t j = (int64_t)it.blk * 64 + lane;
  const int d = I.d;
  double acc = 0.0;
  if (j < d && op != 4)
    for (int g = grp; g < I.G; g += S) acc += I.ypart[(int64_t)g * I.ldy + j];
  part[grp][lane] = acc;
  double alpha = 0.0;
  const int k = I.st->k;
  if (op == 0) {
    const double q = bsum1024(I.qpart, I.G, sh);
    const double pp = bsum1024(I.pppart, I.nvec, sh);
    const double pv = q + I.rho_eff * pp;
    if (!(pv > 0.0)) {
      if (it.blk == 0 && tid == 0) {
        I.st->flags |= (pv != pv) ? kFlagNonfinite : kFlagBreakdown;
        I.st->iters = k;
        I.st->done = 1;
      }
      return;
    }
    alpha = I.wy[k & (kWyRing - 1)] / pv;
  }
  __syncthreads();
  if (grp != 0) return;
  double ww = 0.0, rr = 0.0;
  if (j < d && op == 4) {
    const double wj = I.w[j], r = I.rhs[j];
    ww = wj * wj;
    rr = r * r;
  } else if (j < d) {
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) sum += part[i][lane];
    if (op == 3) {
      I.atb[j] = sum;
      return;
    }
    const double* pv_src = (op == 0) ? I.p : I.x;
    const double pj = pv_src[j];
    const double v = sum + I.rho_eff * pj;
    if (op == 0) {
      I.x[j] += alpha * pj;
      const double wj = I.w[j] - alpha * v;
      I.w[j] = wj;
      ww = wj * wj;
    } else {
      const double r = I.rhs[j];
      const double wj = r - v;
      I.w[j] = wj;
      ww = wj * wj;
      rr = r * r;
    }
  }
  if (op == 3) return;
  ww = wave_sum(ww);
  rr = wave_sum(rr);
  if (lane == 0) {
    I.wwpart[it.blk] = ww;
    if (op != 0) I.rrpart[it.blk] = rr;
  }
}

__device__ double bsum256(const double* __restrict__ a, int n, double* sh4) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += a[i];
  s = wave_sum(s);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = s;
  __syncthreads();
  const double r = ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
  __syncthreads();
  return r;
}

// mode 0: iteration test + dots, 1: init test + dots, 3: true residual norm
template <typename UT>
__device__ void bdot_body(const BInst& I, int blk, int mode) {
  __shared__ double sh4[4];
  const int tid = threadIdx.x;
  if (mode == 0 || mode == 1) {
    if (I.st->done) return;
    const double ww = bsum256(I.wwpart, I.nred, sh4);
    double thr2;
    bool zero_rhs = false;
    if (mode == 1) {
      const double rr = bsum256(I.rrpart, I.nred, sh4);
      thr2 = fmax(I.tol_abs * I.tol_abs, I.tol_rel * I.tol_rel * rr);
      zero_rhs = (rr == 0.0);
      if (blk == 0 && tid == 0) {
        I.st->rr = rr;
        I.st->thr2 = thr2;
      }
    } else {
      thr2 = I.st->thr2;
    }
    const bool bad = !(ww == ww) || (ww > 1.7e308);
    if (blk == 0 && tid == 0) I.st->ww = ww;
    if (zero_rhs || bad || ww <= thr2) {
      if (blk == 0 && tid == 0) {
        if (bad) I.st->flags |= kFlagNonfinite;
        if (zero_rhs) I.st->flags |= kFlagZeroRhs;
        I.st->iters = (mode == 1) ? 0 : I.st->k + 1;
        I.st->done = 1;
      }
      return;
    }
  } else {
    const double ww = bsum256(I.wwpart, I.nred, sh4);
    if (blk == 0 && tid == 0) I.st->true_rr = ww;
    return;
  }
  const int lane = tid & 63;
  const int col = blk * 4 + (tid >> 6);
  if (col >= I.r) return;
  const UT* u = static_cast<const UT*>(I.U) + (int64_t)col * I.d;
  double acc = 0.0;
  for (int64_t j = lane; j < I.d; j += 64) acc = fma((double)u[j], I.w[j], acc);
  acc = wave_sum(acc);
  if (lane == 0) I.cvec[col] = acc;
}

__global__ __launch_bounds__(256) void k_bdot(const BInst* __restrict__ insts,
                                              const BItem* __restrict__ items, int mode) {
  const BItem it = items[blockIdx.x];
  const BInst& I = insts[it.inst];
  if (!I.active) return;
  if (I.u32)
    bdot_body<float>(I, it.blk, mode);
  else
    bdot_body<double>(I, it.blk, mode);
}

// mode 0: p = y + beta p, wy[k+1]; mode 1: p = y, wy[0]
template <typename UT>
__device__ void bupdate_body(const BInst& I, int blk, int mode) {
  __shared__ double g[1024];
  __shared__ double sh4[4];
  const int tid = threadIdx.x;
  const int r = I.r;
  double sc = 0.0;
  for (int i = tid; i < r; i += 256) {
    const double s = (I.lam_s + I.rho) / (I.lam[i] + I.rho) - 1.0;
    const double ci = I.cvec[i];
    g[i] = s * ci;
    sc += s * ci * ci;
  }
  const double ww = bsum256(I.wwpart, I.nred, sh4);
  sc = wave_sum(sc);
  if ((tid & 63) == 0) sh4[tid >> 6] = sc;
  __syncthreads();
  const double wy_new = ww + (((sh4[0] + sh4[1]) + sh4[2]) + sh4[3]);
  const int k = I.st->k;
  const int64_t j = (int64_t)blk * 256 + tid;
  double pj = 0.0;
  if (j < I.d) {
    double y = I.w[j];
    const UT* u = static_cast<const UT*>(I.U) + j;
    for (int i = 0; i < r; ++i) y = fma((double)u[(int64_t)i * I.d], g[i], y);
    pj = (mode == 0) ? y + (wy_new / I.wy[k & (kWyRing - 1)]) * I.p[j] : y;
    I.p[j] = pj;
  }
  double pp = wave_sum(pj * pj);
  __syncthreads();
  if ((tid & 63) == 0) sh4[tid >> 6] = pp;
  __syncthreads();
  if (tid == 0) {
    I.pppart[blk] = ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
    if (blk == 0) I.wy[mode == 1 ? 0 : (k + 1) & (kWyRing - 1)] = wy_new;
  }
}

__global__ __launch_bounds__(256) void k_bupdate(const BInst* __restrict__ insts,
                                                 const BItem* __restrict__ items, int mode) {
  const BItem it = items[blockIdx.x];
  const BInst& I = insts[it.inst];
  if (!I.active || I.st->done) return;
  if (I.u32)
    bupdate_body<float>(I, it.blk, mode);
  else
    bupdate_body<double>(I, it.blk, mode);
}

// End of a PCG iteration: advance k of every running instance, stop those at
// max_iter, count the ones still running.
__global__ __launch_bounds__(256) void k_btick(const BInst* __restrict__ insts, int count,
                                               int* __restrict__ running) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < count; q += 256) {
    const BInst& I = insts[q];
    if (!I.active || I.st->done) continue;
    const int k = I.st->k + 1;
    I.st->k = k;
    if (k >= I.max_iter) {
      I.st->iters = k;
      I.st->done = 1;
    } else {
      atomicAdd(&cnt, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *running = cnt;
}

// Reset the PCG state of every instance (done, k, flags) without a memset,
// so the sequence can live in a captured graph.
__global__ void k_breset(const BInst* __restrict__ insts, int count) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= count) return;
  PcgDev* s = insts[q].st;
  s->done = insts[q].active ? 0 : 1;
  s->iters = 0;
  s->flags = 0;
  s->k = 0;
  s->thr2 = s->ww = s->rr = 0.0;
  s->true_rr = -1.0;
}

// rhs = rho (z - u) + A^T b for active instances; carry: the PCG residual
// w = rhs - H_rho x of the last solve follows the change of rhs (x unchanged)
__global__ __launch_bounds__(256) void k_brhs(const BInst* __restrict__ insts,
                                              const BItem* __restrict__ items, int carry) {
  const BItem it = items[blockIdx.x];
  const BInst& I = insts[it.inst];
  if (!I.active) return;
  const int64_t j = (int64_t)it.blk * 256 + threadIdx.x;
  if (j < I.d) {
    const double rn = I.rho * (I.z[j] - I.u[j]) + I.atb[j];
    if (carry) I.w[j] += rn - I.rhs[j];
    I.rhs[j] = rn;
  }
}

// z = S_{gamma/rho}(x + u), u += x - z, with the kNS residual partials per block
__global__ __launch_bounds__(256) void k_bprox(const BInst* __restrict__ insts,
                                               const BItem* __restrict__ items) {
  const BItem it = items[blockIdx.x];
  const BInst& I = insts[it.inst];
  if (!I.active) return;
  const int64_t j = (int64_t)it.blk * 256 + threadIdx.x;
  double v[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (j < I.d) {
    const double kappa = I.gamma / I.rho;
    const double xj = I.x[j], zo = I.z[j], uj = I.u[j];
    const double a = xj + uj;
    const double zn = copysign(fmax(fabs(a) - kappa, 0.0), a);
    const double un = uj + xj - zn;
    I.z[j] = zn;
    I.u[j] = un;
    v[0] = (xj - zn) * (xj - zn);
    v[1] = (zo - zn) * (zo - zn);
    v[2] = xj * xj;
    v[3] = zn * zn;
    v[4] = un * un;
    v[5] = fabs(zn);
    v[6] = fabs(zo);
    v[7] = fabs(zn - zo);
  }
  __shared__ double sh[kNS][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < kNS; ++s) {
    const double r = s < 6 ? wave_sum(v[s]) : wave_max(v[s]);
    if (lane == 0) sh[s][wv] = r;
  }
  __syncthreads();
  if (threadIdx.x < kNS) {
    const int s = threadIdx.x;
    const double r = s < 6 ? ((sh[s][0] + sh[s][1]) + sh[s][2]) + sh[s][3]
                           : fmax(fmax(sh[s][0], sh[s][1]), fmax(sh[s][2], sh[s][3]));
    I.part[(int64_t)s * I.nbp + it.blk] = r;
  }
}

// per-instance scalars out[q*kNS + s] from the prox partials
__global__ __launch_bounds__(256) void k_bscalars(const BInst* __restrict__ insts, int count,
                                                  double* __restrict__ out) {
  const int q = blockIdx.x;
  const BInst& I = insts[q];
  __shared__ double sh[4];
  for (int s = 0; s < kNS; ++s) {
    const bool mx = (s == 6 || s == 7);
    double acc = 0.0;
    if (I.active)
      for (int i = threadIdx.x; i < I.nbp; i += 256) {
        const double v = I.part[(int64_t)s * I.nbp + i];
        acc = mx ? fmax(acc, v) : acc + v;
      }
    acc = mx ? wave_max(acc) : wave_sum(acc);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
      out[(int64_t)q * kNS + s] = mx ? fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]))
                                     : ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ host side

struct Bucket {
  int f64 = 0, waves = 4, cpl = 2, rows = 4, aligned = 1;
  int per_cu = 2;
  int64_t tile_rows = 256;
  std::vector<int> insts;
  BTile* tiles = nullptr;   // device (inside the batch buffer)
  int ntiles = 0;
  int grid = 0;
};

struct Batch {
  int count = 0;
  std::vector<BInst> h;
  DevBuf dev;             // BInst array, tiles, items, per-instance storage
  BInst* insts = nullptr;
  BItem *it64 = nullptr, *itdot = nullptr, *it256 = nullptr;
  int n64 = 0, ndot = 0, n256 = 0;
  std::vector<Bucket> buckets;
  int* running = nullptr;
  double* scal = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  std::string key;
};

template <typename T, int W, int C, int RR>
nys_status launch_bg(const Bucket& b, const BInst* insts, int mode, int vecsel, int skip,
                     hipStream_t st) {
  if (b.aligned) {
    hipLaunchKernelGGL((k_bgram<T, W, C, RR, true>), dim3(b.grid), dim3(W * 64), 0, st, insts,
                       b.tiles, b.ntiles, mode, vecsel, skip);
  } else {
    // unaligned rows with 8-row groups would spill (never a candidate)
    if constexpr (RR == 8) return NYS_ERR_INVALID;
    else
      hipLaunchKernelGGL((k_bgram<T, W, C, RR, false>), dim3(b.grid), dim3(W * 64), 0, st,
                         insts, b.tiles, b.ntiles, mode, vecsel, skip);
  }
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

template <typename T>
nys_status launch_bg_t(const Bucket& b, const BInst* insts, int mode, int vecsel, int skip,
                       hipStream_t st) {
#define NYS_BC(W, C, RR) \
  if (b.waves == W && b.cpl == C && b.rows == RR) return launch_bg<T, W, C, RR>(b, insts, mode, vecsel, skip, st);
  NYS_BC(1, 2, 4) NYS_BC(2, 2, 4) NYS_BC(4, 2, 4) NYS_BC(8, 2, 4)
  NYS_BC(1, 2, 8) NYS_BC(2, 2, 8) NYS_BC(4, 2, 8) NYS_BC(8, 2, 8)
  NYS_BC(1, 3, 2) NYS_BC(2, 3, 2) NYS_BC(4, 3, 2) NYS_BC(8, 3, 2)
  NYS_BC(1, 4, 2) NYS_BC(2, 4, 2) NYS_BC(4, 4, 2) NYS_BC(8, 4, 2)
#undef NYS_BC
  return NYS_ERR_INVALID;
}

// Side streams and events of the context (created on first use, default
// priority, non-blocking)
nys_status side_init(nys_ctx ctx) {
  for (int k = 0; k < nys_ctx_s::kSideStreams; ++k) {
    if (ctx->side_stream[k] == nullptr)
      NYS_TRY_HIP(hipStreamCreateWithFlags(&ctx->side_stream[k], hipStreamNonBlocking));
    if (ctx->side_join[k] == nullptr)
      NYS_TRY_HIP(hipEventCreateWithFlags(&ctx->side_join[k], hipEventDisableTiming));
  }
  if (ctx->side_fork == nullptr)
    NYS_TRY_HIP(hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming));
  return NYS_OK;
}

// The matvec pair of every bucket with tiles.  With side (the context, its
// side streams initialised) the buckets are dealt round-robin over st and the
// side streams, forked from st and joined back to it with events: their
// kernels touch disjoint instances, so one bucket's tail overlaps the next
// bucket's work, and everything after the call stays ordered on st (also
// under graph capture, where the events become graph edges).
nys_status bgram(const Batch& B, int mode, int vecsel, int skip, hipStream_t st,
                 nys_ctx side = nullptr) {
  std::vector<const Bucket*> bs;
  for (const Bucket& b : B.buckets)
    if (b.ntiles > 0) bs.push_back(&b);
  auto launch = [&](const Bucket& b, hipStream_t s) {
    return b.f64 ? launch_bg_t<double>(b, B.insts, mode, vecsel, skip, s)
                 : launch_bg_t<float>(b, B.insts, mode, vecsel, skip, s);
  };
  if (side == nullptr || bs.size() <= 1) {
    for (const Bucket* b : bs) NYS_TRY(launch(*b, st));
    return NYS_OK;
  }
  const int ns = (int)std::min<size_t>(bs.size(), 1 + nys_ctx_s::kSideStreams);
  NYS_TRY_HIP(hipEventRecord(side->side_fork, st));
  for (int k = 1; k < ns; ++k)
    NYS_TRY_HIP(hipStreamWaitEvent(side->side_stream[k - 1], side->side_fork, 0));
  for (size_t i = 0; i < bs.size(); ++i) {
    const int k = (int)(i % ns);
    NYS_TRY(launch(*bs[i], k == 0 ? st : side->side_stream[k - 1]));
  }
  for (int k = 1; k < ns; ++k) {
    NYS_TRY_HIP(hipEventRecord(side->side_join[k - 1], side->side_stream[k - 1]));
    NYS_TRY_HIP(hipStreamWaitEvent(st, side->side_join[k - 1], 0));
  }
  return NYS_OK;
}

nys_status pcg_iteration(nys_ctx ctx, const Batch& B, hipStream_t st) {
  NYS_TRY(bgram(B, kModeHess, 1, 1, st, ctx));
  hipLaunchKernelGGL(k_breduce, dim3(B.n64), dim3(1024), 0, st, B.insts, B.it64, 0);
  hipLaunchKernelGGL(k_bdot, dim3(B.ndot), dim3(256), 0, st, B.insts, B.itdot, 0);
  hipLaunchKernelGGL(k_bupdate, dim3(B.n256), dim3(256), 0, st, B.insts, B.it256, 0);
  hipLaunchKernelGGL(k_btick, dim3(1), dim3(256), 0, st, B.insts, B.count, B.running);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status bpcg_init(nys_ctx ctx, const Batch& B, hipStream_t st, bool carry) {
  hipLaunchKernelGGL(k_breset, dim3((B.count + 255) / 256), dim3(256), 0, st, B.insts, B.count);
  if (carry) {
    hipLaunchKernelGGL(k_breduce, dim3(B.n64), dim3(1024), 0, st, B.insts, B.it64, 4);
  } else {
    NYS_TRY(bgram(B, kModeHess, 0, 0, st, ctx));
    hipLaunchKernelGGL(k_breduce, dim3(B.n64), dim3(1024), 0, st, B.insts, B.it64, 1);
  }
  hipLaunchKernelGGL(k_bdot, dim3(B.ndot), dim3(256), 0, st, B.insts, B.itdot, 1);
  hipLaunchKernelGGL(k_bupdate, dim3(B.n256), dim3(256), 0, st, B.insts, B.it256, 1);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

inline size_t au(size_t x) { return (x + 255) / 256 * 256; }

int cover_of(int waves, int cpl, int vn) { return waves * 64 * cpl * vn; }

// candidate launch shapes for a bucket whose widest instance has d_max columns
std::vector<Bucket> bucket_candidates(const Bucket& base, int d_max, int num_cu) {
  static const int shapes[][3] = {{1, 2, 4}, {1, 2, 8}, {2, 2, 4}, {2, 2, 8}, {4, 2, 4},
                                  {4, 2, 8}, {8, 2, 4}, {8, 2, 8}, {1, 3, 2}, {2, 3, 2},
                                  {4, 3, 2}, {8, 3, 2}, {1, 4, 2}, {2, 4, 2}, {4, 4, 2},
                                  {8, 4, 2}};
  const int vn = base.f64 ? 2 : 4;
  int best = -1;
  for (auto& sh : shapes) {
    const int c = cover_of(sh[0], sh[1], vn);
    if (c >= d_max && (best < 0 || c < best)) best = c;
  }
  std::vector<Bucket> out;
  for (auto& sh : shapes) {
    const int c = cover_of(sh[0], sh[1], vn);
    if (c < d_max || c > 2 * best) continue;
    if (!base.aligned && sh[2] == 8) continue;   // realignment state would spill
    for (int64_t tr : {128, 256, 1024}) {
      Bucket b = base;
      b.waves = sh[0];
      b.cpl = sh[1];
      b.rows = sh[2];
      b.per_cu = std::max(1, 8 / sh[0]);
      b.tile_rows = tr;
      out.push_back(b);
    }
  }
  return out;
}

void make_tiles(const Bucket& b, const std::vector<BInst>& h, std::vector<BTile>* tiles) {
  tiles->clear();
  // round-robin over instances so that consecutive tiles (and so concurrently
  // running workgroups) spread over different matrices
  std::vector<int64_t> next(b.insts.size(), 0);
  bool any = true;
  while (any) {
    any = false;
    for (size_t k = 0; k < b.insts.size(); ++k) {
      const int q = b.insts[k];
      if (next[k] >= h[q].n) continue;
      any = true;
      BTile t;
      t.inst = q;
      t.slot = (int)(next[k] / b.tile_rows);
      t.r0 = next[k];
      t.r1 = std::min<int64_t>(h[q].n, next[k] + b.tile_rows);
      next[k] = t.r1;
      tiles->push_back(t);
    }
  }
}

// Lay out the batch: per-instance vectors, partial sums sized for the finest
constexpr int64_t kFinest = 128;   // finest tiling the tuner may choose

// device bytes of one instance's vectors and partial sums in the batch buffer
size_t inst_bytes(int64_t n, int64_t d) {
  const int G = (int)((n + kFinest - 1) / kFinest);
  const int ldy = (int)((d + 63) / 64 * 64);
  return 5 * au(sizeof(double) * d) + au(sizeof(double) * 1024) + au(sizeof(double) * kWyRing) +
         au(sizeof(double) * (size_t)G * ldy) + au(sizeof(double) * G) +
         3 * au(sizeof(double) * ((d + 63) / 64)) + au(sizeof(double) * ((d + 255) / 256)) +
         au(sizeof(double) * kNS * ((d + 255) / 256)) + au(sizeof(PcgDev));
}

// tiling, tile and item lists; bucket the instances by row width.
nys_status batch_build(nys_ctx ctx, int count, const nys_problem* P, const nys_admm_opts* O,
                       nys_factor* F, nys_admm_state* S, int max_iter, Batch* B) {
  B->count = count;
  B->h.assign(count, BInst{});
  size_t bytes = au(sizeof(BInst) * count);
  std::vector<size_t> off(count);
  for (int q = 0; q < count; ++q) {
    off[q] = bytes;
    bytes += inst_bytes(P[q].A.n, P[q].A.d);
  }
  // buckets by row width
  std::map<std::pair<int, int>, std::vector<int>> groups;   // (f64|aligned, cover class)
  for (int q = 0; q < count; ++q) {
    const nys_dense& A = P[q].A;
    const int vn = A.dtype == NYS_F64 ? 2 : 4;
    const int esize = vn == 2 ? 8 : 4;
    const int aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
    // classes at the column counts the launch shapes cover exactly (128 vn
    // times 1, 1.5, 2, 3, 4, 6, ...), so that an instance leaves at most a
    // third of a bucket's lanes idle
    int cls = 128 * vn, lo = cls;
    while (cls < A.d) {
      if (cls == lo) {
        cls = lo * 3 / 2;
      } else {
        lo *= 2;
        cls = lo;
      }
    }
    groups[{(A.dtype == NYS_F64 ? 2 : 0) | aligned, cls}].push_back(q);
  }
  size_t tiles_total = 0;
  for (auto& g : groups) {
    for (int q : g.second) tiles_total += (size_t)((P[q].A.n + kFinest - 1) / kFinest);
  }
  const size_t tiles_off = bytes;
  bytes += au(sizeof(BTile) * std::max<size_t>(tiles_total, 1));
  int n64 = 0, ndot = 0, n256 = 0;
  for (int q = 0; q < count; ++q) {
    n64 += (int)((P[q].A.d + 63) / 64);
    ndot += std::max(1, (F[q]->r + 3) / 4);
    n256 += (int)((P[q].A.d + 255) / 256);
  }
  const size_t items_off = bytes;
  bytes += au(sizeof(BItem) * n64) + au(sizeof(BItem) * ndot) + au(sizeof(BItem) * n256);
  const size_t misc_off = bytes;
  bytes += au(sizeof(int)) + au(sizeof(double) * kNS * count);
  NYS_TRY(B->dev.reserve(bytes));
  char* base = static_cast<char*>(B->dev.ptr);
  B->insts = reinterpret_cast<BInst*>(base);
  for (int q = 0; q < count; ++q) {
    const nys_dense& A = P[q].A;
    const int64_t d = A.d, n = A.n;
    const int G = (int)((n + kFinest - 1) / kFinest);
    const int ldy = (int)((d + 63) / 64 * 64);
    char* p = base + off[q];
    auto take = [&](size_t b) { char* r = p; p += b; return reinterpret_cast<double*>(r); };
    BInst& I = B->h[q];
    I.A = A.data;
    I.n = n;
    I.ld = A.ld;
    I.d = (int)d;
    const int esize = A.dtype == NYS_F64 ? 8 : 4;
    I.aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
    I.rho = O[q].rho;
    I.rho_eff = O[q].rho + P[q].c;
    I.gamma = P[q].gamma;
    I.tol_rel = O[q].pcg.tol_abs ? 0.0 : O[q].pcg.tol;
    I.tol_abs = O[q].pcg.tol_abs ? O[q].pcg.tol : 0.0;
    I.U = F[q]->use_u32 ? F[q]->U32.ptr : F[q]->U.ptr;
    I.u32 = F[q]->use_u32 ? 1 : 0;
    I.r = F[q]->r;
    I.lam = F[q]->lam.as<double>();
    I.lam_s = F[q]->lam_host[F[q]->r - 1];
    I.active = 1;
    I.max_iter = max_iter;
    I.x = S[q].x;
    I.z = S[q].z;
    I.u = S[q].u;
    I.b = P[q].b;
    I.w = take(au(sizeof(double) * d));
    I.p = take(au(sizeof(double) * d));
    I.rhs = take(au(sizeof(double) * d));
    I.atb = take(au(sizeof(double) * d));
    (void)take(au(sizeof(double) * d));
    I.cvec = take(au(sizeof(double) * 1024));
    I.wy = take(au(sizeof(double) * kWyRing));
    I.ypart = take(au(sizeof(double) * (size_t)G * ldy));
    I.qpart = take(au(sizeof(double) * G));
    I.G = G;
    I.ldy = ldy;
    I.nred = (int)((d + 63) / 64);
    I.nvec = (int)((d + 255) / 256);
    I.nbp = I.nvec;
    I.wwpart = take(au(sizeof(double) * I.nred));
    I.rrpart = take(au(sizeof(double) * I.nred));
    (void)take(au(sizeof(double) * I.nred));
    I.pppart = take(au(sizeof(double) * I.nvec));
    I.part = take(au(sizeof(double) * kNS * I.nbp));
    I.st = reinterpret_cast<PcgDev*>(take(au(sizeof(PcgDev))));
  }
  // items
  std::vector<BItem> it64, itdot, it256;
  for (int q = 0; q < count; ++q) {
    for (int k = 0; k < B->h[q].nred; ++k) it64.push_back({q, k});
    for (int k = 0; k < std::max(1, (B->h[q].r + 3) / 4); ++k) itdot.push_back({q, k});
    for (int k = 0; k < B->h[q].nvec; ++k) it256.push_back({q, k});
  }
  B->it64 = reinterpret_cast<BItem*>(base + items_off);
  B->itdot = B->it64 + 0;
  B->itdot = reinterpret_cast<BItem*>(base + items_off + au(sizeof(BItem) * n64));
  B->it256 = reinterpret_cast<BItem*>(base + items_off + au(sizeof(BItem) * n64) +
                                      au(sizeof(BItem) * ndot));
  B->n64 = n64;
  B->ndot = ndot;
  B->n256 = n256;
  B->running = reinterpret_cast<int*>(base + misc_off);
  B->scal = reinterpret_cast<double*>(base + misc_off + au(sizeof(int)));
  hipStream_t st = ctx->stream;
  NYS_TRY_HIP(hipMemcpyAsync(B->it64, it64.data(), sizeof(BItem) * n64, hipMemcpyHostToDevice, st));
  NYS_TRY_HIP(hipMemcpyAsync(B->itdot, itdot.data(), sizeof(BItem) * ndot, hipMemcpyHostToDevice, st));
  NYS_TRY_HIP(hipMemcpyAsync(B->it256, it256.data(), sizeof(BItem) * n256, hipMemcpyHostToDevice, st));
  // buckets with the heuristic shape first (tuned below)
  BTile* tiles_dev = reinterpret_cast<BTile*>(base + tiles_off);
  size_t tile_cursor = 0;
  B->buckets.clear();
  for (auto& g : groups) {
    Bucket b;
    b.f64 = (g.first.first & 2) ? 1 : 0;
    b.aligned = g.first.first & 1;
    b.insts = g.second;
    int d_max = 0;
    int64_t finest_tiles = 0;
    for (int q : b.insts) {
      d_max = std::max(d_max, B->h[q].d);
      finest_tiles += (P[q].A.n + kFinest - 1) / kFinest;
    }
    std::vector<Bucket> c = bucket_candidates(b, d_max, ctx->num_cu);
    if (c.empty()) return NYS_ERR_INVALID;
    b = c[0];
    b.tiles = tiles_dev + tile_cursor;
    tile_cursor += (size_t)finest_tiles;
    B->buckets.push_back(b);
  }
  NYS_TRY_HIP(hipMemcpyAsync(B->insts, B->h.data(), sizeof(BInst) * count, hipMemcpyHostToDevice, st));
  return NYS_OK;
}

nys_status upload_tiles(nys_ctx ctx, Bucket* b, const std::vector<BInst>& h, int num_cu) {
  std::vector<BTile> t;
  make_tiles(*b, h, &t);
  b->ntiles = (int)t.size();
  // one workgroup per tile: the dispatcher hands tiles to CUs as they free
  // up, which balances tiles of uneven width and skipped (converged) ones
  b->grid = std::max(1, b->ntiles);
  if (!t.empty())
    NYS_TRY_HIP(hipMemcpyAsync(b->tiles, t.data(), sizeof(BTile) * t.size(), hipMemcpyHostToDevice,
                               ctx->stream));
  return NYS_OK;
}

// Time every candidate shape of every bucket on the batch (matvec pair of all
// its instances, x as input) and keep the fastest; cached per batch signature.
nys_status batch_tune(nys_ctx ctx, Batch* B) {
  hipStream_t st = ctx->stream;
  hipEvent_t e0, e1;
  NYS_TRY_HIP(hipEventCreate(&e0));
  NYS_TRY_HIP(hipEventCreate(&e1));
  for (Bucket& bk : B->buckets) {
    int d_max = 0;
    for (int q : bk.insts) d_max = std::max(d_max, B->h[q].d);
    std::string key = "batch|" + std::to_string(bk.f64) + "|" + std::to_string(bk.aligned);
    for (int q : bk.insts)
      key += "|" + std::to_string(B->h[q].n) + "x" + std::to_string(B->h[q].d);
    auto hit = ctx->bplans.find(key);
    std::vector<Bucket> cands;
    if (hit != ctx->bplans.end()) {
      Bucket b = bk;
      b.waves = hit->second[0];
      b.cpl = hit->second[1];
      b.rows = hit->second[2];
      b.per_cu = hit->second[3];
      b.tile_rows = hit->second[4];
      cands.push_back(b);
    } else {
      cands = bucket_candidates(bk, d_max, ctx->num_cu);
      const char* tune = getenv("NYSADMM_TUNE");
      if (tune != nullptr && tune[0] == '0') cands.resize(1);
    }
    float best = 1e30f;
    Bucket bestb = cands[0];
    for (Bucket c : cands) {
      c.tiles = bk.tiles;
      NYS_TRY(upload_tiles(ctx, &c, B->h, ctx->num_cu));
      if (cands.size() == 1) {
        bestb = c;
        break;
      }
      Batch one;
      one.insts = B->insts;
      one.buckets.push_back(c);
      NYS_TRY(bgram(one, kModeHess, 0, 0, st));
      NYS_TRY_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < 2; ++r) NYS_TRY(bgram(one, kModeHess, 0, 0, st));
      NYS_TRY_HIP(hipEventRecord(e1, st));
      NYS_TRY_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      NYS_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        bestb = c;
      }
    }
    NYS_TRY(upload_tiles(ctx, &bestb, B->h, ctx->num_cu));
    bk = bestb;
    ctx->bplans[key] = {bk.waves, bk.cpl, bk.rows, bk.per_cu, (int)bk.tile_rows};
    if (getenv("NYSADMM_VERBOSE"))
      fprintf(stderr, "nysadmm: batched bucket (%zu instances, d <= %d): waves %d, chunks %d, "
              "rows %d, %d wg/CU, tile %lld rows, %d tiles (%.1f us)\n", bk.insts.size(), d_max,
              bk.waves, bk.cpl, bk.rows, bk.per_cu, (long long)bk.tile_rows, bk.ntiles,
              cands.size() > 1 ? 1e3 * best / 2 : -1.0);
    // the partial-sum count of each instance follows the chosen tiling
    for (int q : bk.insts) B->h[q].G = (int)((B->h[q].n + bk.tile_rows - 1) / bk.tile_rows);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  NYS_TRY_HIP(hipMemcpyAsync(B->insts, B->h.data(), sizeof(BInst) * B->count,
                             hipMemcpyHostToDevice, st));
  return NYS_OK;
}

constexpr int kGraphIters = 4;

nys_status batch_graph(nys_ctx ctx, Batch* B) {
  if (B->graph != nullptr) return NYS_OK;
  if (ctx->cap_stream == nullptr)
    NYS_TRY_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  NYS_TRY_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  nys_status s = NYS_OK;
  for (int i = 0; i < kGraphIters && s == NYS_OK; ++i) s = pcg_iteration(ctx, *B, ctx->cap_stream);
  hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
  if (s != NYS_OK) return s;
  NYS_TRY_HIP(e);
  e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  NYS_TRY_HIP(e);
  B->graph_iters = kGraphIters;
  return NYS_OK;
}

// Batched Algorithm Nystrom PCG: every active instance from its x, replays of
// the captured iteration chunk until all have converged or hit max_iter.
// carry: w already holds rhs - H_rho x (see k_brhs); check: end with the
// FP64 true residual (which also leaves it in w).
nys_status batch_pcg(nys_ctx ctx, Batch* B, int max_iter, std::vector<PcgDev>* states, bool carry,
                     bool check) {
  hipStream_t st = ctx->stream;
  NYS_TRY(side_init(ctx));
  NYS_TRY(bpcg_init(ctx, *B, st, carry));
  NYS_TRY(batch_graph(ctx, B));
  int done_iters = 0;
  for (;;) {
    NYS_TRY_HIP(hipGraphLaunch(B->graph, st));
    done_iters += B->graph_iters;
    NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, B->running, sizeof(int), hipMemcpyDeviceToHost, st));
    NYS_TRY_HIP(hipStreamSynchronize(st));
    const int running = *static_cast<int*>(ctx->host_pinned);
    if (running == 0 || done_iters >= max_iter + B->graph_iters) break;
  }
  if (check) {
    // FP64-accumulated true residual of every active instance: a full pass
    // over each active instance's A, bracketed by timing events while the
    // context's kernel timing is on
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->prof_on) {
      while (ctx->prof_used + 2 > ctx->prof_ev.size()) {
        hipEvent_t e;
        NYS_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        ctx->prof_ev.push_back(e);
      }
      e0 = ctx->prof_ev[ctx->prof_used];
      e1 = ctx->prof_ev[ctx->prof_used + 1];
      NYS_TRY_HIP(hipEventRecord(e0, st));
    }
    NYS_TRY(bgram(*B, kModeHess, 0, 0, st, ctx));
    if (e1 != nullptr) {
      NYS_TRY_HIP(hipEventRecord(e1, st));
      ctx->prof_used += 2;
    }
    hipLaunchKernelGGL(k_breduce, dim3(B->n64), dim3(1024), 0, st, B->insts, B->it64, 2);
    hipLaunchKernelGGL(k_bdot, dim3(B->ndot), dim3(256), 0, st, B->insts, B->itdot, 3);
  }
  NYS_TRY_HIP(hipGetLastError());
  states->resize(B->count);
  for (int q = 0; q < B->count; ++q)
    NYS_TRY_HIP(hipMemcpyAsync(&(*states)[q], B->h[q].st, sizeof(PcgDev), hipMemcpyDeviceToHost, st));
  NYS_TRY_HIP(hipStreamSynchronize(st));
  return NYS_OK;
}

}  // namespace

// Device bytes batch_build takes for `count` instances of shape n x d at rank r
// (the same sums as batch_build).
size_t batch_workspace_bytes(int count, int64_t n, int64_t d, int r) {
  const size_t tiles = (size_t)count * (size_t)((n + kFinest - 1) / kFinest);
  const size_t n64 = (size_t)count * (size_t)((d + 63) / 64);
  const size_t ndot = (size_t)count * (size_t)std::max(1, (r + 3) / 4);
  const size_t n256 = (size_t)count * (size_t)((d + 255) / 256);
  return au(sizeof(BInst) * count) + (size_t)count * inst_bytes(n, d) +
         au(sizeof(BTile) * std::max<size_t>(tiles, 1)) + au(sizeof(BItem) * n64) +
         au(sizeof(BItem) * ndot) + au(sizeof(BItem) * n256) + au(sizeof(int)) +
         au(sizeof(double) * kNS * count);
}

// Lockstep NysADMM over `count` least-squares problems (see batched.hip header).
nys_status admm_solve_batched(nys_ctx ctx, int count, const nys_problem* P,
                              const nys_admm_opts* O, nys_admm_state* S, nys_admm_info* I) {
  hipStream_t st = ctx->stream;
  std::vector<nys_factor> F(count, nullptr);
  std::vector<char> owned(count, 0);
  nys_status s = NYS_OK;
  for (int q = 0; q < count && s == NYS_OK; ++q) {
    if (O[q].factor != nullptr) {
      F[q] = O[q].factor;
      continue;
    }
    owned[q] = 1;
    if (O[q].rank_max > O[q].rank && O[q].ada_tol >= 1.0)
      s = nys_sketch_adaptive(ctx, &P[q].A, nullptr, P[q].c, O[q].omega, O[q].rank, O[q].rank_max,
                              O[q].rho, O[q].ada_tol, O[q].sketch_prec, &F[q]);
    else
      s = nys_sketch(ctx, &P[q].A, nullptr, P[q].c, O[q].omega, O[q].rank, O[q].sketch_prec, &F[q]);
  }
  int max_iter = 0, pcg_max = 0, tr_every = 0;
  bool want_tr = false;
  for (int q = 0; q < count; ++q) {
    max_iter = std::max(max_iter, O[q].max_iter > 0 ? O[q].max_iter : 100);
    pcg_max = std::max(pcg_max, O[q].pcg.max_iter > 0 ? O[q].pcg.max_iter : 1000);
    const int e = O[q].true_res_every > 0 ? O[q].true_res_every : 1;
    tr_every = tr_every == 0 ? e : std::min(tr_every, e);
    want_tr = want_tr || O[q].pcg.true_residual != 0;
  }
  Batch B;
  if (s == NYS_OK) s = batch_build(ctx, count, P, O, F.data(), S, pcg_max, &B);
  if (s == NYS_OK) s = batch_tune(ctx, &B);
  std::vector<nys_admm_info> info(count);
  for (auto& x : info) {
    x = nys_admm_info{};
    x.eta = x.obj = x.true_res_max = -1.0;
  }
  // A^T b of every instance, one batched pass
  if (s == NYS_OK) {
    s = bgram(B, kModeTOnly, 2, 0, st);
    if (s == NYS_OK)
      hipLaunchKernelGGL(k_breduce, dim3(B.n64), dim3(1024), 0, st, B.insts, B.it64, 3);
  }
  std::vector<double> sc((size_t)kNS * count);
  std::vector<PcgDev> pst;
  for (int it = 0; s == NYS_OK && it < max_iter; ++it) {
    // true residual at every tr_every-th step and at each instance's last
    bool check = want_tr && (it + 1) % tr_every == 0;
    for (int q = 0; q < count && want_tr && !check; ++q)
      if (B.h[q].active && info[q].iters + 1 >= (O[q].max_iter > 0 ? O[q].max_iter : 100))
        check = true;
    // from the second step on, the residual of the last solve is carried
    const int carry = it > 0 ? 1 : 0;
    hipLaunchKernelGGL(k_brhs, dim3(B.n256), dim3(256), 0, st, B.insts, B.it256, carry);
    s = batch_pcg(ctx, &B, pcg_max, &pst, carry != 0, check);
    if (s != NYS_OK) break;
    hipLaunchKernelGGL(k_bprox, dim3(B.n256), dim3(256), 0, st, B.insts, B.it256);
    hipLaunchKernelGGL(k_bscalars, dim3(count), dim3(256), 0, st, B.insts, count, B.scal);
    if (hipMemcpyAsync(sc.data(), B.scal, sizeof(double) * kNS * count, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      s = NYS_ERR_HIP;
      break;
    }
    bool changed = false, any_active = false;
    for (int q = 0; q < count; ++q) {
      BInst& h = B.h[q];
      if (!h.active) continue;
      const double* v = &sc[(size_t)q * kNS];
      nys_admm_info& f = info[q];
      const PcgDev& ps = pst[q];
      f.iters += 1;
      f.pcg_iters += ps.iters;
      f.pcg_max = std::max(f.pcg_max, ps.iters);
      f.r_p = std::sqrt(v[0]);
      f.r_d = O[q].rho * std::sqrt(v[1]);
      f.rank = F[q]->r;
      const double res2 = check ? ps.true_rr : ps.ww;
      const nys_status step_status =
          (ps.flags & kFlagNonfinite) ? NYS_ERR_NONFINITE
          : (ps.flags & kFlagBreakdown) ? NYS_ERR_BREAKDOWN
          : (!(res2 <= ps.thr2) && !(ps.flags & kFlagZeroRhs)) ? NYS_ERR_MAXITER
                                                              : NYS_OK;
      if (step_status == NYS_ERR_MAXITER) f.maxiter_solves += 1;
      if (f.status == NYS_OK) f.status = step_status;   // sticky: first non-OK
      if (check && ps.true_rr >= 0.0)
        f.true_res_max = std::max(f.true_res_max,
                                  ps.rr > 0.0 ? std::sqrt(ps.true_rr / ps.rr) : 0.0);
      S[q].k += 1;
      bool stop = (f.iters >= (O[q].max_iter > 0 ? O[q].max_iter : 100));
      if (O[q].eps_rel > 0.0) {
        const double tp = O[q].eps_abs + O[q].eps_rel * std::max(std::sqrt(v[2]), std::sqrt(v[3]));
        const double td = O[q].eps_abs + O[q].eps_rel * O[q].rho * std::sqrt(v[4]);
        if (f.r_p <= tp && f.r_d <= td) {
          stop = true;
          f.converged = 1;
        }
      }
      if (O[q].rel_change_tol > 0.0 && f.iters > 1 && v[6] > 0.0 &&
          v[7] / v[6] < O[q].rel_change_tol) {
        stop = true;
        f.converged = 1;
      }
      if (step_status == NYS_ERR_NONFINITE || step_status == NYS_ERR_BREAKDOWN) stop = true;
      if (stop) {
        h.active = 0;
        changed = true;
      } else {
        any_active = true;
      }
    }
    if (changed)
      if (hipMemcpyAsync(B.insts, B.h.data(), sizeof(BInst) * count, hipMemcpyHostToDevice, st) !=
          hipSuccess)
        s = NYS_ERR_HIP;
    if (!any_active) break;
  }
  if (B.graph != nullptr) (void)hipGraphExecDestroy(B.graph);
  (void)hipStreamSynchronize(st);
  B.dev.release();
  // only the batched passes are timed: the closing per-instance KKT passes
  // would mix single-matrix launches into the batched average
  const bool prof_on = ctx->prof_on;
  ctx->prof_on = false;
  for (int q = 0; q < count; ++q) {
    if (s == NYS_OK) {
      nys_status ks = admm_kkt(ctx, P[q], S[q].z, &info[q].eta, &info[q].obj);
      if (ks != NYS_OK) s = ks;
    }
    if (owned[q] && F[q] != nullptr) nys_factor_destroy(F[q]);
    if (I) I[q] = info[q];
  }
  ctx->prof_on = prof_on;
  return s;
}

}  // namespace nys
