// C ABI: contexts, factors, preconditioner apply and the PCG driver.
// The sketch entry points live in sketch.hip, the ADMM drivers in admm.hip.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

namespace nys {

static thread_local char g_last_err[256] = {0};

void set_last_hip_error(hipError_t e, const char* what, const char* file, int line) {
  snprintf(g_last_err, sizeof(g_last_err), "%s failed (%s) at %s:%d", what,
           hipGetErrorString(e), file, line);
}

// ---- block cache
// Released device blocks are kept (up to kPoolCap bytes per process) with one
// event per live context stream of their device, recorded at release; a block
// is handed out again once all of its events have completed, i.e. once no work
// that was queued when it was released can still touch it.  Library kernels
// run only on context streams, so this is the guarantee hipFree gives, without
// its device-wide synchronisation.  The cache of a device is emptied when its
// last context is destroyed.
namespace {
struct PoolBlock {
  void* ptr;
  size_t bytes;
  int device;
  std::vector<hipEvent_t> evs;
};
struct Pool {
  std::mutex mu;
  std::vector<PoolBlock> blocks;
  std::vector<std::pair<int, hipStream_t>> streams;
  std::vector<std::pair<int, hipEvent_t>> spare_events;
  size_t cached = 0;
};
Pool& pool() {
  static Pool* p = new Pool();   // lives until the process ends
  return *p;
}
constexpr size_t kPoolCap = size_t(4) << 30;

size_t pool_round(size_t want) {
  if (want == 0) want = 256;
  const size_t g = want > (size_t(1) << 20) ? (size_t(2) << 20) : 4096;
  return (want + g - 1) / g * g;
}

bool pool_ready(const PoolBlock& b) {
  for (hipEvent_t e : b.evs) {
    const hipError_t r = hipEventQuery(e);
    if (r != hipSuccess) {
      if (r != hipErrorNotReady) (void)hipGetLastError();
      return false;
    }
  }
  return true;
}

// caller holds the lock; the block's device is current
void pool_recycle_events(Pool& P, PoolBlock& b) {
  for (hipEvent_t e : b.evs) P.spare_events.emplace_back(b.device, e);
  b.evs.clear();
}

// free every cached block of `device` (waits for their events)
void pool_trim_locked(Pool& P, int device) {
  for (size_t i = 0; i < P.blocks.size();) {
    PoolBlock& b = P.blocks[i];
    if (b.device != device) {
      ++i;
      continue;
    }
    for (hipEvent_t e : b.evs) (void)hipEventSynchronize(e);
    pool_recycle_events(P, b);
    (void)hipFree(b.ptr);
    P.cached -= b.bytes;
    P.blocks.erase(P.blocks.begin() + (long)i);
  }
  for (size_t i = 0; i < P.spare_events.size();) {
    if (P.spare_events[i].first == device) {
      (void)hipEventDestroy(P.spare_events[i].second);
      P.spare_events.erase(P.spare_events.begin() + (long)i);
    } else {
      ++i;
    }
  }
}
}  // namespace

void pool_register_stream(int device, hipStream_t st) {
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  P.streams.emplace_back(device, st);
}

void pool_unregister_stream(int device, hipStream_t st) {
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  for (size_t i = 0; i < P.streams.size(); ++i)
    if (P.streams[i].first == device && P.streams[i].second == st) {
      P.streams.erase(P.streams.begin() + (long)i);
      break;
    }
  bool live = false;
  for (auto& s : P.streams) live = live || s.first == device;
  if (!live) pool_trim_locked(P, device);
}

// ---- caller workspaces
namespace {
thread_local std::shared_ptr<Arena> tls_arena;
constexpr size_t kArenaGrain = 256;
}  // namespace

Arena::Arena(void* p, size_t n, int dev) : device(dev) {
  // the usable range starts at the first 256-byte boundary
  const uintptr_t b = reinterpret_cast<uintptr_t>(p);
  const uintptr_t a = (b + kArenaGrain - 1) / kArenaGrain * kArenaGrain;
  const size_t skip = (size_t)(a - b);
  base = reinterpret_cast<char*>(a);
  bytes = n > skip ? (n - skip) / kArenaGrain * kArenaGrain : 0;
  if (bytes > 0) free_blocks[0] = bytes;
}

void* Arena::alloc(size_t want) {
  want = (std::max<size_t>(want, 1) + kArenaGrain - 1) / kArenaGrain * kArenaGrain;
  std::lock_guard<std::mutex> g(mu);
  for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
    if (it->second < want) continue;
    const size_t off = it->first, sz = it->second;
    free_blocks.erase(it);
    if (sz > want) free_blocks[off + want] = sz - want;
    in_use += want;
    peak = std::max(peak, in_use);
    return base + off;
  }
  return nullptr;
}

void Arena::free(void* p, size_t n) {
  if (p == nullptr) return;
  n = (std::max<size_t>(n, 1) + kArenaGrain - 1) / kArenaGrain * kArenaGrain;
  std::lock_guard<std::mutex> g(mu);
  size_t off = (size_t)(static_cast<char*>(p) - base);
  in_use -= std::min(in_use, n);
  auto next = free_blocks.lower_bound(off);
  if (next != free_blocks.end() && off + n == next->first) {
    n += next->second;
    next = free_blocks.erase(next);
  }
  if (next != free_blocks.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      off = prev->first;
      n += prev->second;
      free_blocks.erase(prev);
    }
  }
  free_blocks[off] = n;
}

CtxScope::CtxScope(nys_ctx ctx) : prev_(tls_arena) { tls_arena = ctx ? ctx->arena : nullptr; }
CtxScope::~CtxScope() { tls_arena = prev_; }

nys_status DevBuf::reserve(size_t want) {
  if (want <= bytes && ptr != nullptr) return NYS_OK;
  release();
  if (std::shared_ptr<Arena> ar = tls_arena) {
    // carved from the caller's workspace; never hipMalloc
    want = (std::max<size_t>(want, 1) + kArenaGrain - 1) / kArenaGrain * kArenaGrain;
    void* p = ar->alloc(want);
    if (p == nullptr) return NYS_ERR_NOMEM;
    ptr = p;
    bytes = want;
    device = ar->device;
    arena = ar;
    return NYS_OK;
  }
  want = pool_round(want);
  int dev = 0;
  NYS_TRY_HIP(hipGetDevice(&dev));
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> g(P.mu);
    long best = -1;
    for (size_t i = 0; i < P.blocks.size(); ++i) {
      const PoolBlock& b = P.blocks[i];
      if (b.device != dev || b.bytes < want || b.bytes > 2 * want) continue;
      if (best >= 0 && b.bytes >= P.blocks[(size_t)best].bytes) continue;
      if (!pool_ready(b)) continue;
      best = (long)i;
    }
    if (best >= 0) {
      PoolBlock& b = P.blocks[(size_t)best];
      ptr = b.ptr;
      bytes = b.bytes;
      device = dev;
      pool_recycle_events(P, b);
      P.cached -= b.bytes;
      P.blocks.erase(P.blocks.begin() + best);
      return NYS_OK;
    }
  }
  if (hipMalloc(&ptr, want) != hipSuccess) {
    (void)hipGetLastError();
    // give the cached blocks of this device back and try once more
    {
      std::lock_guard<std::mutex> g(P.mu);
      pool_trim_locked(P, dev);
    }
    if (hipMalloc(&ptr, want) != hipSuccess) {
      ptr = nullptr;
      (void)hipGetLastError();
      return NYS_ERR_NOMEM;
    }
  }
  bytes = want;
  device = dev;
  return NYS_OK;
}

void DevBuf::release() {
  if (ptr == nullptr) return;
  if (arena) {
    // the context's later work is ordered after every use of the block
    arena->free(ptr, bytes);
    arena.reset();
    ptr = nullptr;
    bytes = 0;
    device = -1;
    return;
  }
  Pool& P = pool();
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != device) (void)hipSetDevice(device);
  bool cached = false;
  {
    std::lock_guard<std::mutex> g(P.mu);
    bool live = false;
    for (auto& s : P.streams) live = live || s.first == device;
    if (live && P.cached + bytes <= kPoolCap) {
      PoolBlock b{ptr, bytes, device, {}};
      bool ok = true;
      for (auto& s : P.streams) {
        if (s.first != device) continue;
        hipEvent_t e = nullptr;
        for (size_t i = P.spare_events.size(); i-- > 0;)
          if (P.spare_events[i].first == device) {
            e = P.spare_events[i].second;
            P.spare_events.erase(P.spare_events.begin() + (long)i);
            break;
          }
        if (e == nullptr && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
          ok = false;
          break;
        }
        b.evs.push_back(e);
        if (hipEventRecord(e, s.second) != hipSuccess) {
          ok = false;
          break;
        }
      }
      if (ok) {
        P.blocks.push_back(std::move(b));
        P.cached += bytes;
        cached = true;
      } else {
        (void)hipGetLastError();
        pool_recycle_events(P, b);
      }
    }
  }
  if (!cached) {
    (void)hipDeviceSynchronize();   // kernels in flight may still use the block
    (void)hipFree(ptr);
  }
  if (cur != device) (void)hipSetDevice(cur);
  ptr = nullptr;
  bytes = 0;
  device = -1;
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

nys_status validate_dense(const nys_dense* A) {
  if (A == nullptr || A->data == nullptr) return NYS_ERR_INVALID;
  if (A->n < 0 || A->d < 1 || A->ld < A->d) return NYS_ERR_INVALID;
  if (A->dtype == NYS_CSR) {
    const nys_sparse_s* S = static_cast<const nys_sparse_s*>(A->data);
    return (S->n == A->n && S->d == A->d) ? NYS_OK : NYS_ERR_INVALID;
  }
  if (A->dtype != NYS_F32 && A->dtype != NYS_F64) return NYS_ERR_INVALID;
  return NYS_OK;
}

nys_status check_vector(nys_ctx ctx, const double* v, int64_t n, int kind) {
  if (v == nullptr || n <= 0) return NYS_OK;
  NYS_TRY(ctx->check.reserve(256));
  int* flag = ctx->check.as<int>();
  NYS_TRY_HIP(hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
  NYS_TRY(launch_check_vec(v, n, kind, flag, ctx->stream));
  NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, flag, sizeof(int), hipMemcpyDeviceToHost,
                             ctx->stream));
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  int bits = 0;
  std::memcpy(&bits, ctx->host_pinned, sizeof(int));
  if (bits & kCheckNonfinite) return NYS_ERR_NONFINITE;
  if (bits & kCheckBad) return NYS_ERR_INVALID;
  return NYS_OK;
}

// Carves the PCG workspace out of the context buffers.
nys_status pcg_workspace(nys_ctx ctx, const GramPlan& pl, int64_t d, int max_iter, PcgWs* ws) {
  const size_t yb = align_up(sizeof(double) * ((size_t)pl.ny() * pl.ldy));
  const size_t ypb = yb + align_up(sizeof(double) * (size_t)std::max(pl.nq(), 1)) +
                     align_up(sizeof(double) * pl.tmp_doubles());
  NYS_TRY(ctx->ypart.reserve(ypb));
  ws->ypart = ctx->ypart.as<double>();
  ws->qpart = reinterpret_cast<double*>(reinterpret_cast<char*>(ctx->ypart.ptr) + yb);
  const size_t nv = align_up(sizeof(double) * d);
  const size_t cb = align_up(sizeof(double) * kCvecDoubles);
  const size_t vb = 3 * nv + cb + align_up(sizeof(double) * kWyRing);
  NYS_TRY(ctx->vecs.reserve(vb));
  char* v = static_cast<char*>(ctx->vecs.ptr);
  ws->w = reinterpret_cast<double*>(v);
  ws->p = reinterpret_cast<double*>(v + nv);
  ws->cvec = reinterpret_cast<double*>(v + 2 * nv);
  ws->wy = reinterpret_cast<double*>(v + 2 * nv + cb);
  ws->w2 = reinterpret_cast<double*>(v + 2 * nv + cb + align_up(sizeof(double) * kWyRing));
  ws->rj = red_block(pl.ny());
  ws->nred = nblk(d, ws->rj);
  ws->nvec = nblk(d, vec_block(d));
  const size_t sb = align_up(sizeof(PcgDev)) + 4 * align_up(sizeof(double) * ws->nred) +
                    align_up(sizeof(double) * ws->nvec);
  NYS_TRY(ctx->small.reserve(sb));
  char* s = static_cast<char*>(ctx->small.ptr);
  ws->st = reinterpret_cast<PcgDev*>(s);
  s += align_up(sizeof(PcgDev));
  ws->wwpart = reinterpret_cast<double*>(s);
  s += align_up(sizeof(double) * ws->nred);
  ws->rrpart = reinterpret_cast<double*>(s);
  s += align_up(sizeof(double) * ws->nred);
  ws->pppart = reinterpret_cast<double*>(s);
  s += align_up(sizeof(double) * ws->nvec);
  ws->wwpart2 = reinterpret_cast<double*>(s);
  s += align_up(sizeof(double) * ws->nred);
  ws->rrpart2 = reinterpret_cast<double*>(s);
  return NYS_OK;
}

nys_status ctx_gram(nys_ctx ctx, const nys_dense& A, const GramPlan& plan, int mode,
                    const double* p, const double* aux, double* auxout, double* ypart,
                    double* qpart, const int* done, PcgDev* note, int note_seq) {
  if (note != nullptr && done == nullptr) return NYS_ERR_INVALID;
  if (plan.symv && (mode != kModeHess || aux != nullptr)) return NYS_ERR_INVALID;
  if (plan.sparse != nullptr) {
    const bool ev = ctx->prof_on;
    if (ev && ctx->prof_used + 2 > ctx->prof_ev.size())
      for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        NYS_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        ctx->prof_ev.push_back(e);
      }
    NYS_TRY(launch_sparse_pair(plan.sparse, plan, mode, p, aux, auxout, ypart, qpart, done,
                               ctx->stream, ev ? ctx->prof_ev[ctx->prof_used] : nullptr,
                               ev ? ctx->prof_ev[ctx->prof_used + 1] : nullptr, note,
                               note_seq));
    if (ev) ctx->prof_used += 2;
    return NYS_OK;
  }
  if (plan.wide) {
    const bool ev = ctx->prof_on;
    if (ev && ctx->prof_used + 2 > ctx->prof_ev.size())
      for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        NYS_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        ctx->prof_ev.push_back(e);
      }
    NYS_TRY(launch_wide(A, plan, mode, p, aux, auxout, ypart, qpart, done, ctx->stream,
                        ev ? ctx->prof_ev[ctx->prof_used] : nullptr,
                        ev ? ctx->prof_ev[ctx->prof_used + 1] : nullptr, note, note_seq));
    if (ev && plan.grid > 0 && A.n > 0) ctx->prof_used += 2;
    return NYS_OK;
  }
  if (plan.grid == 0 || A.n == 0) {
    // nothing to launch: publish the state from a one-thread kernel instead
    if (note != nullptr) NYS_TRY(launch_note(reinterpret_cast<const PcgDev*>(done), note, note_seq,
                                             ctx->stream));
    return NYS_OK;
  }
  if (!ctx->prof_on)
    return plan.symv ? launch_symv(A, plan, p, ypart, qpart, done, ctx->stream, nullptr, nullptr,
                                   note, note_seq)
                     : launch_gram(A, plan, mode, p, aux, auxout, ypart, qpart, done, ctx->stream,
                                   nullptr, nullptr, note, note_seq);
  if (ctx->prof_used + 2 > ctx->prof_ev.size()) {
    for (int i = 0; i < 2; ++i) {
      // timing-only events: no system-scope fence (cache writeback) at each
      // record, which would lengthen the measured kernel itself
      hipEvent_t e;
      NYS_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      ctx->prof_ev.push_back(e);
    }
  }
  if (plan.symv)
    NYS_TRY(launch_symv(A, plan, p, ypart, qpart, done, ctx->stream, ctx->prof_ev[ctx->prof_used],
                        ctx->prof_ev[ctx->prof_used + 1], note, note_seq));
  else
    NYS_TRY(launch_gram(A, plan, mode, p, aux, auxout, ypart, qpart, done, ctx->stream,
                        ctx->prof_ev[ctx->prof_used], ctx->prof_ev[ctx->prof_used + 1], note,
                        note_seq));
  ctx->prof_used += 2;
  return NYS_OK;
}

nys_status ctx_gram_plan(nys_ctx ctx, const nys_dense& A, GramPlan* out) {
  if (const nys_sparse_s* S = as_sparse(A)) {
    *out = make_sparse_plan(S);
    return NYS_OK;
  }
  if (A.d > gram_max_cols(A.dtype)) {
    // wider than one workgroup's row: the two-pass form, one fixed shape
    *out = make_wide_plan(A, ctx->num_cu);
    return NYS_OK;
  }
  const char* forced = getenv("NYSADMM_GRAM_PLAN");
  const char* tune = getenv("NYSADMM_TUNE");
  if (forced != nullptr || (tune != nullptr && tune[0] == '0') || A.n < 4096) {
    *out = make_gram_plan(A, ctx->num_cu);
    return NYS_OK;
  }
  const int esize = A.dtype == NYS_F64 ? 8 : 4;
  const bool aligned = ((uintptr_t)A.data % 16 == 0) && ((A.ld * esize) % 16 == 0);
  char key[160];
  snprintf(key, sizeof(key), "%d|%lld|%lld|%lld|%d", (int)A.dtype, (long long)A.n,
           (long long)A.d, (long long)A.ld, (int)aligned);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    GramPlan pl = it->second;
    pl.aligned = aligned;
    // the grid depends only on n and the shape; recompute for this pointer
    *out = pl;
    return NYS_OK;
  }
  std::vector<GramPlan> cands = gram_candidates(A, ctx->num_cu);
  if (cands.empty()) {
    *out = make_gram_plan(A, ctx->num_cu);
    return NYS_OK;
  }
  int gmax = 0;
  for (auto& c : cands) gmax = std::max(gmax, c.grid);
  const int ldy = cands[0].ldy;
  // scratch: partial sums of the widest candidate, and an input vector of zeros
  DevBuf scratch;
  const size_t yb = align_up(sizeof(double) * (size_t)gmax * ldy);
  NYS_TRY(scratch.reserve(yb + align_up(sizeof(double) * gmax) + align_up(sizeof(double) * A.d)));
  double* yp = scratch.as<double>();
  double* qp = reinterpret_cast<double*>(static_cast<char*>(scratch.ptr) + yb);
  double* pv = reinterpret_cast<double*>(static_cast<char*>(scratch.ptr) + yb +
                                         align_up(sizeof(double) * gmax));
  NYS_TRY_HIP(hipMemsetAsync(pv, 0, sizeof(double) * A.d, ctx->stream));
  hipEvent_t e0, e1;
  NYS_TRY_HIP(hipEventCreate(&e0));
  NYS_TRY_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  GramPlan bestp = cands[0];
  for (const GramPlan& c : cands) {
    if (launch_gram(A, c, kModeHess, pv, nullptr, nullptr, yp, qp, nullptr, ctx->stream) != NYS_OK)
      continue;
    (void)hipEventRecord(e0, ctx->stream);
    for (int r = 0; r < 3; ++r)
      (void)launch_gram(A, c, kModeHess, pv, nullptr, nullptr, yp, qp, nullptr, ctx->stream);
    (void)hipEventRecord(e1, ctx->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms > 0.f && ms < best) {
      best = ms;
      bestp = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  scratch.release();
  ctx->plans[key] = bestp;
  if (getenv("NYSADMM_VERBOSE"))
    fprintf(stderr, "nysadmm: matvec plan for %lld x %lld: waves %d, chunks %d, rows %d, %d wg/CU, "
            "grid %d (%.1f us, %zu candidates)\n", (long long)A.n, (long long)A.d, bestp.waves,
            bestp.cpl, bestp.rows, bestp.per_cu, bestp.grid, 1e3 * best / 3, cands.size());
  *out = bestp;
  return NYS_OK;
}

nys_status read_pcg_state(nys_ctx ctx, const PcgWs& ws, PcgDev* out) {
  NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, ws.st, sizeof(PcgDev), hipMemcpyDeviceToHost,
                             ctx->stream));
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(out, ctx->host_pinned, sizeof(PcgDev));
  return NYS_OK;
}

// Wait until the kernel of PCG iteration seq-1 has written its state into the
// pinned slot (sequence number seq in PcgDev::k).  The wait spins on the host
// memory; once the slot has stayed unwritten for a few milliseconds the stream
// is queried (PollPace) so that a failed stream returns an error, and a stream
// that has drained without the slot being written is reported as an internal
// error.
nys_status wait_slot(hipStream_t st, const char* slot, int seq, PcgDev* out) {
  const volatile PcgDev* v = reinterpret_cast<const volatile PcgDev*>(slot);
  PollPace pace;
  for (long n = 1;; ++n) {
    if (v->k == seq) break;
    if (pace.due(n)) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        if (v->k == seq) break;
        return NYS_ERR_HIP;
      }
      if (e != hipErrorNotReady) return NYS_ERR_HIP;
    }
    __builtin_ia32_pause();
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  std::memcpy(out, const_cast<const PcgDev*>(reinterpret_cast<const volatile PcgDev*>(slot)),
              sizeof(PcgDev));
  return NYS_OK;
}

// Algorithm Nystrom PCG (see pcg_solve in nysadmm.h).
nys_status pcg_run(nys_ctx ctx, const nys_dense& A, const double* D, double c, double rho,
                   nys_factor F, const double* rhs, double* x, const nys_pcg_opts& o,
                   nys_pcg_info* info, double abs_tol, int64_t hx_tag, const double* x_alt,
                   int* used_alt, bool symv) {
  if (used_alt) *used_alt = 0;
  const double tol_rel = o.tol_abs ? 0.0 : o.tol;
  const double tol_abs = o.tol_abs ? o.tol : abs_tol;
  const int64_t d = A.d;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 1000;
  const int ahead = o.check_every > 0 ? std::min(o.check_every, 4) : 2;
  const int max_restarts = o.max_restarts > 0 ? o.max_restarts : 2;
  GramPlan pl;
  if (symv) {
    if (D != nullptr || A.n != A.d) return NYS_ERR_INVALID;
    pl = make_symv_plan(A, ctx->num_cu);
  } else {
    NYS_TRY(ctx_gram_plan(ctx, A, &pl));
  }
  PcgWs ws;
  NYS_TRY(pcg_workspace(ctx, pl, d, max_iter, &ws));
  const double rho_eff = rho + c;
  hipStream_t st = ctx->stream;

  const int r = F ? F->r : 0;
  const void* U = F ? (F->use_u32 ? F->U32.ptr : F->U.ptr) : nullptr;
  const bool u32 = F ? F->use_u32 : false;
  const double* lam = F ? F->lam.as<double>() : nullptr;
  const double lam_s = (F && r > 0) ? F->lam_host[r - 1] : 0.0;

  int total_iters = 0, restarts = 0;
  PcgDev h{};
  nys_status status = NYS_OK;
  double true_rr = -1.0;
  for (;;) {
    NYS_TRY(launch_zero_state(ws.st, st));
    // w0 = rhs - H_rho x0 ; y0 = P^-1 w0 ; p0 = y0
    const AtbKey key{A.data, D, A.n, d, A.ld, x};
    if (hx_tag >= 0 && restarts == 0 && ctx->hx_tag == hx_tag && ctx->hx_key == key &&
        ctx->hx_rho == rho && ctx->hx_c == c) {
      // H_rho x0 from the previous solve's true-residual pass (x0 unchanged)
      NYS_TRY(launch_reduce_update(1, ws.ypart, 0, pl.ldy, ws.qpart, d, 1.0, ctx->hx.as<double>(),
                                   nullptr, ws.w, rhs, ws.wy, 0, nullptr, 0, ws.wwpart, ws.rrpart,
                                   ws.st, st, -1, false, ws.rj));
    } else {
      NYS_TRY(ctx_gram(ctx, A, pl, kModeHess, x, D, nullptr, ws.ypart, ws.qpart, nullptr));
      NYS_TRY(launch_reduce_update(1, ws.ypart, pl.ny(), pl.ldy, ws.qpart, d, rho_eff, x, nullptr,
                                   ws.w, rhs, ws.wy, 0, nullptr, 0, ws.wwpart, ws.rrpart, ws.st,
                                   st, pl.nq()));
    }
    ctx->hx_key = AtbKey{};
    if (x_alt != nullptr && restarts == 0) {
      // judge: residual of the candidate start next to that of x, decided on
      // the device (the smaller ||w|| wins; ties keep x)
      NYS_TRY(ctx_gram(ctx, A, pl, kModeHess, x_alt, D, nullptr, ws.ypart, ws.qpart, nullptr));
      NYS_TRY(launch_reduce_update(1, ws.ypart, pl.ny(), pl.ldy, ws.qpart, d, rho_eff, x_alt,
                                   nullptr, ws.w2, rhs, ws.wy, 0, nullptr, 0, ws.wwpart2,
                                   ws.rrpart2, ws.st, st, pl.nq()));
      NYS_TRY(launch_judge(ws.wwpart, ws.wwpart2, ws.nred, x, x_alt, ws.w, ws.w2, d, ws.st, st));
    }
    NYS_TRY(launch_precond_dot(U, u32, d, r, ws.w, ws.cvec, ws.st, ws.wwpart, ws.nred,
                               ws.rrpart, -1, 1, tol_rel, tol_abs, st));
    NYS_TRY(launch_precond_update(U, u32, d, r, lam, lam_s, rho, ws.cvec, ws.w, ws.p, ws.wy, 0,
                                  ws.wwpart, ws.nred, ws.pppart, ws.st, 1, st));
    // Iterations are enqueued `ahead` at a time beyond the last state the host
    // has read: the state after each iteration reaches a pinned host slot with
    // a sequence number (copied there by the first thread of the next
    // iteration's matvec kernel, or by a one-thread kernel when no iteration
    // follows), and the host waits only for the oldest iteration in flight, so
    // the GPU never idles on a host round trip or an event marker.  Iterations
    // queued after convergence return at once (every kernel checks
    // PcgDev::done).
    const int limit = max_iter - total_iters;
    char* slots = static_cast<char*>(ctx->host_pinned) + kPollOffset;
    int seqs[4] = {0, 0, 0, 0};
    auto slot_dev = [&](int k) {
      return reinterpret_cast<PcgDev*>(static_cast<char*>(ctx->host_pinned_dev) + kPollOffset +
                                       64 * (k % 4));
    };
    // large d: p^T v and ||w||^2 summed once per iteration (their partial
    // counts grow with d) instead of by every workgroup of the vector kernels
    const bool pre = d > kPreReduceDim;
    auto enqueue = [&](int k) -> nys_status {
      NYS_TRY(ctx_gram(ctx, A, pl, kModeHess, ws.p, D, nullptr, ws.ypart, ws.qpart, &ws.st->done,
                       k > 0 ? slot_dev(k - 1) : nullptr, k > 0 ? seqs[(k - 1) % 4] : 0));
      if (pre)
        NYS_TRY(launch_pcg_scalar(0, ws.qpart, pl.nq(), ws.pppart, ws.nvec, rho_eff, ws.st, st));
      NYS_TRY(launch_reduce_update(0, ws.ypart, pl.ny(), pl.ldy, ws.qpart, d, rho_eff, ws.p, x,
                                   ws.w, nullptr, ws.wy, k, ws.pppart, ws.nvec, ws.wwpart, nullptr,
                                   ws.st, st, pl.nq(), pre));
      if (pre) NYS_TRY(launch_pcg_scalar(1, ws.wwpart, ws.nred, nullptr, 0, 0.0, ws.st, st));
      NYS_TRY(launch_precond_dot(U, u32, d, r, ws.w, ws.cvec, ws.st, ws.wwpart, ws.nred, nullptr,
                                 k, 0, tol_rel, tol_abs, st, pre));
      // sequence numbers are unique per context, so a late write from an
      // earlier solve's queued iteration can never be taken for this one
      const int seq = ctx->poll_seq = (ctx->poll_seq % 1000000000) + 1;
      seqs[k % 4] = seq;
      // large d: c, g = s o c and sum s c^2 reduced once (k_c_reduce) rather
      // than from the slices by every workgroup of the update
      double* gvec = ws.cvec + (size_t)1024 * kDotSlicesMax;
      if (pre) NYS_TRY(launch_c_reduce(ws.cvec, d, r, lam, lam_s, rho, gvec, ws.st, st));
      NYS_TRY(launch_precond_update(U, u32, d, r, lam, lam_s, rho, ws.cvec, ws.w, ws.p, ws.wy, k,
                                    ws.wwpart, ws.nred, ws.pppart, ws.st, 0, st, nullptr, seq,
                                    pre, pre ? gvec : nullptr));
      return NYS_OK;
    };
    int it = 0, consumed = 0;
    for (;;) {
      while (it < limit && it - consumed < ahead) {
        NYS_TRY(enqueue(it));
        ++it;
      }
      if (it == consumed) {   // nothing in flight: the iteration limit is reached
        NYS_TRY(read_pcg_state(ctx, ws, &h));
        break;
      }
      // no iteration follows the oldest one in flight: publish its state
      if (it == consumed + 1)
        NYS_TRY(launch_note(ws.st, slot_dev(consumed), seqs[consumed % 4], st));
      NYS_TRY(wait_slot(st, slots + 64 * (consumed % 4), seqs[consumed % 4], &h));
      ++consumed;
      if (h.done) break;
    }
    if (restarts == 0 && used_alt) *used_alt = (h.flags & kFlagAltStart) ? 1 : 0;
    total_iters += h.done ? h.iters : it;
    // launches enqueued after convergence return at once; not counted as work
    if (ctx->prof_on && h.done && it > h.iters) ctx->prof_skipped += it - h.iters;
    if (h.flags & kFlagZeroRhs) {
      NYS_TRY_HIP(hipMemsetAsync(x, 0, sizeof(double) * d, st));
      status = NYS_OK;
      true_rr = 0.0;
      break;
    }
    if (h.flags & kFlagNonfinite) {
      status = NYS_ERR_NONFINITE;
      break;
    }
    if (h.flags & kFlagBreakdown) {
      status = NYS_ERR_BREAKDOWN;
      break;
    }
    if (!h.done) status = NYS_ERR_MAXITER;
    if (!o.true_residual) {
      // no true-residual pass: H_rho x of the last iterate is rhs - w, the
      // recursive residual (consistent with x at every iteration)
      if (hx_tag >= 0) {
        NYS_TRY(ctx->hx.reserve(sizeof(double) * d));
        NYS_TRY(launch_reduce_update(4, nullptr, 0, 0, nullptr, d, 0.0, nullptr,
                                     ctx->hx.as<double>(), ws.w, rhs, nullptr, 0, nullptr, 0,
                                     nullptr, nullptr, ws.st, st));
        ctx->hx_key = key;
        ctx->hx_rho = rho;
        ctx->hx_c = c;
        ctx->hx_tag = hx_tag + 1;
      }
      break;
    }
    // true residual rhs - H_rho x with FP64 accumulation (H_rho x kept when asked)
    double* hx_out = nullptr;
    if (hx_tag >= 0) {
      NYS_TRY(ctx->hx.reserve(sizeof(double) * d));
      hx_out = ctx->hx.as<double>();
    }
    NYS_TRY(ctx_gram(ctx, A, pl, kModeHess, x, D, nullptr, ws.ypart, ws.qpart, nullptr));
    NYS_TRY(launch_reduce_update(2, ws.ypart, pl.ny(), pl.ldy, ws.qpart, d, rho_eff, x, hx_out,
                                 ws.w, rhs, ws.wy, 0, nullptr, 0, ws.wwpart, nullptr, ws.st, st,
                                 pl.nq()));
    if (hx_tag >= 0) {
      ctx->hx_key = key;
      ctx->hx_rho = rho;
      ctx->hx_c = c;
      ctx->hx_tag = hx_tag + 1;
    }
    NYS_TRY(launch_precond_dot(U, u32, d, 0, ws.w, ws.cvec, ws.st, ws.wwpart, ws.nred, nullptr,
                               0, 3, 0.0, 0, st));
    NYS_TRY(read_pcg_state(ctx, ws, &h));
    true_rr = h.true_rr;
    if (!(true_rr <= h.thr2) && status == NYS_OK && restarts < max_restarts &&
        total_iters < max_iter) {
      ++restarts;
      continue;
    }
    if (!(true_rr <= h.thr2) && status == NYS_OK) status = NYS_ERR_MAXITER;
    break;
  }
  if (info) {
    info->iters = total_iters;
    info->restarts = restarts;
    info->rhs_norm = std::sqrt(h.rr);
    info->res_norm = std::sqrt(h.ww);
    info->true_res_norm = true_rr >= 0 ? std::sqrt(true_rr) : -1.0;
    info->status = status;
  }
  return status;
}

}  // namespace nys

using namespace nys;

extern "C" {

const char* nys_status_string(nys_status s) {
  switch (s) {
    case NYS_OK: return "ok";
    case NYS_ERR_INVALID: return "invalid argument";
    case NYS_ERR_HIP: return g_last_err[0] ? g_last_err : "HIP runtime error";
    case NYS_ERR_NOT_SPD: return "Cholesky of Omega^T Y_nu failed after shift retries";
    case NYS_ERR_BREAKDOWN: return "PCG breakdown: p^T H p <= 0";
    case NYS_ERR_MAXITER: return "PCG reached max_iter above tolerance";
    case NYS_ERR_NONFINITE: return "non-finite value";
    case NYS_ERR_NOMEM: return "device allocation failed";
    case NYS_ERR_NOT_CONVERGED: return "eigensolver did not converge";
  }
  return "unknown status";
}

nys_status nys_ctx_create(int device, void* hip_stream, nys_ctx* out) {
  if (out == nullptr) return NYS_ERR_INVALID;
  *out = nullptr;
  int ndev = 0;
  NYS_TRY_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(device));
  nys_ctx c = new (std::nothrow) nys_ctx_s();
  if (c == nullptr) return NYS_ERR_NOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cu = prop.multiProcessorCount;
  if (hipHostMalloc(&c->host_pinned, kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return NYS_ERR_NOMEM;
  }
  pool_register_stream(device, c->stream);
  if (hipHostGetDevicePointer(&c->host_pinned_dev, c->host_pinned, 0) != hipSuccess) {
    nys_ctx_destroy(c);
    return NYS_ERR_HIP;
  }
  const nys_status ns = noalloc_init(device);
  if (ns != NYS_OK) {
    nys_ctx_destroy(c);
    return ns;
  }
  *out = c;
  return NYS_OK;
}

nys_status nys_ctx_destroy(nys_ctx ctx) {
  if (ctx == nullptr) return NYS_ERR_INVALID;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->ypart.release();
  ctx->hx.release();
  ctx->vecs.release();
  ctx->small.release();
  ctx->gemm_ws.release();
  ctx->core_ws.release();
  ctx->admm_ws.release();
  ctx->svm_ws.release();
  ctx->check.release();
  pool_unregister_stream(ctx->device, ctx->stream);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->pcg_ev) (void)hipEventDestroy(e);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (int k = 0; k < nys_ctx_s::kSideStreams; ++k) {
    if (ctx->side_stream[k]) (void)hipStreamDestroy(ctx->side_stream[k]);
    if (ctx->side_join[k]) (void)hipEventDestroy(ctx->side_join[k]);
  }
  if (ctx->side_fork) (void)hipEventDestroy(ctx->side_fork);
  delete ctx;
  return NYS_OK;
}

nys_status nys_ctx_profile_start(nys_ctx ctx) {
  if (ctx == nullptr) return NYS_ERR_INVALID;
  ctx->prof_on = true;
  ctx->prof_used = 0;
  ctx->prof_skipped = 0;
  return NYS_OK;
}

nys_status nys_ctx_profile_pcg_enable(nys_ctx ctx, int on) {
  if (ctx == nullptr) return NYS_ERR_INVALID;
  if (on && !ctx->pcg_time_on) ctx->pcg_used = 0;
  ctx->pcg_time_on = on != 0;
  return NYS_OK;
}

nys_status nys_ctx_profile_pcg(nys_ctx ctx, long* solves, double* total_ms) {
  if (ctx == nullptr) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  for (size_t i = 0; i + 1 < ctx->pcg_used; i += 2) {
    float ms = 0.f;
    NYS_TRY_HIP(hipEventElapsedTime(&ms, ctx->pcg_ev[i], ctx->pcg_ev[i + 1]));
    tot += ms;
  }
  if (solves) *solves = (long)(ctx->pcg_used / 2);
  if (total_ms) *total_ms = tot;
  return NYS_OK;
}

nys_status nys_ctx_profile_stop(nys_ctx ctx, long* launches, double* total_ms) {
  if (ctx == nullptr) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  for (size_t i = 0; i + 1 < ctx->prof_used; i += 2) {
    float ms = 0.f;
    NYS_TRY_HIP(hipEventElapsedTime(&ms, ctx->prof_ev[i], ctx->prof_ev[i + 1]));
    tot += ms;
  }
  if (launches) *launches = (long)(ctx->prof_used / 2) - ctx->prof_skipped;
  if (total_ms) *total_ms = tot;
  ctx->prof_on = false;
  ctx->prof_used = 0;
  return NYS_OK;
}

nys_status nys_ctx_set_stream(nys_ctx ctx, void* hip_stream) {
  if (ctx == nullptr) return NYS_ERR_INVALID;
  // workspace blocks are reused in stream order: finish the old stream's work
  if (ctx->arena) NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  // the block cache guards released blocks with events on every live stream
  pool_register_stream(ctx->device, static_cast<hipStream_t>(hip_stream));
  pool_unregister_stream(ctx->device, ctx->stream);
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return NYS_OK;
}

size_t nys_ctx_workspace_bytes(nys_ctx ctx) {
  if (ctx == nullptr) return 0;
  return ctx->ypart.bytes + ctx->vecs.bytes + ctx->small.bytes + ctx->gemm_ws.bytes +
         ctx->core_ws.bytes + ctx->admm_ws.bytes;
}

nys_status nys_ctx_set_workspace(nys_ctx ctx, void* dev_ptr, size_t bytes) {
  if (ctx == nullptr || (dev_ptr == nullptr) != (bytes == 0)) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  if (dev_ptr != nullptr) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, dev_ptr) != hipSuccess) {
      (void)hipGetLastError();
      return NYS_ERR_INVALID;
    }
    if (at.type != hipMemoryTypeDevice || at.device != ctx->device) return NYS_ERR_INVALID;
  }
  // the context's own buffers go back to where they came from; the cached
  // A^T b and H_rho x go with them
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  ctx->ypart.release();
  ctx->hx.release();
  ctx->vecs.release();
  ctx->small.release();
  ctx->gemm_ws.release();
  ctx->core_ws.release();
  ctx->admm_ws.release();
  ctx->svm_ws.release();
  ctx->check.release();
  ctx->atb_key = AtbKey{};
  ctx->atb_next_k = -1;
  ctx->hx_key = AtbKey{};
  ctx->hx_tag = -1;
  if (dev_ptr == nullptr) {
    ctx->arena.reset();
    return NYS_OK;
  }
  auto ar = std::make_shared<Arena>(dev_ptr, bytes, ctx->device);
  if (ar->bytes == 0) return NYS_ERR_INVALID;
  ctx->arena = ar;
  return NYS_OK;
}

size_t nys_ctx_workspace_peak(nys_ctx ctx) {
  if (ctx == nullptr || !ctx->arena) return 0;
  std::lock_guard<std::mutex> g(ctx->arena->mu);
  return ctx->arena->peak;
}

nys_status nys_workspace_query(nys_ctx ctx, const nys_dense* A, int r_max, int count,
                               size_t* bytes) {
  if (ctx == nullptr || bytes == nullptr || count < 1) return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(A));
  if (r_max < 0 || r_max >= A->d || r_max > 1024) return NYS_ERR_INVALID;
  const int64_t n = A->n, d = A->d;
  size_t total = 0;
  // matvec partial sums (the widest launch shape the tuner may pick), twice:
  // the tuner's trial buffer and the kept one
  size_t part = 0;
  if (const nys_sparse_s* S = as_sparse(*A)) {
    const GramPlan pl = make_sparse_plan(S);
    part = align_up(sizeof(double) * (size_t)pl.ny() * pl.ldy) +
           align_up(sizeof(double) * (size_t)std::max(pl.nq(), 1));
    total += sparse_handle_bytes(n, d, S->nnz);
  } else {
    std::vector<GramPlan> c;
    if (d > gram_max_cols(A->dtype)) {
      c.push_back(make_wide_plan(*A, ctx->num_cu));
    } else {
      c = gram_candidates(*A, ctx->num_cu);
      c.push_back(make_gram_plan(*A, ctx->num_cu));
    }
    for (const GramPlan& pl : c)
      part = std::max(part, align_up(sizeof(double) * (size_t)pl.ny() * pl.ldy) +
                                align_up(sizeof(double) * (size_t)std::max(pl.nq(), 1)) +
                                align_up(sizeof(double) * pl.tmp_doubles()));
  }
  total += 2 * part + align_up(sizeof(double) * d);
  // PCG vectors and scalars, H_rho x, the argument-check flag
  const size_t nv = align_up(sizeof(double) * d);
  total += 3 * nv + align_up(sizeof(double) * kCvecDoubles) +
           align_up(sizeof(double) * kWyRing);
  total += align_up(sizeof(PcgDev)) + 4 * align_up(sizeof(double) * (size_t)nblk(d, kRedBlock)) +
           align_up(sizeof(double) * (size_t)nblk(d, vec_block(d)));
  total += nv + 256;
  // ADMM vectors
  total += admm_ws_bytes(n, d);
  // sketch temporaries and the factors alive at once: one per instance when
  // they run batched, two for a logistic refresh (old and new)
  if (r_max > 0) {
    size_t tmp = 0, factor = 0;
    sketch_ws_bytes(*A, r_max, r_max, ctx->num_cu, &tmp, &factor);
    total += tmp + (size_t)std::max(count, 2) * factor;
  }
  if (count > 1) total += batch_workspace_bytes(count, n, d, std::max(r_max, 1));
  // first-fit fragmentation and 256-byte granularity
  total += total / 8 + (size_t(16) << 20);
  *bytes = total;
  return NYS_OK;
}

nys_status nys_factor_import(nys_ctx ctx, int64_t d, int r, const double* U,
                             const double* lambda_host, double nu, nys_factor* F) {
  if (ctx == nullptr || F == nullptr || U == nullptr || lambda_host == nullptr)
    return NYS_ERR_INVALID;
  if (d < 2 || r < 1 || r >= d || r > 1024) return NYS_ERR_INVALID;
  for (int i = 0; i < r; ++i) {
    if (!(lambda_host[i] >= 0.0) || !std::isfinite(lambda_host[i])) return NYS_ERR_INVALID;
    if (i > 0 && lambda_host[i] > lambda_host[i - 1]) return NYS_ERR_INVALID;
  }
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  nys_factor f = new (std::nothrow) nys_factor_s();
  if (f == nullptr) return NYS_ERR_NOMEM;
  f->d = d;
  f->r = r;
  f->cap = r;
  f->nu = nu;
  f->device = ctx->device;
  f->prec = NYS_F64;
  f->use_u32 = false;
  nys_status s = f->U.reserve(sizeof(double) * d * r);
  if (s == NYS_OK) s = f->lam.reserve(sizeof(double) * r);
  if (s != NYS_OK) {
    nys_factor_destroy(f);
    return s;
  }
  f->lam_host.assign(lambda_host, lambda_host + r);
  if (hipMemcpyAsync(f->U.ptr, U, sizeof(double) * d * r, hipMemcpyDeviceToDevice,
                     ctx->stream) != hipSuccess ||
      hipMemcpyAsync(f->lam.ptr, f->lam_host.data(), sizeof(double) * r, hipMemcpyHostToDevice,
                     ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    nys_factor_destroy(f);
    return NYS_ERR_HIP;
  }
  *F = f;
  return NYS_OK;
}

nys_status nys_factor_info(nys_factor F, int* rank, double* nu, double* lambda_s,
                           double* lambda_host) {
  if (F == nullptr) return NYS_ERR_INVALID;
  if (rank) *rank = F->r;
  if (nu) *nu = F->nu;
  if (lambda_s) *lambda_s = F->r > 0 ? F->lam_host[F->r - 1] : 0.0;
  if (lambda_host && F->r > 0) std::memcpy(lambda_host, F->lam_host.data(), sizeof(double) * F->r);
  return NYS_OK;
}

nys_status nys_factor_get_U(nys_ctx ctx, nys_factor F, double* U_out) {
  if (ctx == nullptr || F == nullptr || U_out == nullptr) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipMemcpyAsync(U_out, F->U.ptr, sizeof(double) * F->d * F->r,
                             hipMemcpyDeviceToDevice, ctx->stream));
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  return NYS_OK;
}

nys_status nys_factor_destroy(nys_factor F) {
  if (F == nullptr) return NYS_ERR_INVALID;
  (void)hipSetDevice(F->device);
  (void)hipDeviceSynchronize();
  F->U.release();
  F->U32.release();
  F->lam.release();
  F->Omega.release();
  F->Y.release();
  F->T.release();
  F->Mbase.release();
  delete F;
  return NYS_OK;
}

nys_status nys_precond_apply(nys_ctx ctx, nys_factor F, double rho, const double* w, double* y) {
  if (ctx == nullptr || F == nullptr || w == nullptr || y == nullptr) return NYS_ERR_INVALID;
  if (!(rho > 0.0) || F->r < 1) return NYS_ERR_INVALID;
  if (w == y) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  PcgWs ws;
  GramPlan pl;
  pl.grid = 0;
  pl.ldy = 64;
  NYS_TRY(pcg_workspace(ctx, pl, F->d, 1, &ws));
  const void* U = F->use_u32 ? F->U32.ptr : F->U.ptr;
  NYS_TRY(launch_precond_dot(U, F->use_u32, F->d, F->r, w, ws.cvec, ws.st, nullptr, 0, nullptr, 0,
                             2, 0.0, 0, ctx->stream));
  NYS_TRY(launch_precond_update(U, F->use_u32, F->d, F->r, F->lam.as<double>(),
                                F->lam_host[F->r - 1], rho, ws.cvec, w, y, nullptr, 0, nullptr, 0,
                                nullptr, ws.st, 2, ctx->stream));
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  return NYS_OK;
}

nys_status nys_hessian_apply(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                             double rho, const double* p, double* v, double* pv_host) {
  if (ctx == nullptr || p == nullptr || v == nullptr || p == v) return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(A));
  if (!(rho + c >= 0.0)) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  NYS_TRY(check_vector(ctx, D, A->n, 0));
  GramPlan pl;
  NYS_TRY(ctx_gram_plan(ctx, *A, &pl));
  PcgWs ws;
  NYS_TRY(pcg_workspace(ctx, pl, A->d, 1, &ws));
  NYS_TRY(ctx_gram(ctx, *A, pl, kModeHess, p, D, nullptr, ws.ypart, ws.qpart, nullptr));
  NYS_TRY(launch_reduce_update(3, ws.ypart, pl.ny(), pl.ldy, ws.qpart, A->d, rho + c, p, nullptr,
                               v, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, ws.st,
                               ctx->stream, pl.nq()));
  if (pv_host != nullptr) {
    NYS_TRY(launch_dot(v, p, A->d, &ws.st->true_rr, ctx->stream));
    PcgDev h;
    NYS_TRY(read_pcg_state(ctx, ws, &h));
    *pv_host = h.true_rr;
  }
  return NYS_OK;
}

nys_status pcg_solve(nys_ctx ctx, const nys_dense* A, const double* D, double c, double rho,
                     nys_factor F, const double* rhs, double* x, const nys_pcg_opts* opts,
                     nys_pcg_info* info) {
  if (ctx == nullptr || rhs == nullptr || x == nullptr || opts == nullptr)
    return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(A));
  if (!(rho > 0.0) || !(c >= 0.0) || !(opts->tol >= 0.0) || opts->max_iter < 0)
    return NYS_ERR_INVALID;
  if (F != nullptr && F->d != A->d) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  NYS_TRY(check_vector(ctx, D, A->n, 0));
  return pcg_run(ctx, *A, D, c, rho, F, rhs, x, *opts, info);
}

nys_status pcg_solve_sym(nys_ctx ctx, const nys_dense* K, double c, double rho, nys_factor F,
                         const double* rhs, double* x, const nys_pcg_opts* opts,
                         nys_pcg_info* info) {
  if (ctx == nullptr || rhs == nullptr || x == nullptr || opts == nullptr)
    return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(K));
  if (K->n != K->d || !(rho > 0.0) || !(c >= 0.0) || !(opts->tol >= 0.0) || opts->max_iter < 0)
    return NYS_ERR_INVALID;
  if (F != nullptr && F->d != K->d) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  return pcg_run(ctx, *K, nullptr, c, rho, F, rhs, x, *opts, info, 0.0, -1, nullptr, nullptr,
                 true);
}

}  // extern "C"
