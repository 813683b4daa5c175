// Hessian-vector product without any device allocation, for callers that
// cannot allocate (HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Same product as nys_hessian_apply,
//     v = (A^T diag(D) A + (c + rho) I) p        (eq. ADMMSubProb),
// with the workgroup partial sums kept in a fixed-size scratch array that the
// library holds on every device it runs on until the process ends.
//
// The array is a file-scope __device__ symbol.  Its name, used in host code,
// is only a host-side stand-in: the device address is looked up once per
// device with hipGetSymbolAddress (noalloc_init, called by nys_ctx_create with
// that device current) and only that address is handed to kernels, fills and
// copies.  Every call on one device shares the array, so calls that overlap on
// one device (different streams) race; calls in one stream are ordered.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace nys {
namespace {

// partial sums: grid x ldy doubles (grid capped to fit), then the q partials,
// then the scalar slots
constexpr size_t kPartBytes = size_t(16) << 20;
constexpr size_t kQBytes = size_t(32) << 10;    // up to 4096 workgroups
constexpr size_t kSlotBytes = 256;              // p^T v (double) and the check flag (int)
constexpr size_t kScratchBytes = kPartBytes + kQBytes + kSlotBytes;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  return g_scratch[device];
}

}  // namespace

nys_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return NYS_ERR_INVALID;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch[device] != nullptr) return NYS_OK;
  void* ptr = nullptr;
  NYS_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (ptr == nullptr) return NYS_ERR_HIP;
  g_scratch[device] = ptr;
  return NYS_OK;
}

}  // namespace nys

using namespace nys;

extern "C" {

nys_status nys_hessian_apply_noalloc(nys_ctx ctx, const nys_dense* A, const double* D, double c,
                                     double rho, const double* p, double* v, double* pv_host) {
  if (ctx == nullptr || p == nullptr || v == nullptr || p == v) return NYS_ERR_INVALID;
  NYS_TRY(validate_dense(A));
  if (A->dtype != NYS_F32 && A->dtype != NYS_F64) return NYS_ERR_INVALID;
  if (A->d > gram_max_cols(A->dtype)) return NYS_ERR_INVALID;
  if (!(rho + c >= 0.0)) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  char* base = static_cast<char*>(scratch_of(ctx->device));
  if (base == nullptr) return NYS_ERR_HIP;
  double* ypart = reinterpret_cast<double*>(base);
  double* qpart = reinterpret_cast<double*>(base + kPartBytes);
  double* pv_dev = reinterpret_cast<double*>(base + kPartBytes + kQBytes);
  int* flag = reinterpret_cast<int*>(base + kPartBytes + kQBytes + 64);
  hipStream_t st = ctx->stream;

  if (D != nullptr) {
    // D >= 0 and finite, as nys_hessian_apply checks it (synchronises)
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, flag);
    NYS_TRY(launch_check_vec(D, A->n, 0, flag, st));
    NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    NYS_TRY_HIP(hipStreamSynchronize(st));
    int bits = 0;
    std::memcpy(&bits, ctx->host_pinned, sizeof(int));
    if (bits & kCheckNonfinite) return NYS_ERR_NONFINITE;
    if (bits & kCheckBad) return NYS_ERR_INVALID;
  }

  // the heuristic launch shape (the autotuner would allocate), with at most as
  // many workgroups as the scratch holds partial rows for
  const int64_t ldy = (A->d + 63) / 64 * 64;
  const int64_t max_grid =
      std::min<int64_t>((int64_t)(kPartBytes / (sizeof(double) * ldy)),
                        (int64_t)(kQBytes / sizeof(double)));
  const GramPlan pl = make_gram_plan_capped(*A, ctx->num_cu, max_grid);
  if ((int64_t)pl.grid > max_grid || pl.ldy != ldy) return NYS_ERR_INVALID;
  NYS_TRY(launch_gram(*A, pl, kModeHess, p, D, nullptr, ypart, qpart, nullptr, st));
  NYS_TRY(launch_reduce_update(3, ypart, pl.ny(), pl.ldy, qpart, A->d, rho + c, p, nullptr, v,
                               nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr, st,
                               pl.nq()));
  if (pv_host != nullptr) {
    NYS_TRY(launch_dot(v, p, A->d, pv_dev, st));
    NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, pv_dev, sizeof(double), hipMemcpyDeviceToHost,
                               st));
    NYS_TRY_HIP(hipStreamSynchronize(st));
    std::memcpy(pv_host, ctx->host_pinned, sizeof(double));
  }
  return NYS_OK;
}

}  // extern "C"
