// Bandwidth probe of the fused matvec pair through the C ABI, with a plain
// device copy of the same byte count as the reference for HBM counters.
//
//   gram_probe [n] [d] [reps] [f32|f64]
//
// A is filled with a constant byte pattern (values do not change the memory
// traffic).  Prints per-call times measured with HIP events.  The launch shape
// can be overridden with NYSADMM_GRAM_PLAN="waves,cpl,rows,wg_per_cu".
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "nysadmm.h"

#define CHECK(x)                                                                   \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));               \
      return 1;                                                                    \
    }                                                                              \
  } while (0)

int main(int argc, char** argv) {
  const long long n = argc > 1 ? atoll(argv[1]) : 100000;
  const long long d = argc > 2 ? atoll(argv[2]) : 4000;
  const int reps = argc > 3 ? atoi(argv[3]) : 20;
  const bool f64 = argc > 4 && strcmp(argv[4], "f64") == 0;
  const size_t es = f64 ? 8 : 4;
  const size_t bytes = (size_t)n * d * es;
  void *A = nullptr, *B = nullptr;
  double *p = nullptr, *v = nullptr;
  CHECK(hipMalloc(&A, bytes));
  CHECK(hipMalloc(&p, sizeof(double) * d));
  CHECK(hipMalloc(&v, sizeof(double) * d));
  CHECK(hipMemset(A, 0x3c, bytes));
  CHECK(hipMemset(p, 0x3f, sizeof(double) * d));
  nys_ctx ctx = nullptr;
  if (nys_ctx_create(0, nullptr, &ctx) != NYS_OK) return 1;
  nys_dense Ad = {n, d, d, f64 ? NYS_F64 : NYS_F32, A};
  for (int i = 0; i < 3; ++i)
    if (nys_hessian_apply(ctx, &Ad, nullptr, 0.0, 1e-4, p, v, nullptr) != NYS_OK) return 1;
  CHECK(hipDeviceSynchronize());
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  nys_ctx_profile_start(ctx);
  CHECK(hipEventRecord(e0, nullptr));
  for (int i = 0; i < reps; ++i)
    if (nys_hessian_apply(ctx, &Ad, nullptr, 0.0, 1e-4, p, v, nullptr) != NYS_OK) return 1;
  CHECK(hipEventRecord(e1, nullptr));
  CHECK(hipEventSynchronize(e1));
  long launches = 0;
  double kms = 0.0;
  nys_ctx_profile_stop(ctx, &launches, &kms);
  float ms = 0.f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  const char* plan = getenv("NYSADMM_GRAM_PLAN");
  printf("gram %lldx%lld %s plan=%s: kernel %.2f us (%.0f GB/s), call %.2f us (%.0f GB/s)\n", n,
         d, f64 ? "f64" : "f32", plan ? plan : "default", 1e3 * kms / launches,
         bytes / (kms / launches * 1e-3) / 1e9, 1e3 * ms / reps, bytes / (ms / reps * 1e-3) / 1e9);
  // reference: device-to-device copy of the same bytes
  CHECK(hipMalloc(&B, bytes));
  CHECK(hipMemcpy(B, A, bytes, hipMemcpyDeviceToDevice));
  CHECK(hipEventRecord(e0, nullptr));
  CHECK(hipMemcpyAsync(B, A, bytes, hipMemcpyDeviceToDevice, nullptr));
  CHECK(hipEventRecord(e1, nullptr));
  CHECK(hipEventSynchronize(e1));
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  printf("copy %zu bytes: %.2f us (%.0f GB/s read+write)\n", bytes, 1e3 * ms,
         2.0 * bytes / (ms * 1e-3) / 1e9);
  nys_ctx_destroy(ctx);
  CHECK(hipFree(A));
  CHECK(hipFree(B));
  CHECK(hipFree(p));
  CHECK(hipFree(v));
  return 0;
}
