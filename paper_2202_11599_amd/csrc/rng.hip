// Gaussian entries of the Nystrom test matrix (Algorithm RandNysAppx starts
// from a standard Gaussian d x r matrix) drawn on the device: a counter-based
// generator, so that any sample of the stream is computed on its own, in any
// order, by any thread.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): four 32-bit counter words and two key words;
// each of the ten rounds multiplies words 0 and 2 by two odd constants,
// keeps both halves of the 64-bit products and mixes them with words 1 and 3
// and the key; the key grows by two Weyl constants between rounds.
// Box-Muller (1958) turns two uniforms into two independent N(0, 1) values.
//
// Stream layout: sample e of seed s comes from the Philox call with counter
// (q mod 2^32, q div 2^32, 0, 0), q = e div 4, key (s mod 2^32, s div 2^32);
// the call's words w0..w3 give samples 4q, 4q + 1 as the Box-Muller pair of
// (w0, w1) and 4q + 2, 4q + 3 as that of (w2, w3), with u = (w + 1/2) 2^-32.
#include <cstdint>

#include "internal.h"

namespace nys {
namespace {

constexpr uint32_t kPhiloxMul0 = 0xD2511F53u;
constexpr uint32_t kPhiloxMul1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeyl0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeyl1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t (&x)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    const uint64_t pa = (uint64_t)kPhiloxMul0 * x[0];
    const uint64_t pb = (uint64_t)kPhiloxMul1 * x[2];
    const uint32_t y0 = (uint32_t)(pb >> 32) ^ x[1] ^ k0;
    const uint32_t y2 = (uint32_t)(pa >> 32) ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = (uint32_t)pb;
    x[2] = y2;
    x[3] = (uint32_t)pa;
    k0 += kPhiloxWeyl0;
    k1 += kPhiloxWeyl1;
  }
}

// out[i] = sample offset + i, i < count (grid-stride over i)
__global__ __launch_bounds__(256) void k_gaussian(uint64_t seed, uint64_t offset, int64_t count,
                                                  double* __restrict__ out) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const uint64_t e = offset + (uint64_t)i;
    const uint64_t q = e >> 2;
    const int slot = (int)(e & 3u);
    uint32_t x[4] = {(uint32_t)q, (uint32_t)(q >> 32), 0u, 0u};
    philox4x32_10(x, k0, k1);
    const uint32_t wa = slot < 2 ? x[0] : x[2];
    const uint32_t wb = slot < 2 ? x[1] : x[3];
    const double u1 = ((double)wa + 0.5) * 0x1p-32;
    const double u2 = ((double)wb + 0.5) * 0x1p-32;
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    out[i] = (slot & 1) ? rad * sn : rad * cs;
  }
}

}  // namespace
}  // namespace nys

using namespace nys;

extern "C" {

nys_status nys_gaussian(nys_ctx ctx, uint64_t seed, uint64_t offset, int64_t count, double* out) {
  if (ctx == nullptr || count < 0 || (count > 0 && out == nullptr)) return NYS_ERR_INVALID;
  if (count == 0) return NYS_OK;
  if (offset > UINT64_MAX - (uint64_t)count) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, (int64_t)1 << 20);
  hipLaunchKernelGGL(k_gaussian, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, seed, offset,
                     count, out);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

}  // extern "C"
