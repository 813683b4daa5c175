// Warm-start network for the PCG start of the ADMM x-subproblem (not part of
// the paper's method; the previous iterate stays the fallback):
//   f  = [U^T rhs, log gamma, log rho]           (features, n_in = r + 2)
//   f' = (f - mu) / sigma                          (standardisation, stored in the model)
//   h1 = gelu(f' W1 + b1), h2 = gelu(h1 W2 + b2), o = h2 W3 + b3
//   c  = o * s_out [+ (Lambda + rho I)^-1 U^T rhs], x0 = U c   (Nystrom basis)
// With the optional analytic skip the network learns the correction to the
// start that is exact on span(U) for exact eigenvectors.
// gelu(a) = a/2 (1 + erf(a/sqrt 2)).  Training minimises the weighted squared
// error (1/B) sum w_ik (o_ik - t_ik)^2 on standardised targets t = c* / s_out
// with Adam (bias-corrected).
//
// Precisions (nys_ws_set_precision):
//   FP64  everything FP64: the library's tiled FP64 GEMM and the elementwise
//         kernels here (the form that matches the FP64 oracle to rounding);
//   FP32  FP32 master weights, activations, gradients and Adam state; the
//         matrix products on FP32 MFMA (16x16x4) with FP32 accumulation;
//   BF16  as FP32, but every matrix-product operand (weights, activations,
//         back-propagated gradients) rounded to BF16 for the BF16 MFMA
//         (16x16x32) with FP32 accumulation; master weights, the elementwise
//         work (bias, GELU, loss) and Adam stay FP32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace nys {
namespace {

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

__device__ __forceinline__ double gelu_d(double a) {
  return 0.5 * a * (1.0 + erf(a * 0.70710678118654752440));
}
__device__ __forceinline__ double gelu_grad_d(double a) {
  return 0.5 * (1.0 + erf(a * 0.70710678118654752440)) +
         a * exp(-0.5 * a * a) * 0.39894228040143267794;
}

// A (M x N) += bias; H = gelu(A)
__global__ void k_bias_gelu(double* __restrict__ A, const double* __restrict__ bias, int64_t M,
                            int N, double* __restrict__ H) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M * N) return;
  const double a = A[e] + bias[e % N];
  A[e] = a;
  H[e] = gelu_d(a);
}

__global__ void k_bias(double* __restrict__ A, const double* __restrict__ bias, int64_t M, int N) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < M * N) A[e] += bias[e % N];
}

// Xn = (X - mu) / sigma   (M x N)
__global__ void k_standardise(const double* __restrict__ X, const double* __restrict__ mu,
                              const double* __restrict__ sig, int64_t M, int N,
                              double* __restrict__ Xn) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < M * N) Xn[e] = (X[e] - mu[e % N]) / sig[e % N];
}

// g = 2 w (o - t) / B, loss partials per block
__global__ __launch_bounds__(256) void k_loss_grad(const double* __restrict__ O,
                                                   const double* __restrict__ Tg,
                                                   const double* __restrict__ W, int64_t MN,
                                                   int B, double* __restrict__ G,
                                                   double* __restrict__ part) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (e < MN) {
    const double r = O[e] - Tg[e];
    const double w = W ? W[e] : 1.0;
    l = w * r * r / B;
    G[e] = 2.0 * w * r / B;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// column sums of G (M x N) into out (N), one thread per column, fixed order
__global__ void k_colsum(const double* __restrict__ G, int64_t M, int N, double* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  double s = 0.0;
  for (int64_t i = 0; i < M; ++i) s += G[i * N + c];
  out[c] = s;
}

// gA = gH o gelu'(A)
__global__ void k_gelu_back(const double* __restrict__ gH, const double* __restrict__ A, int64_t n,
                            double* __restrict__ gA) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) gA[e] = gH[e] * gelu_grad_d(A[e]);
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *out = s;
}

__global__ void k_adam(double* __restrict__ p, const double* __restrict__ g, double* __restrict__ m,
                       double* __restrict__ v, int64_t n, double lr, double b1, double b2,
                       double eps, double c1, double c2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double ge = g[e];
  const double me = b1 * m[e] + (1.0 - b1) * ge;
  const double ve = b2 * v[e] + (1.0 - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  p[e] -= lr * (me / c1) / (sqrt(ve / c2) + eps);
}

// features [U^T rhs, log gamma, log rho] from the precomputed U^T rhs
__global__ void k_features(const double* __restrict__ c, int r, double lg, double lr,
                           double* __restrict__ f) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < r) f[i] = c[i];
  if (i == r) f[r] = lg;
  if (i == r + 1) f[r + 1] = lr;
}

// c = u / (lambda + rho)
__global__ void k_shift_div(const double* __restrict__ u, const double* __restrict__ lam, int r,
                            double rho, double* __restrict__ c) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < r) c[i] = u[i] / (lam[i] + rho);
}

// c = o * s_out (+ u / (lambda + rho) when the analytic skip is on)
__global__ void k_scale(const double* __restrict__ o, const double* __restrict__ s, int n,
                        const double* __restrict__ u, const double* __restrict__ lam, double rho,
                        double* __restrict__ c) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double v = o[i] * s[i];
  if (u != nullptr) v += u[i] / (lam[i] + rho);
  c[i] = v;
}

// ------------------------------------------------ FP32 / BF16-MFMA form

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu_f(float a) {
  return 0.5f * a * (1.0f + erff(a * 0.70710678118654752440f));
}
__device__ __forceinline__ float gelu_grad_f(float a) {
  return 0.5f * (1.0f + erff(a * 0.70710678118654752440f)) +
         a * expf(-0.5f * a * a) * 0.39894228040143267794f;
}

// C(m, n) = alpha sum_k A(m, k) B(k, n) + beta C(m, n), FP32 in memory,
// A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn], C(m, n) = C[m scm + n scn].
// Workgroup: 4 wavefronts, a 32 x 32 tile of C; wavefront w owns the 16 x 16
// block (w & 1, w >> 1).  Per K step of 32, lane (q = lane / 16, i = lane % 16)
// takes A(row i, k0 + 8q .. 8q + 7) and B(k0 + 8q .. 8q + 7, column i), zero
// outside the matrices; the accumulator element v of the lane is C(4q + v, i).
// BF: the eight operands are rounded to BF16 and one 16x16x32 BF16 MFMA
// consumes them; otherwise eight 16x16x4 FP32 MFMAs (lane group q supplies
// k = 8q + s at step s).  The operands are tiny and cache-resident, so they
// are read straight from memory without staging.
template <bool BF>
__global__ __launch_bounds__(256) void k_mlp_gemm(int M, int N, int K, const float* __restrict__ A,
                                                  int64_t sam, int64_t sak,
                                                  const float* __restrict__ B, int64_t sbk,
                                                  int64_t sbn, float* __restrict__ C, int64_t scm,
                                                  int64_t scn, float alpha, float beta) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, i = lane & 15;
  const int row0 = blockIdx.x * 32 + 16 * (w & 1);
  const int col0 = blockIdx.y * 32 + 16 * (w >> 1);
  const int ar = row0 + i, bc = col0 + i;
  f4_t acc = (f4_t)0.0f;
  for (int k0 = 0; k0 < K; k0 += 32) {
    float av[8], bv[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = k0 + 8 * q + s;
      av[s] = (ar < M && k < K) ? A[(int64_t)ar * sam + (int64_t)k * sak] : 0.0f;
      bv[s] = (bc < N && k < K) ? B[(int64_t)k * sbk + (int64_t)bc * sbn] : 0.0f;
    }
    if constexpr (BF) {
      bf16x8_t a8, b8;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        a8[s] = (__bf16)av[s];
        b8[s] = (__bf16)bv[s];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b8, acc, 0, 0, 0);
    } else {
#pragma unroll
      for (int s = 0; s < 8; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = row0 + 4 * q + v;
    if (r < M && bc < N) {
      float* c = C + (int64_t)r * scm + (int64_t)bc * scn;
      *c = beta == 0.0f ? alpha * acc[v] : alpha * acc[v] + beta * *c;
    }
  }
}

__global__ void k_bias_gelu_f(float* __restrict__ A, const float* __restrict__ bias, int64_t M,
                              int N, float* __restrict__ H) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M * N) return;
  const float a = A[e] + bias[e % N];
  A[e] = a;
  H[e] = gelu_f(a);
}

__global__ void k_bias_f(float* __restrict__ A, const float* __restrict__ bias, int64_t M, int N) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < M * N) A[e] += bias[e % N];
}

// Xn = (X - mu) / sigma from the FP64 feature rows, rounded to FP32
__global__ void k_standardise_f(const double* __restrict__ X, const float* __restrict__ mu,
                                const float* __restrict__ sig, int64_t M, int N,
                                float* __restrict__ Xn) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < M * N) Xn[e] = ((float)X[e] - mu[e % N]) / sig[e % N];
}

// g = 2 w (o - t) / B in FP32 from FP32 outputs and FP64 targets/weights;
// the loss terms are summed in FP64 (per block, fixed order)
__global__ __launch_bounds__(256) void k_loss_grad_f(const float* __restrict__ O,
                                                     const double* __restrict__ Tg,
                                                     const double* __restrict__ W, int64_t MN,
                                                     int B, float* __restrict__ G,
                                                     double* __restrict__ part) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (e < MN) {
    const float r = O[e] - (float)Tg[e];
    const float w = W ? (float)W[e] : 1.0f;
    l = (double)w * (double)r * (double)r / B;
    G[e] = 2.0f * w * r / (float)B;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// column sums of G (M x N), one thread per column, fixed order, FP32
__global__ void k_colsum_f(const float* __restrict__ G, int64_t M, int N, float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  float s = 0.0f;
  for (int64_t i = 0; i < M; ++i) s += G[i * N + c];
  out[c] = s;
}

__global__ void k_gelu_back_f(const float* __restrict__ gH, const float* __restrict__ A, int64_t n,
                              float* __restrict__ gA) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) gA[e] = gH[e] * gelu_grad_f(A[e]);
}

__global__ void k_adam_f(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                         float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                         float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.0f - b1) * ge;
  const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

__global__ void k_f64_to_f32(const double* __restrict__ x, int64_t n, float* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) y[e] = (float)x[e];
}

__global__ void k_f32_to_f64(const float* __restrict__ x, int64_t n, double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) y[e] = (double)x[e];
}

// c = o * s_out (+ u / (lambda + rho)) from the FP32 network output
__global__ void k_scale_f(const float* __restrict__ o, const float* __restrict__ s, int n,
                          const double* __restrict__ u, const double* __restrict__ lam, double rho,
                          double* __restrict__ c) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double v = (double)o[i] * (double)s[i];
  if (u != nullptr) v += u[i] / (lam[i] + rho);
  c[i] = v;
}

}  // namespace
}  // namespace nys

struct nys_ws_model_s {
  int n_in = 0, hidden = 0, n_out = 0;
  int device = 0;
  int skip = 0;               // c = analytic coefficients + network output
  long t = 0;                 // Adam step count
  nys::DevBuf params;         // W1 b1 W2 b2 W3 b3 (row-major), then mu, sigma, s_out
  nys::DevBuf adam;           // m, v
  nys::DevBuf grads;
  nys::DevBuf act;            // activations workspace
  int64_t act_batch = 0;
  // FP32 / BF16-MFMA form: FP32 master weights (and mu, sigma, s_out), Adam
  // state, gradients and activations
  nys_dtype prec = NYS_F64;
  nys::DevBuf params32, adam32, grads32, act32;
  long t32 = 0;
};

namespace nys {

size_t ws_count(int ni, int h, int no) {
  return (size_t)ni * h + h + (size_t)h * h + h + (size_t)h * no + no;
}

struct WsPtrs {
  double *W1, *b1, *W2, *b2, *W3, *b3, *mu, *sig, *sout;
};

WsPtrs ws_ptrs(nys_ws_model m, double* base) {
  WsPtrs p;
  const int ni = m->n_in, h = m->hidden, no = m->n_out;
  p.W1 = base;
  p.b1 = p.W1 + (size_t)ni * h;
  p.W2 = p.b1 + h;
  p.b2 = p.W2 + (size_t)h * h;
  p.W3 = p.b2 + h;
  p.b3 = p.W3 + (size_t)h * no;
  p.mu = p.b3 + no;
  p.sig = p.mu + ni;
  p.sout = p.sig + ni;
  return p;
}

struct Act {
  double *Xn, *A1, *H1, *A2, *H2, *O, *G, *gH, *gA, *part;
};

nys_status ws_act(nys_ws_model m, int64_t B, Act* a) {
  const int ni = m->n_in, h = m->hidden, no = m->n_out;
  const size_t need = (size_t)B * (ni + 4 * h + 2 * no + h + h) + blocks(B * std::max(no, h)) + 64;
  NYS_TRY(m->act.reserve(sizeof(double) * need));
  double* p = m->act.as<double>();
  a->Xn = p;
  p += B * ni;
  a->A1 = p;
  p += B * h;
  a->H1 = p;
  p += B * h;
  a->A2 = p;
  p += B * h;
  a->H2 = p;
  p += B * h;
  a->O = p;
  p += B * no;
  a->G = p;
  p += B * no;
  a->gH = p;
  p += B * h;
  a->gA = p;
  p += B * h;
  a->part = p;
  return NYS_OK;
}

// forward of B standardised rows into a.O (and the activations for backward)
nys_status ws_forward(nys_ctx ctx, nys_ws_model m, const double* X, int64_t B, Act* a) {
  hipStream_t st = ctx->stream;
  const int ni = m->n_in, h = m->hidden, no = m->n_out;
  WsPtrs p = ws_ptrs(m, m->params.as<double>());
  hipLaunchKernelGGL(k_standardise, dim3(blocks(B * ni)), dim3(256), 0, st, X, p.mu, p.sig, B, ni,
                     a->Xn);
  NYS_TRY(gemm64(st, (int)B, h, ni, a->Xn, false, ni, 1, p.W1, false, h, 1, a->A1, h, 1, 1.0, 0.0,
                 nullptr, 0));
  hipLaunchKernelGGL(k_bias_gelu, dim3(blocks(B * h)), dim3(256), 0, st, a->A1, p.b1, B, h, a->H1);
  NYS_TRY(gemm64(st, (int)B, h, h, a->H1, false, h, 1, p.W2, false, h, 1, a->A2, h, 1, 1.0, 0.0,
                 nullptr, 0));
  hipLaunchKernelGGL(k_bias_gelu, dim3(blocks(B * h)), dim3(256), 0, st, a->A2, p.b2, B, h, a->H2);
  NYS_TRY(gemm64(st, (int)B, no, h, a->H2, false, h, 1, p.W3, false, no, 1, a->O, no, 1, 1.0, 0.0,
                 nullptr, 0));
  hipLaunchKernelGGL(k_bias, dim3(blocks(B * no)), dim3(256), 0, st, a->O, p.b3, B, no);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

// loss (device scalar at *loss_dev) and gradients into m->grads
nys_status ws_backward(nys_ctx ctx, nys_ws_model m, const double* Tg, const double* Wt, int64_t B,
                       Act* a, double* loss_dev) {
  hipStream_t st = ctx->stream;
  const int ni = m->n_in, h = m->hidden, no = m->n_out;
  WsPtrs p = ws_ptrs(m, m->params.as<double>());
  WsPtrs g = ws_ptrs(m, m->grads.as<double>());
  const unsigned nb = blocks(B * no);
  hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, st, a->O, Tg, Wt, B * no, (int)B, a->G,
                     a->part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, a->part, (int)nb, loss_dev);
  // layer 3
  NYS_TRY(gemm64(st, h, no, (int)B, a->H2, false, 1, h, a->G, false, no, 1, g.W3, no, 1, 1.0, 0.0,
                 nullptr, 0));
  hipLaunchKernelGGL(k_colsum, dim3(blocks(no)), dim3(256), 0, st, a->G, B, no, g.b3);
  NYS_TRY(gemm64(st, (int)B, h, no, a->G, false, no, 1, p.W3, false, 1, no, a->gH, h, 1, 1.0, 0.0,
                 nullptr, 0));
  hipLaunchKernelGGL(k_gelu_back, dim3(blocks(B * h)), dim3(256), 0, st, a->gH, a->A2, B * h, a->gA);
  // layer 2
  NYS_TRY(gemm64(st, h, h, (int)B, a->H1, false, 1, h, a->gA, false, h, 1, g.W2, h, 1, 1.0, 0.0,
                 nullptr, 0));
  hipLaunchKernelGGL(k_colsum, dim3(blocks(h)), dim3(256), 0, st, a->gA, B, h, g.b2);
  NYS_TRY(gemm64(st, (int)B, h, h, a->gA, false, h, 1, p.W2, false, 1, h, a->gH, h, 1, 1.0, 0.0,
                 nullptr, 0));
  hipLaunchKernelGGL(k_gelu_back, dim3(blocks(B * h)), dim3(256), 0, st, a->gH, a->A1, B * h, a->gA);
  // layer 1
  NYS_TRY(gemm64(st, ni, h, (int)B, a->Xn, false, 1, ni, a->gA, false, h, 1, g.W1, h, 1, 1.0, 0.0,
                 nullptr, 0));
  hipLaunchKernelGGL(k_colsum, dim3(blocks(h)), dim3(256), 0, st, a->gA, B, h, g.b1);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

// ---- FP32 / BF16-MFMA form
struct WsPtrs32 {
  float *W1, *b1, *W2, *b2, *W3, *b3, *mu, *sig, *sout;
};

WsPtrs32 ws_ptrs32(nys_ws_model m, float* base) {
  WsPtrs32 p;
  const int ni = m->n_in, h = m->hidden, no = m->n_out;
  p.W1 = base;
  p.b1 = p.W1 + (size_t)ni * h;
  p.W2 = p.b1 + h;
  p.b2 = p.W2 + (size_t)h * h;
  p.W3 = p.b2 + h;
  p.b3 = p.W3 + (size_t)h * no;
  p.mu = p.b3 + no;
  p.sig = p.mu + ni;
  p.sout = p.sig + ni;
  return p;
}

struct Act32 {
  float *Xn, *A1, *H1, *A2, *H2, *O, *G, *gH, *gA;
  double* part;
};

nys_status ws_act32(nys_ws_model m, int64_t B, Act32* a) {
  const int ni = m->n_in, h = m->hidden, no = m->n_out;
  const size_t nf = (size_t)B * (ni + 6 * h + 2 * no);
  const size_t nd = blocks(B * std::max(no, h)) + 64;
  NYS_TRY(m->act32.reserve(sizeof(float) * nf + 256 + sizeof(double) * nd));
  float* p = m->act32.as<float>();
  a->Xn = p;
  p += B * ni;
  a->A1 = p;
  p += B * h;
  a->H1 = p;
  p += B * h;
  a->A2 = p;
  p += B * h;
  a->H2 = p;
  p += B * h;
  a->O = p;
  p += B * no;
  a->G = p;
  p += B * no;
  a->gH = p;
  p += B * h;
  a->gA = p;
  a->part = reinterpret_cast<double*>(m->act32.as<char>() + align_up(sizeof(float) * nf));
  return NYS_OK;
}

nys_status mlp_gemm(hipStream_t st, bool bf, int M, int N, int K, const float* A, int64_t sam,
                    int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C, int64_t scm,
                    int64_t scn) {
  const dim3 grid((unsigned)((M + 31) / 32), (unsigned)((N + 31) / 32));
  if (bf)
    hipLaunchKernelGGL(k_mlp_gemm<true>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn,
                       C, scm, scn, 1.0f, 0.0f);
  else
    hipLaunchKernelGGL(k_mlp_gemm<false>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk,
                       sbn, C, scm, scn, 1.0f, 0.0f);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status ws_forward32(nys_ctx ctx, nys_ws_model m, const double* X, int64_t B, Act32* a) {
  hipStream_t st = ctx->stream;
  const bool bf = m->prec == NYS_BF16;
  const int ni = m->n_in, h = m->hidden, no = m->n_out;
  WsPtrs32 p = ws_ptrs32(m, m->params32.as<float>());
  hipLaunchKernelGGL(k_standardise_f, dim3(blocks(B * ni)), dim3(256), 0, st, X, p.mu, p.sig, B,
                     ni, a->Xn);
  NYS_TRY(mlp_gemm(st, bf, (int)B, h, ni, a->Xn, ni, 1, p.W1, h, 1, a->A1, h, 1));
  hipLaunchKernelGGL(k_bias_gelu_f, dim3(blocks(B * h)), dim3(256), 0, st, a->A1, p.b1, B, h,
                     a->H1);
  NYS_TRY(mlp_gemm(st, bf, (int)B, h, h, a->H1, h, 1, p.W2, h, 1, a->A2, h, 1));
  hipLaunchKernelGGL(k_bias_gelu_f, dim3(blocks(B * h)), dim3(256), 0, st, a->A2, p.b2, B, h,
                     a->H2);
  NYS_TRY(mlp_gemm(st, bf, (int)B, no, h, a->H2, h, 1, p.W3, no, 1, a->O, no, 1));
  hipLaunchKernelGGL(k_bias_f, dim3(blocks(B * no)), dim3(256), 0, st, a->O, p.b3, B, no);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status ws_backward32(nys_ctx ctx, nys_ws_model m, const double* Tg, const double* Wt,
                         int64_t B, Act32* a, double* loss_dev) {
  hipStream_t st = ctx->stream;
  const bool bf = m->prec == NYS_BF16;
  const int ni = m->n_in, h = m->hidden, no = m->n_out;
  WsPtrs32 p = ws_ptrs32(m, m->params32.as<float>());
  WsPtrs32 g = ws_ptrs32(m, m->grads32.as<float>());
  const unsigned nb = blocks(B * no);
  hipLaunchKernelGGL(k_loss_grad_f, dim3(nb), dim3(256), 0, st, a->O, Tg, Wt, B * no, (int)B,
                     a->G, a->part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, a->part, (int)nb, loss_dev);
  // layer 3: gW3 = H2^T G, gb3 = 1^T G, gH2 = G W3^T
  NYS_TRY(mlp_gemm(st, bf, h, no, (int)B, a->H2, 1, h, a->G, no, 1, g.W3, no, 1));
  hipLaunchKernelGGL(k_colsum_f, dim3(blocks(no)), dim3(256), 0, st, a->G, B, no, g.b3);
  NYS_TRY(mlp_gemm(st, bf, (int)B, h, no, a->G, no, 1, p.W3, 1, no, a->gH, h, 1));
  hipLaunchKernelGGL(k_gelu_back_f, dim3(blocks(B * h)), dim3(256), 0, st, a->gH, a->A2, B * h,
                     a->gA);
  // layer 2
  NYS_TRY(mlp_gemm(st, bf, h, h, (int)B, a->H1, 1, h, a->gA, h, 1, g.W2, h, 1));
  hipLaunchKernelGGL(k_colsum_f, dim3(blocks(h)), dim3(256), 0, st, a->gA, B, h, g.b2);
  NYS_TRY(mlp_gemm(st, bf, (int)B, h, h, a->gA, h, 1, p.W2, 1, h, a->gH, h, 1));
  hipLaunchKernelGGL(k_gelu_back_f, dim3(blocks(B * h)), dim3(256), 0, st, a->gH, a->A1, B * h,
                     a->gA);
  // layer 1
  NYS_TRY(mlp_gemm(st, bf, ni, h, (int)B, a->Xn, 1, ni, a->gA, h, 1, g.W1, h, 1));
  hipLaunchKernelGGL(k_colsum_f, dim3(blocks(h)), dim3(256), 0, st, a->gA, B, h, g.b1);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

// x0 = U c with c = s_out * MLP((f - mu)/sigma) [+ (Lambda + rho I)^-1 U^T rhs],
// f = [U^T rhs, log gamma, log rho].
// scratch: >= 2 r + 2 + n_out doubles (device).
nys_status ws_propose(nys_ctx ctx, nys_ws_model m, nys_factor F, const double* rhs, double gamma,
                      double rho, double* x0, double* scratch, double* feat_out) {
  hipStream_t st = ctx->stream;
  const int r = F->r;
  if (m->n_in != r + 2 || m->n_out != r) return NYS_ERR_INVALID;
  double* cU = scratch;                  // U^T rhs (r)
  double* f = scratch + r;               // features (r + 2)
  double* c = f + r + 2;                 // coefficients (r)
  const double* U = F->U.as<double>();
  NYS_TRY(launch_ut_v(U, F->d, r, rhs, cU, st));
  hipLaunchKernelGGL(k_features, dim3(blocks(r + 2)), dim3(256), 0, st, cU, r, std::log(gamma),
                     std::log(rho), f);
  if (feat_out != nullptr)
    NYS_TRY_HIP(hipMemcpyAsync(feat_out, f, sizeof(double) * (r + 2), hipMemcpyDeviceToDevice, st));
  if (m->prec != NYS_F64) {
    Act32 a;
    NYS_TRY(ws_act32(m, 1, &a));
    NYS_TRY(ws_forward32(ctx, m, f, 1, &a));
    WsPtrs32 p = ws_ptrs32(m, m->params32.as<float>());
    hipLaunchKernelGGL(k_scale_f, dim3(blocks(r)), dim3(256), 0, st, a.O, p.sout, r,
                       m->skip ? cU : nullptr, F->lam.as<double>(), rho, c);
  } else {
    Act a;
    NYS_TRY(ws_act(m, 1, &a));
    NYS_TRY(ws_forward(ctx, m, f, 1, &a));
    WsPtrs p = ws_ptrs(m, m->params.as<double>());
    hipLaunchKernelGGL(k_scale, dim3(blocks(r)), dim3(256), 0, st, a.O, p.sout, r,
                       m->skip ? cU : nullptr, F->lam.as<double>(), rho, c);
  }
  NYS_TRY(launch_u_c(U, F->d, r, c, x0, st));
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

// x0 = U (Lambda + rho I)^-1 U^T rhs: the exact solve restricted to the span of
// U (with exact eigenvectors, the coefficient map the network is asked to learn).
// scratch: >= 2 r doubles (device).
nys_status ws_analytic(nys_ctx ctx, nys_factor F, const double* rhs, double rho, double* x0,
                       double* scratch) {
  hipStream_t st = ctx->stream;
  const int r = F->r;
  const double* U = F->U.as<double>();
  NYS_TRY(launch_ut_v(U, F->d, r, rhs, scratch, st));
  hipLaunchKernelGGL(k_shift_div, dim3(blocks(r)), dim3(256), 0, st, scratch, F->lam.as<double>(),
                     r, rho, scratch + r);
  NYS_TRY(launch_u_c(U, F->d, r, scratch + r, x0, st));
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

// features only (for recording training data) and the target U^T x
nys_status ws_record(nys_ctx ctx, nys_factor F, const double* rhs, double gamma, double rho,
                     const double* x, double* feat_out, double* target_out, double* scratch) {
  hipStream_t st = ctx->stream;
  const int r = F->r;
  const double* U = F->U.as<double>();
  if (feat_out != nullptr) {
    NYS_TRY(launch_ut_v(U, F->d, r, rhs, scratch, st));
    hipLaunchKernelGGL(k_features, dim3(blocks(r + 2)), dim3(256), 0, st, scratch, r,
                       std::log(gamma), std::log(rho), feat_out);
  }
  if (target_out != nullptr) NYS_TRY(launch_ut_v(U, F->d, r, x, target_out, st));
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

}  // namespace nys

using namespace nys;

extern "C" {

size_t nys_ws_param_count(int n_in, int hidden, int n_out) {
  if (n_in < 1 || hidden < 1 || n_out < 1) return 0;
  return ws_count(n_in, hidden, n_out);
}

nys_status nys_ws_create(nys_ctx ctx, int n_in, int hidden, int n_out, const double* params_host,
                         const double* in_mean, const double* in_std, const double* out_scale,
                         int analytic_skip, nys_ws_model* out) {
  if (ctx == nullptr || out == nullptr || params_host == nullptr) return NYS_ERR_INVALID;
  if (n_in < 1 || hidden < 1 || n_out < 1 || hidden > 4096) return NYS_ERR_INVALID;
  if (analytic_skip != 0 && n_in != n_out + 2) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  nys_ws_model m = new (std::nothrow) nys_ws_model_s();
  if (m == nullptr) return NYS_ERR_NOMEM;
  m->n_in = n_in;
  m->hidden = hidden;
  m->n_out = n_out;
  m->device = ctx->device;
  m->skip = analytic_skip != 0;
  const size_t np = ws_count(n_in, hidden, n_out);
  const size_t tot = np + 2 * (size_t)n_in + n_out;
  std::vector<double> h(tot);
  std::memcpy(h.data(), params_host, sizeof(double) * np);
  for (int i = 0; i < n_in; ++i) {
    h[np + i] = in_mean ? in_mean[i] : 0.0;
    h[np + n_in + i] = in_std ? in_std[i] : 1.0;
    if (!(h[np + n_in + i] > 0.0)) {
      delete m;
      return NYS_ERR_INVALID;
    }
  }
  for (int i = 0; i < n_out; ++i) h[np + 2 * n_in + i] = out_scale ? out_scale[i] : 1.0;
  nys_status s = m->params.reserve(sizeof(double) * tot);
  if (s == NYS_OK) s = m->grads.reserve(sizeof(double) * tot);
  if (s == NYS_OK) s = m->adam.reserve(sizeof(double) * 2 * np);
  if (s != NYS_OK) {
    nys_ws_destroy(m);
    return s;
  }
  if (hipMemcpyAsync(m->params.ptr, h.data(), sizeof(double) * tot, hipMemcpyHostToDevice,
                     ctx->stream) != hipSuccess ||
      hipMemsetAsync(m->adam.ptr, 0, sizeof(double) * 2 * np, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    nys_ws_destroy(m);
    return NYS_ERR_HIP;
  }
  *out = m;
  return NYS_OK;
}

nys_status nys_ws_set_precision(nys_ctx ctx, nys_ws_model m, nys_dtype prec) {
  if (ctx == nullptr || m == nullptr) return NYS_ERR_INVALID;
  if (prec != NYS_F64 && prec != NYS_F32 && prec != NYS_BF16) return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  hipStream_t st = ctx->stream;
  const int64_t np = (int64_t)ws_count(m->n_in, m->hidden, m->n_out);
  const int64_t tot = np + 2 * (int64_t)m->n_in + m->n_out;
  const bool was32 = m->prec != NYS_F64, now32 = prec != NYS_F64;
  if (now32 && !was32) {
    // FP32 master copy of the FP64 parameters (and statistics); fresh Adam state
    NYS_TRY(m->params32.reserve(sizeof(float) * tot));
    NYS_TRY(m->grads32.reserve(sizeof(float) * tot));
    NYS_TRY(m->adam32.reserve(sizeof(float) * 2 * np));
    hipLaunchKernelGGL(k_f64_to_f32, dim3(blocks(tot)), dim3(256), 0, st, m->params.as<double>(),
                       tot, m->params32.as<float>());
    NYS_TRY_HIP(hipMemsetAsync(m->adam32.ptr, 0, sizeof(float) * 2 * np, st));
    m->t32 = 0;
  } else if (was32 && !now32) {
    // back to FP64: the FP32 master weights become the parameters
    hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks(tot)), dim3(256), 0, st, m->params32.as<float>(),
                       tot, m->params.as<double>());
    NYS_TRY_HIP(hipMemsetAsync(m->adam.ptr, 0, sizeof(double) * 2 * np, st));
    m->t = 0;
  }
  NYS_TRY_HIP(hipGetLastError());
  NYS_TRY_HIP(hipStreamSynchronize(st));
  m->prec = prec;
  return NYS_OK;
}

nys_status nys_ws_get_params(nys_ctx ctx, nys_ws_model m, double* params_host) {
  if (ctx == nullptr || m == nullptr || params_host == nullptr) return NYS_ERR_INVALID;
  if (m->prec != NYS_F64) {
    // the FP32 master weights, widened
    NYS_TRY_HIP(hipSetDevice(ctx->device));
    const int64_t np = (int64_t)ws_count(m->n_in, m->hidden, m->n_out);
    hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks(np)), dim3(256), 0, ctx->stream,
                       m->params32.as<float>(), np, m->grads.as<double>());
    NYS_TRY_HIP(hipMemcpyAsync(params_host, m->grads.ptr, sizeof(double) * np,
                               hipMemcpyDeviceToHost, ctx->stream));
    NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
    return NYS_OK;
  }
  NYS_TRY_HIP(hipMemcpyAsync(params_host, m->params.ptr,
                             sizeof(double) * ws_count(m->n_in, m->hidden, m->n_out),
                             hipMemcpyDeviceToHost, ctx->stream));
  NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
  return NYS_OK;
}

nys_status nys_ws_forward(nys_ctx ctx, nys_ws_model m, const double* X, int batch, double* out) {
  if (ctx == nullptr || m == nullptr || X == nullptr || out == nullptr || batch < 1)
    return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  if (m->prec != NYS_F64) {
    Act32 a;
    NYS_TRY(ws_act32(m, batch, &a));
    NYS_TRY(ws_forward32(ctx, m, X, batch, &a));
    const int64_t no = (int64_t)batch * m->n_out;
    hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks(no)), dim3(256), 0, ctx->stream, a.O, no, out);
    return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
  }
  Act a;
  NYS_TRY(ws_act(m, batch, &a));
  NYS_TRY(ws_forward(ctx, m, X, batch, &a));
  NYS_TRY_HIP(hipMemcpyAsync(out, a.O, sizeof(double) * batch * m->n_out, hipMemcpyDeviceToDevice,
                             ctx->stream));
  return NYS_OK;
}

nys_status nys_ws_loss_grad(nys_ctx ctx, nys_ws_model m, const double* X, const double* T,
                            const double* W, int batch, double* loss_host, double* grad_out) {
  if (ctx == nullptr || m == nullptr || X == nullptr || T == nullptr || batch < 1)
    return NYS_ERR_INVALID;
  NYS_TRY_HIP(hipSetDevice(ctx->device));
  nys::CtxScope ctx_scope(ctx);
  const int64_t np = (int64_t)ws_count(m->n_in, m->hidden, m->n_out);
  double* loss_dev = nullptr;
  if (m->prec != NYS_F64) {
    Act32 a;
    NYS_TRY(ws_act32(m, batch, &a));
    NYS_TRY(ws_forward32(ctx, m, X, batch, &a));
    loss_dev = a.part + blocks((int64_t)batch * std::max(m->n_out, m->hidden)) + 1;
    NYS_TRY(ws_backward32(ctx, m, T, W, batch, &a, loss_dev));
    if (grad_out != nullptr)
      hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks(np)), dim3(256), 0, ctx->stream,
                         m->grads32.as<float>(), np, grad_out);
  } else {
    Act a;
    NYS_TRY(ws_act(m, batch, &a));
    NYS_TRY(ws_forward(ctx, m, X, batch, &a));
    loss_dev = a.part + blocks((int64_t)batch * std::max(m->n_out, m->hidden)) + 1;
    NYS_TRY(ws_backward(ctx, m, T, W, batch, &a, loss_dev));
    if (grad_out != nullptr)
      NYS_TRY_HIP(hipMemcpyAsync(grad_out, m->grads.ptr, sizeof(double) * np,
                                 hipMemcpyDeviceToDevice, ctx->stream));
  }
  if (loss_host != nullptr) {
    NYS_TRY_HIP(hipMemcpyAsync(ctx->host_pinned, loss_dev, sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    NYS_TRY_HIP(hipStreamSynchronize(ctx->stream));
    std::memcpy(loss_host, ctx->host_pinned, sizeof(double));
  }
  return NYS_OK;
}

nys_status nys_ws_train_step(nys_ctx ctx, nys_ws_model m, const double* X, const double* T,
                             const double* W, int batch, double lr, double* loss_host) {
  if (!(lr > 0.0)) return NYS_ERR_INVALID;
  NYS_TRY(nys_ws_loss_grad(ctx, m, X, T, W, batch, loss_host, nullptr));
  const int64_t np = (int64_t)ws_count(m->n_in, m->hidden, m->n_out);
  if (m->prec != NYS_F64) {
    m->t32 += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)m->t32));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)m->t32));
    float* mm = m->adam32.as<float>();
    hipLaunchKernelGGL(k_adam_f, dim3(blocks(np)), dim3(256), 0, ctx->stream,
                       m->params32.as<float>(), m->grads32.as<float>(), mm, mm + np, np, (float)lr,
                       b1, b2, 1e-8f, c1, c2);
    return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
  }
  m->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 - std::pow(b1, (double)m->t), c2 = 1.0 - std::pow(b2, (double)m->t);
  double* mm = m->adam.as<double>();
  hipLaunchKernelGGL(k_adam, dim3(blocks(np)), dim3(256), 0, ctx->stream, m->params.as<double>(),
                     m->grads.as<double>(), mm, mm + np, np, lr, b1, b2, 1e-8, c1, c2);
  return hipGetLastError() == hipSuccess ? NYS_OK : NYS_ERR_HIP;
}

nys_status nys_ws_destroy(nys_ws_model m) {
  if (m == nullptr) return NYS_ERR_INVALID;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  m->params.release();
  m->adam.release();
  m->grads.release();
  m->act.release();
  m->params32.release();
  m->adam32.release();
  m->grads32.release();
  m->act32.release();
  delete m;
  return NYS_OK;
}

}  // extern "C"
