// Moment-extrapolation MLP: n_in -> n_hid -> n_hid -> n_out with exact GELU,
// trained and evaluated on the GPU by the kernels below.  It maps the first
// n_in Chebyshev moments of a DOS to the next n_out moments, so that fewer
// recursion steps are needed; the full recursion remains the reference and
// the fallback.  (The paper has no learned component.)
//
// Kernels: one tiled MFMA GEMM (64 x 64 output tile per 256-thread workgroup,
// four 32 x 32 wave tiles) with optional transposed operands and a fused
// bias / bias+GELU epilogue, in FP32 (v_mfma_f32_32x32x2_f32, training) or
// BF16 operands with FP32 accumulation (v_mfma_f32_32x32x16_bf16, inference);
// weighted-MSE loss and its gradient; GELU backward; bias gradients;
// Adam.  Every reduction runs in a fixed order (bitwise reproducible).

#include "kpm_internal.h"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace kpm {

typedef float f32x16m __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8m __attribute__((ext_vector_type(8)));

constexpr int kT = 64;    // output tile
constexpr int kBK = 32;   // k per LDS stage

enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2 };

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

// C[M][N] = op(A) op(B) (+ bias), op(A) = A [M][K] (TA = false) or A^T with A
// stored [K][M]; op(B) = B [K][N] (TB = false) or B^T with B stored [N][K].
// EPI_BIAS_GELU stores the pre-activation in Z and gelu(.) in C.
template <bool TA, bool TB, bool BF16, int EPI>
__global__ void __launch_bounds__(256) mlp_gemm(const float* __restrict__ A, int lda, const float* __restrict__ B,
                                                int ldb, float* __restrict__ C, int ldc, float* __restrict__ Z,
                                                const float* __restrict__ bias, int M, int N, int K) {
  __shared__ float As[kBK][kT + 1];
  __shared__ float Bs[kBK][kT + 1];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wi = wave & 1, wj = wave >> 1;
  const int m0 = blockIdx.y * kT, n0 = blockIdx.x * kT;
  f32x16m acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  for (int k0 = 0; k0 < K; k0 += kBK) {
    // Stage op(A)[m0 .. m0+63][k0 .. k0+31] as As[k][i], op(B) as Bs[k][j].
    for (int q = tid; q < kT * kBK; q += 256) {
      int i, k;
      if (TA) { i = q % kT; k = q / kT; } else { k = q % kBK; i = q / kBK; }
      const int gi = m0 + i, gk = k0 + k;
      float a = 0.f;
      if (gi < M && gk < K) a = TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
      As[k][i] = a;
      int j, kb;
      if (TB) { kb = q % kBK; j = q / kBK; } else { j = q % kT; kb = q / kT; }
      const int gj = n0 + j, gkb = k0 + kb;
      float b = 0.f;
      if (gj < N && gkb < K) b = TB ? B[(int64_t)gj * ldb + gkb] : B[(int64_t)gkb * ldb + gj];
      Bs[kb][j] = b;
    }
    __syncthreads();
    const int r = lane & 31, g = lane >> 5;
    if constexpr (BF16) {
#pragma unroll
      for (int ks = 0; ks < kBK; ks += 16) {
        bf16x8m a8, b8;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          a8[e] = (__bf16)As[ks + 8 * g + e][32 * wi + r];
          b8[e] = (__bf16)Bs[ks + 8 * g + e][32 * wj + r];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b8, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < kBK; ks += 2)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[ks + g][32 * wi + r], Bs[ks + g][32 * wj + r], acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int r = lane & 31, g = lane >> 5;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int i = m0 + 32 * wi + 8 * (e >> 2) + 4 * g + (e & 3);
    const int j = n0 + 32 * wj + r;
    if (i < M && j < N) {
      float v = acc[e];
      if (EPI != EPI_NONE) v += bias[j];
      if (EPI == EPI_BIAS_GELU) {
        Z[(int64_t)i * ldc + j] = v;
        v = gelu_f(v);
      }
      C[(int64_t)i * ldc + j] = v;
    }
  }
}

// dY = 2 w_j^2 (Y - T) / (B n_out); per-block partial loss sums (FP64).
__global__ void mlp_loss_kernel(const float* Y, const float* T, const float* w, int Bn, int n_out, float* dY,
                                double* partial) {
  __shared__ double red[256];
  const int64_t n = (int64_t)Bn * n_out;
  const double inv = 1.0 / (double)n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % n_out);
    const float d = Y[i] - T[i];
    const float wj = w[j];
    dY[i] = (float)(2.0 * inv) * wj * wj * d;
    const double e = (double)wj * (double)d;
    acc += e * e;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] * inv;
}

// err[b] = sqrt(sum_j (w_j (Y_bj - R_bj))^2) / sqrt(sum_j (w_j R_bj)^2) over the
// first n_cmp of the n_out columns of Y, or with noise given,
// sqrt(sum_j (w_j (Y_bj - R_bj))^2) / (noise_b sqrt(sum_j w_j^2)); one
// workgroup per row, FP64 sums in a fixed-order tree.
__global__ void rel_error_kernel(const float* Y, int n_out, const double* R, int n_cmp, const float* w,
                                 const double* noise, double* err) {
  __shared__ double num[256], den[256];
  const int b = blockIdx.x;
  double a = 0.0, d = 0.0;
  for (int j = threadIdx.x; j < n_cmp; j += blockDim.x) {
    const double r = R[(int64_t)b * n_cmp + j], wj = w[j];
    const double e = wj * ((double)Y[(int64_t)b * n_out + j] - r);
    a += e * e;
    d += noise ? wj * wj : (wj * r) * (wj * r);
  }
  num[threadIdx.x] = a;
  den[threadIdx.x] = d;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      num[threadIdx.x] += num[threadIdx.x + st];
      den[threadIdx.x] += den[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) err[b] = sqrt(num[0]) / fmax((noise ? noise[b] : 1.0) * sqrt(den[0]), 1e-300);
}

__global__ void sum_partials_kernel(const double* partial, int n, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s;
  }
}

// dZ = dA * gelu'(Z)
__global__ void gelu_backward_kernel(const float* dA, const float* Z, float* dZ, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dZ[i] = dA[i] * gelu_grad_f(Z[i]);
}

// db[j] = sum_b dZ[b][j] (fixed order over b)
__global__ void bias_grad_kernel(const float* dZ, int Bn, int n, float* db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float s = 0.f;
  for (int b = 0; b < Bn; ++b) s += dZ[(int64_t)b * n + j];
  db[j] = s;
}

// Adam (Kingma & Ba 2015) with bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// He-uniform initialisation from the SplitMix64 stream (purpose 5): W ~ U(-s, s), s = sqrt(3/fan_in).
__global__ void init_uniform_kernel(float* p, int64_t n, uint64_t key, float scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = (float)((2.0 * sm_uniform(key, (uint64_t)i) - 1.0) * scale);
}

// Column statistics of a [n][cols] table (FP64, fixed order): shift = mean,
// scale = standard deviation (1 where it vanishes).
__global__ void column_stats_kernel(const float* X, int64_t n, int cols, float* shift, float* scale) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += X[i * cols + j];
  const double mean = s / (double)n;
  double v = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double d = X[i * cols + j] - mean;
    v += d * d;
  }
  const double sd = sqrt(v / (double)n);
  shift[j] = (float)mean;
  scale[j] = sd > 0.0 ? (float)sd : 1.0f;
}

// out = (in - shift) / scale  (forward = 1)  or  out = shift + scale * in (forward = 0), column-wise.
__global__ void affine_kernel(const float* in, float* out, int64_t rows, int cols, const float* shift,
                              const float* scale, int forward) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int j = (int)(i % cols);
  out[i] = forward ? (in[i] - shift[j]) / scale[j] : shift[j] + scale[j] * in[i];
}

// w' = w * scale (loss weights in normalised output units).
__global__ void mul_kernel(const float* a, const float* b, float* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

__global__ void fill_f32(float* p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace kpm

struct kpm_mlp {
  int n_in = 0, n_hid = 0, n_out = 0;
  int64_t off[6] = {0, 0, 0, 0, 0, 0};   // W1 b1 W2 b2 W3 b3 offsets (floats)
  int64_t n_par = 0;
  float* par = nullptr;
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  int64_t t = 0;
  int cap_b = 0;                          // workspace capacity (batch rows)
  float *Z1 = nullptr, *A1 = nullptr, *Z2 = nullptr, *A2 = nullptr, *Y = nullptr, *dY = nullptr;
  float *dA = nullptr, *dZ = nullptr;
  double* partial = nullptr;
  double* loss_dev = nullptr;
  // Optional per-column standardisation of inputs and outputs.
  bool scaled = false;
  float *x_shift = nullptr, *x_scale = nullptr, *y_shift = nullptr, *y_scale = nullptr;
  float *Xn = nullptr, *Tn = nullptr, *wn = nullptr;   // workspace: normalised batch, weights
};

namespace kpm {

static int mlp_reserve(kpm_mlp* N, int B) {
  if (B <= N->cap_b) return KPM_OK;
  // Drop the old workspace first: after a failed allocation the network holds
  // no workspace (cap_b = 0), and the next call allocates it again.
  N->cap_b = 0;
  float** bufs[] = {&N->Z1, &N->A1, &N->Z2, &N->A2, &N->Y, &N->dY, &N->dA, &N->dZ, &N->Xn, &N->Tn};
  for (float** b : bufs) {
    (void)::kpm::dev_free(*b);
    *b = nullptr;
  }
  const int64_t h = (int64_t)B * N->n_hid, o = (int64_t)B * N->n_out;
  const int64_t wmax = std::max<int64_t>(h, o);
  KPM_TRY_HIP(::kpm::dev_malloc(&N->Z1, h * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->A1, h * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->Z2, h * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->A2, h * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->Y, o * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->dY, o * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->dA, wmax * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->dZ, wmax * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->Xn, (int64_t)B * N->n_in * 4));
  KPM_TRY_HIP(::kpm::dev_malloc(&N->Tn, o * 4));
  N->cap_b = B;
  return KPM_OK;
}

template <bool TA, bool TB, bool BF16, int EPI>
static void gemm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, float* Z, const float* bias,
                 int M, int Nn, int K, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(Nn, kT), (unsigned)ceil_div(M, kT));
  hipLaunchKernelGGL((mlp_gemm<TA, TB, BF16, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, Z, bias, M, Nn,
                     K);
}

static void forward(kpm_mlp* N, const float* X, int B, bool bf16, float* Y, hipStream_t s) {
  const float* P = N->par;
  const int ni = N->n_in, nh = N->n_hid, no = N->n_out;
  if (bf16) {
    gemm<false, false, true, EPI_BIAS_GELU>(X, ni, P + N->off[0], nh, N->A1, nh, N->Z1, P + N->off[1], B, nh, ni, s);
    gemm<false, false, true, EPI_BIAS_GELU>(N->A1, nh, P + N->off[2], nh, N->A2, nh, N->Z2, P + N->off[3], B, nh, nh,
                                            s);
    gemm<false, false, true, EPI_BIAS>(N->A2, nh, P + N->off[4], no, Y, no, nullptr, P + N->off[5], B, no, nh, s);
  } else {
    gemm<false, false, false, EPI_BIAS_GELU>(X, ni, P + N->off[0], nh, N->A1, nh, N->Z1, P + N->off[1], B, nh, ni, s);
    gemm<false, false, false, EPI_BIAS_GELU>(N->A1, nh, P + N->off[2], nh, N->A2, nh, N->Z2, P + N->off[3], B, nh,
                                             nh, s);
    gemm<false, false, false, EPI_BIAS>(N->A2, nh, P + N->off[4], no, Y, no, nullptr, P + N->off[5], B, no, nh, s);
  }
}

// Forward + loss + backward into N->grad; loss (FP64) into N->loss_dev.
static void forward_backward(kpm_mlp* N, const float* X, const float* T, const float* w, int B, hipStream_t s) {
  const int ni = N->n_in, nh = N->n_hid, no = N->n_out;
  const float* P = N->par;
  float* G = N->grad;
  forward(N, X, B, false, N->Y, s);
  const int lb = 256;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(lb), dim3(256), 0, s, N->Y, T, w, B, no, N->dY, N->partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, N->partial, lb, N->loss_dev);
  // Layer 3: dW3 = A2^T dY, db3 = colsum dY, dA2 = dY W3^T.
  gemm<true, false, false, EPI_NONE>(N->A2, nh, N->dY, no, G + N->off[4], no, nullptr, nullptr, nh, no, B, s);
  hipLaunchKernelGGL(bias_grad_kernel, dim3((unsigned)ceil_div(no, 256)), dim3(256), 0, s, N->dY, B, no,
                     G + N->off[5]);
  gemm<false, true, false, EPI_NONE>(N->dY, no, P + N->off[4], no, N->dA, nh, nullptr, nullptr, B, nh, no, s);
  hipLaunchKernelGGL(gelu_backward_kernel, dim3((unsigned)ceil_div((int64_t)B * nh, 256)), dim3(256), 0, s, N->dA,
                     N->Z2, N->dZ, (int64_t)B * nh);
  // Layer 2.
  gemm<true, false, false, EPI_NONE>(N->A1, nh, N->dZ, nh, G + N->off[2], nh, nullptr, nullptr, nh, nh, B, s);
  hipLaunchKernelGGL(bias_grad_kernel, dim3((unsigned)ceil_div(nh, 256)), dim3(256), 0, s, N->dZ, B, nh,
                     G + N->off[3]);
  gemm<false, true, false, EPI_NONE>(N->dZ, nh, P + N->off[2], nh, N->dA, nh, nullptr, nullptr, B, nh, nh, s);
  hipLaunchKernelGGL(gelu_backward_kernel, dim3((unsigned)ceil_div((int64_t)B * nh, 256)), dim3(256), 0, s, N->dA,
                     N->Z1, N->dZ, (int64_t)B * nh);
  // Layer 1.
  gemm<true, false, false, EPI_NONE>(X, ni, N->dZ, nh, G + N->off[0], nh, nullptr, nullptr, ni, nh, B, s);
  hipLaunchKernelGGL(bias_grad_kernel, dim3((unsigned)ceil_div(nh, 256)), dim3(256), 0, s, N->dZ, B, nh,
                     G + N->off[1]);
}

// With standardisation the network sees x' = (x - mx)/sx and predicts
// y' = (y - my)/sy; the loss (w (y - t))^2 = (w sy (y' - t'))^2 is unchanged.
static void normalised_forward_backward(kpm_mlp* N, const float* X, const float* T, const float* w, int B,
                                        hipStream_t s) {
  if (!N->scaled) {
    forward_backward(N, X, T, w, B, s);
    return;
  }
  const int64_t nx = (int64_t)B * N->n_in, ny = (int64_t)B * N->n_out;
  hipLaunchKernelGGL(affine_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, s, X, N->Xn, (int64_t)B, N->n_in,
                     N->x_shift, N->x_scale, 1);
  hipLaunchKernelGGL(affine_kernel, dim3((unsigned)ceil_div(ny, 256)), dim3(256), 0, s, T, N->Tn, (int64_t)B, N->n_out,
                     N->y_shift, N->y_scale, 1);
  hipLaunchKernelGGL(mul_kernel, dim3((unsigned)ceil_div(N->n_out, 256)), dim3(256), 0, s, w, N->y_scale, N->wn,
                     N->n_out);
  forward_backward(N, N->Xn, N->Tn, N->wn, B, s);
}

}  // namespace kpm

extern "C" {

int kpm_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, uint64_t seed, kpm_mlp_t** out) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(out != nullptr, "NULL output");
  *out = nullptr;
  KPM_CHECK_ARG(n_in >= 1 && n_hidden >= 1 && n_out >= 1 && n_in <= 65536 && n_hidden <= 65536 && n_out <= 65536,
                "layer sizes must be in [1, 65536]");
  kpm_mlp* N = new (std::nothrow) kpm_mlp();
  if (!N) {
    set_error("kpm_mlp_create: out of host memory");
    return KPM_E_NOMEM;
  }
  N->n_in = n_in;
  N->n_hid = n_hidden;
  N->n_out = n_out;
  const int64_t sz[6] = {(int64_t)n_in * n_hidden, n_hidden, (int64_t)n_hidden * n_hidden, n_hidden,
                         (int64_t)n_hidden * n_out, n_out};
  int64_t o = 0;
  for (int i = 0; i < 6; ++i) {
    N->off[i] = o;
    o += (sz[i] + 63) / 64 * 64;
  }
  N->n_par = o;
  hipError_t e = ::kpm::dev_malloc(&N->par, o * 4);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&N->grad, o * 4);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&N->m, o * 4);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&N->v, o * 4);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&N->partial, 256 * sizeof(double));
  if (e == hipSuccess) e = ::kpm::dev_malloc(&N->loss_dev, sizeof(double));
  if (e == hipSuccess) {
    const unsigned gb = (unsigned)ceil_div(o, 256);
    hipLaunchKernelGGL(fill_f32, dim3(gb), dim3(256), 0, 0, N->par, o, 0.f);
    hipLaunchKernelGGL(fill_f32, dim3(gb), dim3(256), 0, 0, N->grad, o, 0.f);
    hipLaunchKernelGGL(fill_f32, dim3(gb), dim3(256), 0, 0, N->m, o, 0.f);
    hipLaunchKernelGGL(fill_f32, dim3(gb), dim3(256), 0, 0, N->v, o, 0.f);
    const int fan[3] = {n_in, n_hidden, n_hidden};
    for (int l = 0; l < 3; ++l) {
      const int64_t n = sz[2 * l];
      hipLaunchKernelGGL(init_uniform_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, 0, N->par + N->off[2 * l],
                         n, sm_key(5, seed, (uint64_t)l, 0), (float)std::sqrt(3.0 / fan[l]));
    }
    e = ::kpm::launch_status();
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    set_error("kpm_mlp_create: %s", hipGetErrorString(e));
    kpm_mlp_destroy(N);
    return e == hipErrorOutOfMemory ? KPM_E_NOMEM : KPM_E_DEVICE;
  }
  *out = N;
  return KPM_OK;
}

int kpm_mlp_destroy(kpm_mlp_t* N) {
  if (!N) return KPM_OK;
  void* bufs[] = {N->par, N->grad, N->m, N->v, N->Z1, N->A1, N->Z2, N->A2, N->Y, N->dY, N->dA, N->dZ, N->partial,
                  N->loss_dev, N->x_shift, N->x_scale, N->y_shift, N->y_scale, N->Xn, N->Tn, N->wn};
  for (void* b : bufs)
    if (b) (void)::kpm::dev_free(b);
  delete N;
  return KPM_OK;
}

int kpm_mlp_num_params(const kpm_mlp_t* N, int64_t* n) {
  using namespace kpm;
  KPM_CHECK_ARG(N && n, "NULL argument");
  *n = (int64_t)N->n_in * N->n_hid + N->n_hid + (int64_t)N->n_hid * N->n_hid + N->n_hid +
       (int64_t)N->n_hid * N->n_out + N->n_out;
  return KPM_OK;
}

// Parameters / gradients exchanged in packed order W1 [n_in][n_hid], b1, W2 [n_hid][n_hid], b2, W3 [n_hid][n_out], b3.
static int mlp_copy(kpm_mlp_t* N, float* dev_base, float* host, bool to_host) {
  using namespace kpm;
  const int64_t sz[6] = {(int64_t)N->n_in * N->n_hid, N->n_hid, (int64_t)N->n_hid * N->n_hid, N->n_hid,
                         (int64_t)N->n_hid * N->n_out, N->n_out};
  int64_t h = 0;
  for (int i = 0; i < 6; ++i) {
    if (to_host) KPM_TRY_HIP(hipMemcpy(host + h, dev_base + N->off[i], sz[i] * 4, hipMemcpyDeviceToHost));
    else KPM_TRY_HIP(hipMemcpy(dev_base + N->off[i], host + h, sz[i] * 4, hipMemcpyHostToDevice));
    h += sz[i];
  }
  return KPM_OK;
}

int kpm_mlp_get_params(kpm_mlp_t* N, float* params) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && params, "NULL argument");
  KPM_TRY_SYNC(hipDeviceSynchronize());
  return mlp_copy(N, N->par, params, true);
}

int kpm_mlp_set_params(kpm_mlp_t* N, const float* params) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && params, "NULL argument");
  KPM_TRY_SYNC(hipDeviceSynchronize());
  N->t = 0;
  const unsigned gb = (unsigned)ceil_div(N->n_par, 256);
  hipLaunchKernelGGL(fill_f32, dim3(gb), dim3(256), 0, 0, N->m, N->n_par, 0.f);
  hipLaunchKernelGGL(fill_f32, dim3(gb), dim3(256), 0, 0, N->v, N->n_par, 0.f);
  KPM_TRY_SYNC(hipDeviceSynchronize());
  return mlp_copy(N, N->par, const_cast<float*>(params), false);
}

int kpm_mlp_forward(kpm_mlp_t* N, const float* x, int32_t batch, float* y, int32_t use_bf16, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && x && y && batch >= 1, "bad arguments");
  KPM_TRY(mlp_reserve(N, batch));
  hipStream_t s = (hipStream_t)hip_stream;
  if (N->scaled) {
    const int64_t nx = (int64_t)batch * N->n_in, ny = (int64_t)batch * N->n_out;
    hipLaunchKernelGGL(affine_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, s, x, N->Xn, (int64_t)batch,
                       N->n_in, N->x_shift, N->x_scale, 1);
    forward(N, N->Xn, batch, use_bf16 != 0, y, s);
    hipLaunchKernelGGL(affine_kernel, dim3((unsigned)ceil_div(ny, 256)), dim3(256), 0, s, y, y, (int64_t)batch,
                       N->n_out, N->y_shift, N->y_scale, 0);
  } else {
    forward(N, x, batch, use_bf16 != 0, y, s);
  }
  KPM_TRY_HIP(hipGetLastError());
  return KPM_OK;
}

// The network's output in original units (the fitted standardisation applied
// around it) into N->Y.
static void forward_scaled(kpm_mlp* N, const float* x, int batch, bool bf16, hipStream_t s) {
  using namespace kpm;
  if (N->scaled) {
    const int64_t nx = (int64_t)batch * N->n_in, ny = (int64_t)batch * N->n_out;
    hipLaunchKernelGGL(affine_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, s, x, N->Xn, (int64_t)batch,
                       N->n_in, N->x_shift, N->x_scale, 1);
    forward(N, N->Xn, batch, bf16, N->Y, s);
    hipLaunchKernelGGL(affine_kernel, dim3((unsigned)ceil_div(ny, 256)), dim3(256), 0, s, N->Y, N->Y, (int64_t)batch,
                       N->n_out, N->y_shift, N->y_scale, 0);
  } else {
    forward(N, x, batch, bf16, N->Y, s);
  }
}

int kpm_mlp_rel_error(kpm_mlp_t* N, const float* x, const double* ref, const float* weights, int32_t batch,
                      int32_t n_cmp, int32_t use_bf16, double* err, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && x && ref && weights && err && batch >= 1, "bad arguments");
  KPM_CHECK_ARG(n_cmp >= 1 && n_cmp <= N->n_out, "n_cmp must be in [1, n_out]");
  KPM_TRY(mlp_reserve(N, batch));
  hipStream_t s = (hipStream_t)hip_stream;
  forward_scaled(N, x, batch, use_bf16 != 0, s);
  hipLaunchKernelGGL(rel_error_kernel, dim3(batch), dim3(256), 0, s, N->Y, N->n_out, ref, n_cmp, weights,
                     (const double*)nullptr, err);
  KPM_TRY_HIP(hipGetLastError());
  return KPM_OK;
}

int kpm_mlp_noise_z(kpm_mlp_t* N, const float* x, const double* ref, const double* noise, const float* weights,
                    int32_t batch, int32_t n_cmp, int32_t use_bf16, double* z, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && x && ref && noise && weights && z && batch >= 1, "bad arguments");
  KPM_CHECK_ARG(n_cmp >= 1 && n_cmp <= N->n_out, "n_cmp must be in [1, n_out]");
  KPM_TRY(mlp_reserve(N, batch));
  hipStream_t s = (hipStream_t)hip_stream;
  forward_scaled(N, x, batch, use_bf16 != 0, s);
  hipLaunchKernelGGL(rel_error_kernel, dim3(batch), dim3(256), 0, s, N->Y, N->n_out, ref, n_cmp, weights, noise, z);
  KPM_TRY_HIP(hipGetLastError());
  return KPM_OK;
}

int kpm_mlp_eval_loss(kpm_mlp_t* N, const float* x, const float* target, const float* weights, int32_t batch,
                      int32_t use_bf16, double* loss_dev_out, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && x && target && weights && loss_dev_out && batch >= 1, "bad arguments");
  KPM_TRY(mlp_reserve(N, batch));
  hipStream_t s = (hipStream_t)hip_stream;
  forward_scaled(N, x, batch, use_bf16 != 0, s);
  const int lb = 256;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(lb), dim3(256), 0, s, N->Y, target, weights, batch, N->n_out, N->dY,
                     N->partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, N->partial, lb, loss_dev_out);
  KPM_TRY_HIP(hipGetLastError());
  return KPM_OK;
}

int kpm_mlp_fit_scaling(kpm_mlp_t* N, const float* x, const float* target, int64_t n_rows, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && x && target && n_rows >= 1, "bad arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  // Each buffer on its own, so that a call after a failed allocation completes the set.
  if (!N->x_shift) KPM_TRY_HIP(::kpm::dev_malloc(&N->x_shift, N->n_in * 4));
  if (!N->x_scale) KPM_TRY_HIP(::kpm::dev_malloc(&N->x_scale, N->n_in * 4));
  if (!N->y_shift) KPM_TRY_HIP(::kpm::dev_malloc(&N->y_shift, N->n_out * 4));
  if (!N->y_scale) KPM_TRY_HIP(::kpm::dev_malloc(&N->y_scale, N->n_out * 4));
  if (!N->wn) KPM_TRY_HIP(::kpm::dev_malloc(&N->wn, N->n_out * 4));
  hipLaunchKernelGGL(column_stats_kernel, dim3((unsigned)ceil_div(N->n_in, 64)), dim3(64), 0, s, x, n_rows, N->n_in,
                     N->x_shift, N->x_scale);
  hipLaunchKernelGGL(column_stats_kernel, dim3((unsigned)ceil_div(N->n_out, 64)), dim3(64), 0, s, target, n_rows,
                     N->n_out, N->y_shift, N->y_scale);
  KPM_TRY_HIP(hipGetLastError());
  KPM_TRY_SYNC(hipStreamSynchronize(s));
  N->scaled = true;
  return KPM_OK;
}

int kpm_mlp_gradients(kpm_mlp_t* N, const float* x, const float* target, const float* weights, int32_t batch,
                      float* grads_host, double* loss, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && x && target && weights && batch >= 1, "bad arguments");
  KPM_TRY(mlp_reserve(N, batch));
  hipStream_t s = (hipStream_t)hip_stream;
  normalised_forward_backward(N, x, target, weights, batch, s);
  KPM_TRY_HIP(hipGetLastError());
  KPM_TRY_SYNC(hipStreamSynchronize(s));
  if (loss) KPM_TRY_HIP(hipMemcpy(loss, N->loss_dev, sizeof(double), hipMemcpyDeviceToHost));
  if (grads_host) KPM_TRY(mlp_copy(N, N->grad, grads_host, true));
  return KPM_OK;
}

int kpm_mlp_train_step(kpm_mlp_t* N, const float* x, const float* target, const float* weights, int32_t batch,
                       float lr, double* loss_dev_out, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(N && x && target && weights && batch >= 1, "bad arguments");
  KPM_CHECK_ARG(lr > 0.f && std::isfinite(lr), "lr must be > 0");
  KPM_TRY(mlp_reserve(N, batch));
  hipStream_t s = (hipStream_t)hip_stream;
  normalised_forward_backward(N, x, target, weights, batch, s);
  N->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)N->t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)N->t)));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)ceil_div(N->n_par, 256)), dim3(256), 0, s, N->par, N->grad, N->m,
                     N->v, N->n_par, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  if (loss_dev_out)
    KPM_TRY_HIP(hipMemcpyAsync(loss_dev_out, N->loss_dev, sizeof(double), hipMemcpyDeviceToDevice, s));
  KPM_TRY_HIP(hipGetLastError());
  return KPM_OK;
}

}  // extern "C"
