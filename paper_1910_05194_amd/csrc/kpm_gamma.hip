// Gamma_nm accumulation as a GEMM over stored Chebyshev blocks (paper eq.
// Gammanm; storage and cost of Gamma in Sec. 2(b), "Numerical storage of Gamma").
//
// Blocks: L[n][k] and R[m][k] complex, n, m < M, k < K (orbitals x vectors),
// rows of ld T-elements.  The kernels accumulate
//      G[n][m] += sum_k conj(L[n][k]) R[m][k]
// into an FP64 [M][M][2] array.  Written over interleaved (re, im) reals q:
//      Re G = sum_q Lq Rq,   Im G = sum_q Lq R'q,   R'(2k) = Im R(k), R'(2k+1) = -Re R(k),
// i.e. two real GEMMs with a shared left operand.
//
// Split-BF16 mode: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); a product
// is taken as hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo_a lo_b term, ~2^-16
// relative, is dropped) on v_mfma_f32_32x32x16_bf16 with FP32 accumulation
// inside one K chunk of a workgroup; chunks are combined in FP64 by a
// fixed-order reduction (bitwise reproducible).

#include "kpm_internal.h"

namespace kpm {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Workgroup tile: 128 (n) x 128 (m) complex; 4 waves in a 2 x 2 grid, each
// 64 x 64 complex (2 x 2 MFMA tiles of 32 x 32 for Re and for Im).
constexpr int kGTile = 128;
constexpr int kGWave = 64;

__device__ inline void split8(const f32x4& x0, const f32x4& x1, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 h0 = (__bf16)x0[e];
    const __bf16 h1 = (__bf16)x1[e];
    hi[e] = h0;
    hi[4 + e] = h1;
    lo[e] = (__bf16)(x0[e] - (float)h0);
    lo[4 + e] = (__bf16)(x1[e] - (float)h1);
  }
}

// (x0, x1, x2, ...) -> (x1, -x0, x3, -x2, ...): the imaginary-part operand.
__device__ inline bf16x8 swap_neg(const bf16x8& b) {
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    r[e] = b[e + 1];
    r[e + 1] = -b[e];
  }
  return r;
}

// grid = 8-multiple of (K splits x tiles); block = 256.
// part[ks][n][m][2] (FP64) receives the chunk's result.
__global__ void __launch_bounds__(256) gamma_bf16_kernel(const float* __restrict__ L, const float* __restrict__ R,
                                                         int M, int64_t Kq, int64_t ld, int64_t kchunk, int ntile,
                                                         int n_logical, double* __restrict__ part) {
  // XCD-aware: the workgroups of XCD x take a contiguous range of logical ids,
  // so that the tiles sharing a K chunk run on one L2.
  const int G = gridDim.x;
  const int xcd = blockIdx.x & 7, jx = blockIdx.x >> 3, per = G >> 3;
  const int logical = xcd * per + jx;
  if (logical >= n_logical) return;
  const int tiles = ntile * ntile;
  const int tile = logical % tiles;
  const int ks = logical / tiles;
  const int tn = tile % ntile, tm = tile / ntile;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wn = wave & 1, wm = wave >> 1;
  const int n_base = tn * kGTile + wn * kGWave;
  const int m_base = tm * kGTile + wm * kGWave;
  const int64_t k_begin = (int64_t)ks * kchunk;
  const int64_t k_end = min(Kq, k_begin + kchunk);
  const int r32 = lane & 31, kg = lane >> 5;

  const float* arow[2];
  const float* brow[2];
  bool aval[2], bval[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int n = n_base + 32 * i + r32;
    aval[i] = n < M;
    arow[i] = L + (int64_t)(aval[i] ? n : 0) * ld;
    const int m = m_base + 32 * i + r32;
    bval[i] = m < M;
    brow[i] = R + (int64_t)(bval[i] ? m : 0) * ld;
  }
  f32x16 re[2][2], im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) re[i][j][e] = im[i][j][e] = 0.f;

  for (int64_t q0 = k_begin; q0 < k_end; q0 += 32) {
    // Each lane holds 16 consecutive reals of its row: q0 + 16 kg + [0, 16).
    // Both operands use the same k order, so the contraction is unchanged.
    const int64_t qq = q0 + 16 * kg;
    f32x4 av[2][4], bv[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t q = qq + 4 * c;
        const bool inb = q + 4 <= k_end;
        av[i][c] = (aval[i] && inb) ? *reinterpret_cast<const f32x4*>(arow[i] + q) : f32x4{0.f, 0.f, 0.f, 0.f};
        bv[i][c] = (bval[i] && inb) ? *reinterpret_cast<const f32x4*>(brow[i] + q) : f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 ahi[2], alo[2], bhi[2], blo[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        split8(av[i][2 * s], av[i][2 * s + 1], ahi[i], alo[i]);
        split8(bv[i][2 * s], bv[i][2 * s + 1], bhi[i], blo[i]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bf16x8 b2hi = swap_neg(bhi[j]), b2lo = swap_neg(blo[j]);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[i], bhi[j], re[i][j], 0, 0, 0);
          re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[i], blo[j], re[i][j], 0, 0, 0);
          re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[i], bhi[j], re[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[i], b2hi, im[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[i], b2lo, im[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[i], b2hi, im[i][j], 0, 0, 0);
        }
      }
    }
  }
  // Accumulator layout of a 32x32 MFMA tile: lane l, element e holds
  // row 8 (e/4) + 4 (l/32) + e%4, column l%32.
  double* pb = part + (int64_t)ks * M * M * 2;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int n = n_base + 32 * i + 8 * (e >> 2) + 4 * kg + (e & 3);
        const int m = m_base + 32 * j + r32;
        if (n < M && m < M) {
          pb[((int64_t)n * M + m) * 2] = (double)re[i][j][e];
          pb[((int64_t)n * M + m) * 2 + 1] = (double)im[i][j][e];
        }
      }
}

// FP64 reference GEMM (exact mode): 16 x 16 output tile per workgroup, k tiles
// of 16 complex values staged in LDS; grid.z splits K.
template <typename T>
__global__ void __launch_bounds__(256) gamma_fp64_kernel(const T* __restrict__ L, const T* __restrict__ R, int M,
                                                         int64_t Kc, int64_t ld, int64_t kchunk,
                                                         double* __restrict__ part) {
  __shared__ double ls[16][17][2], rs[16][17][2];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int n0 = blockIdx.y * 16, m0 = blockIdx.x * 16;
  const int64_t k_begin = (int64_t)blockIdx.z * kchunk;
  const int64_t k_end = min(Kc, k_begin + kchunk);
  double ar = 0.0, ai = 0.0;
  for (int64_t k0 = k_begin; k0 < k_end; k0 += 16) {
    // thread (ty, tx) stages L[n0+ty][k0+tx] and R[m0+ty][k0+tx]
    const int64_t k = k0 + tx;
    const int n = n0 + ty, m = m0 + ty;
    const bool kin = k < k_end;
    ls[ty][tx][0] = (kin && n < M) ? (double)L[(int64_t)n * ld + 2 * k] : 0.0;
    ls[ty][tx][1] = (kin && n < M) ? (double)L[(int64_t)n * ld + 2 * k + 1] : 0.0;
    rs[ty][tx][0] = (kin && m < M) ? (double)R[(int64_t)m * ld + 2 * k] : 0.0;
    rs[ty][tx][1] = (kin && m < M) ? (double)R[(int64_t)m * ld + 2 * k + 1] : 0.0;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double lr = ls[ty][kk][0], li = ls[ty][kk][1];
      const double rr = rs[tx][kk][0], ri = rs[tx][kk][1];
      ar += lr * rr + li * ri;
      ai += lr * ri - li * rr;
    }
    __syncthreads();
  }
  const int n = n0 + ty, m = m0 + tx;
  if (n < M && m < M) {
    double* pb = part + (int64_t)blockIdx.z * M * M * 2;
    pb[((int64_t)n * M + m) * 2] = ar;
    pb[((int64_t)n * M + m) * 2 + 1] = ai;
  }
}

// acc[i] += sum_ks part[ks][i] in order (i over M*M*2 reals).
__global__ void gamma_reduce_kernel(const double* __restrict__ part, int KS, int64_t n, double* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < KS; ++k) s += part[(int64_t)k * n + i];
  acc[i] += s;
}

// Split-BF16 accumulation.  Kq = number of reals per row to contract (a
// multiple of 4), ld = row stride in floats; part holds KS * M * M * 2 doubles.
hipError_t gamma_accumulate_bf16(const float* L, const float* R, int M, int64_t Kq, int64_t ld, int KS,
                                 double* part, double* acc, hipStream_t s) {
  const int ntile = (int)ceil_div(M, kGTile);
  int64_t kchunk = ceil_div(ceil_div(Kq, KS), 32) * 32;
  const int ks_used = (int)ceil_div(Kq, kchunk);
  const int n_logical = ks_used * ntile * ntile;
  const int grid = (int)ceil_div(n_logical, 8) * 8;
  hipLaunchKernelGGL(gamma_bf16_kernel, dim3(grid), dim3(256), 0, s, L, R, M, Kq, ld, kchunk, ntile, n_logical,
                     part);
  const int64_t n = (int64_t)M * M * 2;
  hipLaunchKernelGGL(gamma_reduce_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, part, ks_used, n, acc);
  return hipGetLastError();
}

template <typename T>
hipError_t gamma_accumulate_fp64(const T* L, const T* R, int M, int64_t Kc, int64_t ld, int KS, double* part,
                                 double* acc, hipStream_t s) {
  const int64_t kchunk = ceil_div(ceil_div(Kc, KS), 16) * 16;
  const int ks_used = (int)ceil_div(Kc, kchunk);
  dim3 grid((unsigned)ceil_div(M, 16), (unsigned)ceil_div(M, 16), (unsigned)ks_used);
  hipLaunchKernelGGL(gamma_fp64_kernel<T>, grid, dim3(256), 0, s, L, R, M, Kc, ld, kchunk, part);
  const int64_t n = (int64_t)M * M * 2;
  hipLaunchKernelGGL(gamma_reduce_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, part, ks_used, n, acc);
  return hipGetLastError();
}

template hipError_t gamma_accumulate_fp64<float>(const float*, const float*, int, int64_t, int64_t, int, double*,
                                                 double*, hipStream_t);
template hipError_t gamma_accumulate_fp64<double>(const double*, const double*, int, int64_t, int64_t, int,
                                                  double*, double*, hipStream_t);

}  // namespace kpm
