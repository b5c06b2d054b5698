// Gamma_nm accumulation as a GEMM over stored Chebyshev blocks (paper eq.
// Gammanm; storage and cost of Gamma in Sec. 2(b), "Numerical storage of Gamma").
//
// Blocks: L[n][k] and R[m][k] complex, n, m < M, k < K (orbitals x vectors),
// stored K-blocked: element (n, k) at complex index ((k / 16) Mp + n) 16 + k % 16
// (Mp >= M rows, a multiple of the 128-row tile, padding rows zero),
// so that one 16-element K block of 32 consecutive rows is 4 KiB contiguous.
// The kernels accumulate
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
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Workgroup tile: 128 (n) x 128 (m) complex; 4 waves in a 2 x 2 grid, each
// 64 x 64 complex (2 x 2 MFMA tiles of 32 x 32 for Re and for Im).
constexpr int kGTile = 128;
constexpr int kGWave = 64;

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

// grid = 8-multiple of (K splits x tiles); block = 256.  The blocks arrive
// already split into BF16 planes (hi, lo) in the K-blocked layout; Kq = reals
// per row (whole K blocks of 32 reals), kchunk = reals per split (multiple of 32).
// part[ks][n][m][2] (FP64) receives the chunk's result.
__global__ void __launch_bounds__(256) gamma_bf16_kernel(const __bf16* __restrict__ Lh, const __bf16* __restrict__ Ll,
                                                         const __bf16* __restrict__ Rh, const __bf16* __restrict__ Rl,
                                                         int M, int Mp, int64_t Kq, int64_t kchunk, int ntile,
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
  const int64_t block_stride = (int64_t)Mp * 32;   // reals between consecutive K blocks of one row

  // Each lane owns 16 consecutive reals of its row in every K block (offset
  // 16 kg); MFMA step s uses reals [8 s, 8 s + 8) of them.  A and B use the same
  // order of k, so the contraction is unchanged.  The blocks have Mp >= the
  // tiles' rows, padded with zeros, so no load needs a guard.
  int64_t aoff[2], boff[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    aoff[i] = (int64_t)(n_base + 32 * i + r32) * 32 + 16 * kg;
    boff[i] = (int64_t)(m_base + 32 * i + r32) * 32 + 16 * kg;
  }
  f32x16 re[2][2], im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) re[i][j][e] = im[i][j][e] = 0.f;

  // Two K blocks in flight: buffer 0 holds even blocks, buffer 1 odd ones; the
  // loop is unrolled by two so that every buffer index is a constant.
  bf16x8 ah0[2][2], al0[2][2], bh0[2][2], bl0[2][2];
  bf16x8 ah1[2][2], al1[2][2], bh1[2][2], bl1[2][2];
  auto load = [&](int64_t q0, bf16x8 (&ah)[2][2], bf16x8 (&al)[2][2], bf16x8 (&bh)[2][2], bf16x8 (&bl)[2][2]) {
    const int64_t kb = (q0 >> 5) * block_stride;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        ah[i][st] = *reinterpret_cast<const bf16x8*>(Lh + kb + aoff[i] + 8 * st);
        al[i][st] = *reinterpret_cast<const bf16x8*>(Ll + kb + aoff[i] + 8 * st);
        bh[i][st] = *reinterpret_cast<const bf16x8*>(Rh + kb + boff[i] + 8 * st);
        bl[i][st] = *reinterpret_cast<const bf16x8*>(Rl + kb + boff[i] + 8 * st);
      }
  };
  auto compute = [&](const bf16x8 (&ah)[2][2], const bf16x8 (&al)[2][2], const bf16x8 (&bh)[2][2],
                     const bf16x8 (&bl)[2][2]) {
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      bf16x8 b2hi[2], b2lo[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        b2hi[j] = swap_neg(bh[j][st]);
        b2lo[j] = swap_neg(bl[j][st]);
      }
      // The three split products are issued round-robin over the eight
      // accumulators, so consecutive MFMAs never depend on each other.
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i][st], bh[j][st], re[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i][st], b2hi[j], im[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i][st], bl[j][st], re[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i][st], b2lo[j], im[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i][st], bh[j][st], re[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i][st], b2hi[j], im[i][j], 0, 0, 0);
        }
    }
  };
  if (k_begin < k_end) load(k_begin, ah0, al0, bh0, bl0);
  if (k_begin + 32 < k_end) load(k_begin + 32, ah1, al1, bh1, bl1);
  for (int64_t q0 = k_begin; q0 < k_end; q0 += 64) {
    compute(ah0, al0, bh0, bl0);
    if (q0 + 64 < k_end) load(q0 + 64, ah0, al0, bh0, bl0);
    if (q0 + 32 < k_end) {
      compute(ah1, al1, bh1, bl1);
      if (q0 + 96 < k_end) load(q0 + 96, ah1, al1, bh1, bl1);
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
                                                         int Mp, int64_t Kc, int64_t kchunk, double* __restrict__ part) {
  __shared__ double ls[16][17][2], rs[16][17][2];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int n0 = blockIdx.y * 16, m0 = blockIdx.x * 16;
  const int64_t k_begin = (int64_t)blockIdx.z * kchunk;
  const int64_t k_end = min(Kc, k_begin + kchunk);
  double ar = 0.0, ai = 0.0;
  for (int64_t k0 = k_begin; k0 < k_end; k0 += 16) {
    // thread (ty, tx) stages L[n0+ty][k0+tx] and R[m0+ty][k0+tx]; k0 is a multiple
    // of 16, so k0 + tx lies in K block k0/16 at position tx.
    const int64_t kb = (k0 / 16) * (int64_t)Mp;
    const int n = n0 + ty, m = m0 + ty;
    const bool kin = k0 + tx < k_end;
    const int64_t li = 2 * ((kb + n) * 16 + tx), ri = 2 * ((kb + m) * 16 + tx);
    ls[ty][tx][0] = (kin && n < M) ? (double)L[li] : 0.0;
    ls[ty][tx][1] = (kin && n < M) ? (double)L[li + 1] : 0.0;
    rs[ty][tx][0] = (kin && m < M) ? (double)R[ri] : 0.0;
    rs[ty][tx][1] = (kin && m < M) ? (double)R[ri + 1] : 0.0;
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

// Split-BF16 accumulation over K-blocked BF16 planes (hi, lo) of Kc complex
// values per row (a multiple of 16); part holds KS * M * M * 2 doubles.
hipError_t gamma_accumulate_bf16(const __bf16* Lh, const __bf16* Ll, const __bf16* Rh, const __bf16* Rl, int M,
                                 int Mp, int64_t Kc, int KS, double* part, double* acc, hipStream_t s) {
  const int64_t Kq = 2 * Kc;
  const int ntile = (int)ceil_div(M, kGTile);
  const int64_t kchunk = ceil_div(ceil_div(Kq, KS), 32) * 32;
  const int ks_used = (int)ceil_div(Kq, kchunk);
  const int n_logical = ks_used * ntile * ntile;
  const int grid = (int)ceil_div(n_logical, 8) * 8;
  hipLaunchKernelGGL(gamma_bf16_kernel, dim3(grid), dim3(256), 0, s, Lh, Ll, Rh, Rl, M, Mp, Kq, kchunk, ntile,
                     n_logical, part);
  const int64_t n = (int64_t)M * M * 2;
  hipLaunchKernelGGL(gamma_reduce_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, part, ks_used, n, acc);
  return hipGetLastError();
}

template <typename T>
hipError_t gamma_accumulate_fp64(const T* L, const T* R, int M, int Mp, int64_t Kc, int KS, double* part,
                                 double* acc, hipStream_t s) {
  const int64_t kchunk = ceil_div(ceil_div(Kc, KS), 16) * 16;
  const int ks_used = (int)ceil_div(Kc, kchunk);
  dim3 grid((unsigned)ceil_div(M, 16), (unsigned)ceil_div(M, 16), (unsigned)ks_used);
  hipLaunchKernelGGL(gamma_fp64_kernel<T>, grid, dim3(256), 0, s, L, R, M, Mp, Kc, kchunk, part);
  const int64_t n = (int64_t)M * M * 2;
  hipLaunchKernelGGL(gamma_reduce_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, part, ks_used, n, acc);
  return hipGetLastError();
}

template hipError_t gamma_accumulate_fp64<float>(const float*, const float*, int, int, int64_t, int, double*,
                                                 double*, hipStream_t);
template hipError_t gamma_accumulate_fp64<double>(const double*, const double*, int, int, int64_t, int, double*,
                                                  double*, hipStream_t);

}  // namespace kpm
