// Gamma_nm accumulation as a GEMM over stored Chebyshev blocks (paper eq.
// Gammanm; storage and cost of Gamma in Sec. 2(b), "Numerical storage of Gamma").
//
// Blocks: L[n][k] and R[m][k] complex, n, m < M, k < K (orbitals x vectors),
// stored K-blocked: element (n, k) at complex index ((k / kBlkK) Mp + n) kBlkK + k % kBlkK
// (Mp >= M rows, a multiple of the 128-row tile, padding rows zero; K padded
// to whole blocks with zeros).  The kernels accumulate
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

// Workgroup tile: 128 (n) x 256 (m) complex; 8 waves (two per SIMD) in a
// 2 x 4 grid, each 64 x 64 complex (2 x 2 MFMA tiles of 32 x 32 for Re and for
// Im).  Padded row counts are multiples of kGammaRowAlign, so every tile lies
// inside the stored blocks.
constexpr int kGTileN = 128;
constexpr int kGTileM = 256;
constexpr int kGWave = 64;
static_assert(kGammaRowAlign % kGTileM == 0 && kGammaRowAlign % kGTileN == 0, "tiles must divide the row padding");
// K values (complex) per LDS stage, and the LDS row pitch in bf16: 32 reals
// (64 bytes, four 16-byte units), no padding.  The units of a row are
// permuted by an XOR with (row / 4) % 4, so that both the staging stores
// (16 lanes: 4 rows x 4 units) and the MFMA operand reads (16 lanes: 16
// rows, one unit) touch 16 distinct 16-byte bank groups of a 256-byte span
// of the 64 LDS banks.
constexpr int kGStage = 16;
constexpr int kGPitch = 2 * kGStage;
static_assert(kBlkK % kGStage == 0, "an LDS stage must not straddle a K block");
__device__ inline int gslab_unit(int row, int unit) { return unit ^ ((row >> 2) & 3); }

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

// One stage of the four planes: L hi/lo for the 128 n rows, R hi/lo for the
// 256 m rows (49152 bytes).
struct GammaSlab {
  __bf16 l[2][kGTileN][kGPitch];
  __bf16 r[2][kGTileM][kGPitch];
};

// grid = 8-multiple of (K splits x tiles); block = 512.  The blocks arrive
// already split into BF16 planes (hi, lo) in the K-blocked layout; Kc = complex
// values per row (whole K blocks), kchunk = complex values per split (a
// multiple of kGStage).  part[ks][n][m][2] (FP64) receives the chunk's result.
//
// Each stage moves a 16-complex slab of the four planes (48 KiB) from HBM into
// one of two LDS buffers through registers: the loads of stages s + 1 and
// s + 2 are in flight while the waves run the 48 MFMAs each of stage s out of
// the other buffer; one barrier per stage.  Two waves share each SIMD, so one wave's
// MFMAs cover the other's LDS and barrier waits.
__global__ void __launch_bounds__(512) gamma_bf16_kernel(const __bf16* __restrict__ Lh, const __bf16* __restrict__ Ll,
                                                         const __bf16* __restrict__ Rh, const __bf16* __restrict__ Rl,
                                                         int M, int Mp, int64_t Kc, int64_t kchunk, int ntn, int ntm,
                                                         int n_logical, double* __restrict__ part) {
  // Two distinct LDS objects (not one array indexed by a runtime parity), so
  // that the compiler may interleave the stores of one with reads of the other.
  __shared__ __attribute__((aligned(16))) GammaSlab lds0, lds1;
  // XCD-aware: the workgroups of XCD x take a contiguous range of logical ids,
  // so that the tiles sharing a K chunk run on one L2.
  const int G = gridDim.x;
  const int xcd = blockIdx.x & 7, jx = blockIdx.x >> 3, per = G >> 3;
  const int logical = xcd * per + jx;
  if (logical >= n_logical) return;
  const int tiles = ntn * ntm;
  const int tile = logical % tiles;
  const int ks = logical / tiles;
  const int tn = tile % ntn, tm = tile / ntn;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wn = wave & 1, wm = wave >> 1;
  const int r32 = lane & 31, kg = lane >> 5;
  const int n_base = tn * kGTileN + wn * kGWave, m_base = tm * kGTileM + wm * kGWave;
  const int64_t k_begin = (int64_t)ks * kchunk;
  const int64_t k_end = min(Kc, k_begin + kchunk);
  const int64_t n_stage = (k_end - k_begin) / kGStage;

  // Staging: a slab is 3072 16-byte units, L hi (512), L lo (512), R hi (1024),
  // R lo (1024); unit u of a plane is row u / 4, bf16 column 8 (u % 4).  Thread
  // t carries units t (L hi, L lo), t and t + 512 (R hi, R lo).  Their byte
  // offsets inside a K block are constant over the stages (rows < Mp <= 2^22
  // keeps them in 32 bits); the stage adds a wave-uniform offset to the base.
  const int srow = t >> 2, scol = (t & 3) * 8;
  uint32_t voff[3];
  voff[0] = (uint32_t)(((int64_t)(tn * kGTileN + srow) * (2 * kBlkK) + scol) * sizeof(__bf16));
  voff[1] = (uint32_t)(((int64_t)(tm * kGTileM + srow) * (2 * kBlkK) + scol) * sizeof(__bf16));
  voff[2] = (uint32_t)(((int64_t)(tm * kGTileM + 128 + srow) * (2 * kBlkK) + scol) * sizeof(__bf16));
  typedef bf16x8 Staging[6];
  Staging stgA, stgB;
  auto fetch = [&](Staging& stg, int64_t k0) {
    const int64_t soff = ((k0 / kBlkK) * (int64_t)Mp * (2 * kBlkK) + 2 * (k0 % kBlkK)) * (int64_t)sizeof(__bf16);
    const char* lh = reinterpret_cast<const char*>(Lh) + soff;
    const char* ll = reinterpret_cast<const char*>(Ll) + soff;
    const char* rh = reinterpret_cast<const char*>(Rh) + soff;
    const char* rl = reinterpret_cast<const char*>(Rl) + soff;
    stg[0] = *reinterpret_cast<const bf16x8*>(lh + voff[0]);
    stg[1] = *reinterpret_cast<const bf16x8*>(ll + voff[0]);
    stg[2] = *reinterpret_cast<const bf16x8*>(rh + voff[1]);
    stg[3] = *reinterpret_cast<const bf16x8*>(rh + voff[2]);
    stg[4] = *reinterpret_cast<const bf16x8*>(rl + voff[1]);
    stg[5] = *reinterpret_cast<const bf16x8*>(rl + voff[2]);
  };
  // Rows srow and 128 + srow share (row / 4) % 4, so one permuted column serves both.
  const int lcol = 8 * gslab_unit(srow, t & 3);
  auto stash = [&](const Staging& stg, GammaSlab& dst) {
    *reinterpret_cast<bf16x8*>(&dst.l[0][srow][lcol]) = stg[0];
    *reinterpret_cast<bf16x8*>(&dst.l[1][srow][lcol]) = stg[1];
    *reinterpret_cast<bf16x8*>(&dst.r[0][srow][lcol]) = stg[2];
    *reinterpret_cast<bf16x8*>(&dst.r[0][128 + srow][lcol]) = stg[3];
    *reinterpret_cast<bf16x8*>(&dst.r[1][srow][lcol]) = stg[4];
    *reinterpret_cast<bf16x8*>(&dst.r[1][128 + srow][lcol]) = stg[5];
  };

  f32x16 re[2][2], im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      re[i][j] = f32x16{};
      im[i][j] = f32x16{};
    }
  const int an = wn * kGWave + r32, bm = wm * kGWave + r32;
  // MFMA operands of one 16-real K step: rows an + 32 i of L (hi, lo) and
  // bm + 32 j of R (hi, lo).
  struct Ops {
    bf16x8 ah[2], al[2], bh[2], bl[2];
  };
  // Rows an + 32 i and bm + 32 j share (row / 4) % 4 with an and bm.
  const int ca[2] = {8 * gslab_unit(an, kg), 8 * gslab_unit(an, 2 + kg)};
  const int cb[2] = {8 * gslab_unit(bm, kg), 8 * gslab_unit(bm, 2 + kg)};
  auto read_ops = [&](const GammaSlab& src, int kk, Ops& o) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      o.ah[i] = *reinterpret_cast<const bf16x8*>(&src.l[0][an + 32 * i][ca[kk]]);
      o.al[i] = *reinterpret_cast<const bf16x8*>(&src.l[1][an + 32 * i][ca[kk]]);
      o.bh[i] = *reinterpret_cast<const bf16x8*>(&src.r[0][bm + 32 * i][cb[kk]]);
      o.bl[i] = *reinterpret_cast<const bf16x8*>(&src.r[1][bm + 32 * i][cb[kk]]);
    }
  };
  auto mfma = [&](const Ops& o) {
    bf16x8 b2h[2], b2l[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      b2h[j] = swap_neg(o.bh[j]);
      b2l[j] = swap_neg(o.bl[j]);
    }
    // The three split products are issued round-robin over the eight
    // accumulators, so consecutive MFMAs never depend on each other.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[i], o.bh[j], re[i][j], 0, 0, 0);
        im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[i], b2h[j], im[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[i], o.bl[j], re[i][j], 0, 0, 0);
        im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[i], b2l[j], im[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        re[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.al[i], o.bh[j], re[i][j], 0, 0, 0);
        im[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.al[i], b2h[j], im[i][j], 0, 0, 0);
      }
  };
  // One stage: the loads of the slab two stages ahead go out first (into the
  // staging set just emptied), the operands of the second K step are read
  // before the MFMAs of the first, and the next slab (loaded one stage
  // earlier) is stored into the other buffer at the end.  Past the last stage
  // the fetch re-reads the chunk's first slab (in bounds, never used).
  auto stage = [&](const GammaSlab& cur, GammaSlab& nxt, Staging& load_set, const Staging& store_set,
                   int64_t s_load) {
    Ops o0, o1;
    read_ops(cur, 0, o0);
    fetch(load_set, k_begin + (s_load < n_stage ? s_load : 0) * kGStage);
    // Keep the slab loads at the head of the stage (the scheduler would
    // otherwise sink them next to their use and expose their latency).
    __builtin_amdgcn_sched_barrier(0);
    read_ops(cur, 1, o1);
    mfma(o0);
    mfma(o1);
    stash(store_set, nxt);
    __syncthreads();
  };
  static_assert(kGStage / 8 == 2, "stage body is written for two K steps");

  // Stage s reads buffer s % 2, stores slab s + 1 (held in staging set
  // (s + 1) % 2) and loads slab s + 2 into staging set s % 2.
  fetch(stgA, k_begin);
  fetch(stgB, k_begin + (1 < n_stage ? 1 : 0) * kGStage);
  stash(stgA, lds0);
  __syncthreads();
  int64_t s = 0;
  for (; s + 2 <= n_stage; s += 2) {
    stage(lds0, lds1, stgA, stgB, s + 2);
    stage(lds1, lds0, stgB, stgA, s + 3);
  }
  if (s < n_stage) stage(lds0, lds1, stgA, stgB, s + 2);

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
    // of 16 and kBlkK of 16, so k0 + tx lies in K block k0 / kBlkK.
    const int64_t kb = (k0 / kBlkK) * (int64_t)Mp;
    const int64_t kq = k0 % kBlkK + tx;
    const int n = n0 + ty, m = m0 + ty;
    const bool kin = k0 + tx < k_end;
    const int64_t li = 2 * ((kb + n) * kBlkK + kq), ri = 2 * ((kb + m) * kBlkK + kq);
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
// values per row (a multiple of kBlkK); part holds KS * M * M * 2 doubles.
hipError_t gamma_accumulate_bf16(const __bf16* Lh, const __bf16* Ll, const __bf16* Rh, const __bf16* Rl, int M,
                                 int Mp, int64_t Kc, int KS, double* part, double* acc, hipStream_t s) {
  if (Kc % kBlkK != 0 || Mp % kGammaRowAlign != 0 || Mp < M) return hipErrorInvalidValue;
  const int ntn = (int)ceil_div(M, kGTileN), ntm = (int)ceil_div(M, kGTileM);
  const int64_t kchunk = ceil_div(ceil_div(Kc, KS), kGStage) * kGStage;
  const int ks_used = (int)ceil_div(Kc, kchunk);
  const int n_logical = ks_used * ntn * ntm;
  const int grid = (int)ceil_div(n_logical, 8) * 8;
  hipLaunchKernelGGL(gamma_bf16_kernel, dim3(grid), dim3(512), 0, s, Lh, Ll, Rh, Rl, M, Mp, Kc, kchunk, ntn, ntm,
                     n_logical, part);
  const int64_t n = (int64_t)M * M * 2;
  hipLaunchKernelGGL(gamma_reduce_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, part, ks_used, n, acc);
  return ::kpm::launch_status();
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
  return ::kpm::launch_status();
}

template hipError_t gamma_accumulate_fp64<float>(const float*, const float*, int, int, int64_t, int, double*,
                                                 double*, hipStream_t);
template hipError_t gamma_accumulate_fp64<double>(const double*, const double*, int, int, int64_t, int, double*,
                                                  double*, hipStream_t);

}  // namespace kpm
