// Rank-2 conductivity moments Gamma_nm (paper eq. Gammanm) with the
// stochastic trace (Sec. 2(c)):
//
//   Gamma_nm = 1/(R N) sum_r <L_n^r | R_m^r> / ((1 + d_n0)(1 + d_m0)),
//   L_n = T_n(H~) (-h~^a |r>),   R_m = h~^b T_m(H~) |r>,
//
// where h~^a = [r^a, H] (eq. generalized velocity times i hbar) is
// anti-Hermitian, so <r| h~^a T_n h~^b T_m |r> = <L_n | R_m>.  Both chains run
// through the Chebyshev step kernel: the L chain stores every T_n(H~) w as a
// row of the block L; the R chain applies the velocity stencil to T_m |r> in
// the same pass that produces T_{m+1} |r> and stores it as a row of R.  The
// double sum over n, m is a GEMM over the stored blocks (orbitals x vectors
// form the contraction index).  Vectors are processed in batches sized to the
// free device memory.

#include "kpm_internal.h"
#include "kpm_plan.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace kpm {

hipError_t gamma_accumulate_bf16(const __bf16* Lh, const __bf16* Ll, const __bf16* Rh, const __bf16* Rl, int M,
                                 int Mp, int64_t Kc, int KS, double* part, double* acc, hipStream_t s);
template <typename T>
hipError_t gamma_accumulate_fp64(const T* L, const T* R, int M, int Mp, int64_t Kc, int KS, double* part,
                                 double* acc, hipStream_t s);

__global__ void zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Gamma = acc / (R N_active) / ((1 + d_n0)(1 + d_m0)).
__global__ void gamma_scale_kernel(const double* acc, int M, int R, const unsigned long long* active, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * M * 2) return;
  const int64_t nm = i >> 1;
  const int n = (int)(nm / M), m = (int)(nm % M);
  const double d = (n == 0 ? 2.0 : 1.0) * (m == 0 ? 2.0 : 1.0);
  out[i] = acc[i] / ((double)R * (double)active[0]) / d;
}

static thread_local kpm_cond_stats_t g_stats;

static int cond_run(const kpm_lattice_t* lat, const kpm_cond_params_t* p, double* gamma, int32_t on_dev,
                    void* stream) {
  std::memset(&g_stats, 0, sizeof(g_stats));
  KPM_CHECK_ARG(lat && p && gamma, "NULL argument");
  KPM_CHECK_ARG(p->num_moments >= 2, "num_moments must be >= 2");
  KPM_CHECK_ARG(p->num_random >= 1, "num_random must be >= 1");
  KPM_CHECK_ARG((p->alpha == 0 || p->alpha == 1) && (p->beta == 0 || p->beta == 1), "alpha, beta must be 0 (x) or 1 (y)");
  KPM_CHECK_ARG(p->gamma_mode == KPM_GAMMA_FP64 || p->gamma_mode == KPM_GAMMA_SPLIT_BF16,
                "gamma_mode must be KPM_GAMMA_FP64 or KPM_GAMMA_SPLIT_BF16");
  KPM_CHECK_ARG(p->precision == KPM_FP32 || p->precision == KPM_FP64, "precision must be KPM_FP32 or KPM_FP64");
  KPM_CHECK_ARG(!(p->gamma_mode == KPM_GAMMA_SPLIT_BF16 && p->precision != KPM_FP32),
                "KPM_GAMMA_SPLIT_BF16 needs FP32 blocks (precision = KPM_FP32)");
  hipStream_t s = (hipStream_t)stream;
  const int M = p->num_moments, Rtot = p->num_random;
  const int n_sub = lat->kind == KPM_SQUARE ? 1 : 2;
  const int n_spin = lat->kind == KPM_HONEYCOMB_SPIN ? 2 : 1;
  const int64_t n_orb = (int64_t)lat->L1 * lat->L2 * n_sub * n_spin;
  const size_t tsize = p->precision == KPM_FP32 ? 4 : 8;

  // Vectors per batch: two [M][n_orb][Rb] blocks must fit in free memory.
  size_t free_b = 0, total_b = 0;
  KPM_TRY_HIP(hipMemGetInfo(&free_b, &total_b));
  const double per_vec = 2.0 * M * (double)n_orb * 2 * tsize + 2.0 * (double)n_orb * 2 * tsize;
  const double usable = 0.85 * (double)free_b - 4.0e9;   // plan buffers and moment partials
  int rb_max = (int)std::max(0.0, std::floor(usable / per_vec));
  if (p->max_batch > 0) rb_max = std::min(rb_max, p->max_batch);
  if (rb_max < 1) {
    set_error("not enough device memory for one vector: need %.1f GB of Chebyshev blocks", per_vec / 1e9);
    return KPM_E_NOMEM;
  }
  rb_max = std::min(rb_max, Rtot);
  const int n_batch = (int)ceil_div(Rtot, rb_max);
  const int Rb = (int)ceil_div(Rtot, n_batch);

  kpm_dos_params_t dp;
  std::memset(&dp, 0, sizeof(dp));
  dp.num_moments = M;
  dp.num_random = Rb;
  dp.vector_seed = p->vector_seed;
  dp.precision = p->precision;
  dp.start = KPM_START_RANDOM_PHASE;
  kpm_tune_t tune;
  std::memset(&tune, 0, sizeof(tune));
  tune.use_graph = 0;
  tune.kernel = 2;   // single steps (the chains interleave velocity and block stores)
  kpm_plan* P = nullptr;
  KPM_TRY(plan_create(lat, 1, &dp, &tune, &P));

  const int64_t vec_elems = n_orb * P->Rp * 2;   // T elements per Chebyshev vector
  // Rows of the Gamma blocks: complex length padded to whole K blocks (zeros).
  const int64_t kpad = ceil_div(n_orb * P->Rp, kBlkK) * kBlkK;
  const int64_t row_elems = 2 * kpad;
  // Rows of the blocked store: M rounded up to whole GEMM tiles (zero rows).
  const int Mp = (int)ceil_div(M, kGammaRowAlign) * kGammaRowAlign;
  const int KS = 64;
  // Split-BF16 mode stores each block as two BF16 planes (hi, lo): the same
  // bytes as FP32; the FP64 mode stores the blocks in the vectors' precision.
  const bool split = p->gamma_mode == KPM_GAMMA_SPLIT_BF16;
  void *Lb = nullptr, *Rblk = nullptr, *Llo = nullptr, *Rlo = nullptr;
  double *acc = nullptr, *part = nullptr, *gdev = nullptr;
  int st = KPM_OK;
  auto fail = [&](hipError_t e, const char* what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    (void)hipGetLastError();
    st = (e == hipErrorOutOfMemory) ? KPM_E_NOMEM : KPM_E_DEVICE;
  };
  const size_t plane_bytes = split ? (size_t)Mp * row_elems * 2 : (size_t)Mp * row_elems * tsize;
  hipError_t e = ::kpm::dev_malloc(&Lb, plane_bytes);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&Rblk, plane_bytes);
  if (e == hipSuccess && split) e = ::kpm::dev_malloc(&Llo, plane_bytes);
  if (e == hipSuccess && split) e = ::kpm::dev_malloc(&Rlo, plane_bytes);
  if (e == hipSuccess && (kpad != n_orb * P->Rp || Mp != M)) {   // padding rows / K block stay zero
    for (void* b : {Lb, Rblk, Llo, Rlo})
      if (b && e == hipSuccess) e = hipMemsetAsync(b, 0, plane_bytes, s);
  }
  if (e == hipSuccess) e = ::kpm::dev_malloc(&acc, (size_t)M * M * 2 * sizeof(double));
  if (e == hipSuccess) e = ::kpm::dev_malloc(&part, (size_t)KS * M * M * 2 * sizeof(double));
  if (e == hipSuccess && !on_dev) e = ::kpm::dev_malloc(&gdev, (size_t)M * M * 2 * sizeof(double));
  if (e != hipSuccess) fail(e, "allocating Gamma blocks");
  double* gout = on_dev ? gamma : gdev;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  if (e != hipSuccess && st == KPM_OK) fail(e, "creating events");
  // Multi-step chain sweeps: KS = 4 steps per launch on the spinful lattice
  // (3 in FP64), 2 on the spinless ones (the fastest measured on 1024^2
  // lattices; the spinless kernels are bound by instruction issue at larger
  // KS).  KPM_CHAIN_STEPS=1 keeps single steps, 2..4 sets KS; KPM_CHAIN_ROWS
  // sets the rows per tile.  Without a tile shape that fits, single steps.
  ChainPlan C;
  bool sweep_chains = false;
  if (st == KPM_OK) {
    int ks = (P->n_spin == 2) ? 4 : 2, rows = 0;
    if (const char* cs = std::getenv("KPM_CHAIN_STEPS"); cs && *cs) ks = std::atoi(cs);
    if (const char* cr = std::getenv("KPM_CHAIN_ROWS"); cr && *cr) rows = std::max(0, std::atoi(cr));
    if (ks >= 2) {
      const int cst = chain_plan_create(P, std::min(ks, 4), rows, Mp, &C);
      if (cst == KPM_OK) sweep_chains = true;
      else if (cst == KPM_E_UNSUPPORTED) clear_error();   // single steps
      else st = cst;
    }
  }
  if (st == KPM_OK) e = hipEventRecord(ev[3], s);
  g_stats.n_batches = n_batch;
  g_stats.vectors_per_batch = Rb;
  const double vec_bytes = (double)vec_elems * tsize;
  const double site_bytes = (P->has_onsite ? (double)P->n_sites * tsize : 0.0) + (P->has_mask ? (double)P->n_sites : 0.0);
  auto step_bytes = [&](const StepLaunch& S) {
    // The block copy costs one vector (FP32/FP64) or two BF16 planes (the same bytes in FP32).
    return vec_bytes * (1.0 + S.read_w + S.write_out + (S.vel ? 1.0 : 0.0) + (S.blk ? 1.0 : 0.0)) + site_bytes;
  };
  if (st == KPM_OK) {
    hipLaunchKernelGGL(zero_f64, dim3((unsigned)ceil_div((int64_t)M * M * 2, 256)), dim3(256), 0, s, acc,
                       (int64_t)M * M * 2);
  }
  for (int b = 0; b < n_batch && st == KPM_OK; ++b) {
    const int r0 = b * Rb;
    P->R = std::min(Rb, Rtot - r0);   // vectors of this batch beyond Rtot start as zero
    st = plan_set_vector_base(P, r0);
    if (st != KPM_OK) break;
    e = plan_launch_prep(P, s);
    if (e != hipSuccess) { fail(e, "model/start kernels"); break; }
    e = hipEventRecord(ev[0], s);
    if (sweep_chains) {
      // L_0 = -h~^a xi by one velocity launch (into Y and block row 0), then L_1 .. L_{M-1}
      // by sweeps, each level into its block row.
      StepLaunch S0;
      S0.dots = 0;
      S0.blk = Lb;
      S0.blk_lo = Llo;
      S0.blk_row = 0;
      S0.blk_rows = Mp;
      S0.v = P->X; S0.out = P->Y; S0.write_out = 0; S0.read_w = 0; S0.a = 0.0; S0.b = 0.0;
      S0.velocity = true; S0.vel = P->Y; S0.vdir = p->alpha; S0.vel_scale = -1.0; S0.blk_src = 1;
      if (e == hipSuccess) e = plan_launch_step(P, s, S0);
      g_stats.chain_bytes += step_bytes(S0);
      if (e == hipSuccess && M > 1)
        e = chain_run(P, C, s, 0, P->Y, P->X, M - 1, Lb, Llo, Mp, 0, 1.0, &g_stats.chain_bytes);
      // R chain from xi again: R_m = h~^b T_m(H~) xi for m = 0 .. M-1 (M levels, each
      // giving the velocity of the level below).
      if (e == hipSuccess) e = plan_launch_prep(P, s);
      if (e == hipSuccess) e = chain_run(P, C, s, 1, P->X, P->Y, M, Rblk, Rlo, Mp, p->beta, 1.0, &g_stats.chain_bytes);
    }
    // L chain: L_0 = -h~^a xi, L_1 = H~ L_0, L_n = 2 H~ L_{n-1} - L_{n-2}, kept in the
    // plan's two vector buffers (L_n in X for odd n, in Y for even n >= 2) and
    // copied row by row into the K-blocked block Lb.
    for (int n = 0; n < M && e == hipSuccess && !sweep_chains; ++n) {
      StepLaunch S;
      S.dots = 0;
      S.blk = Lb;
      S.blk_lo = Llo;
      S.blk_row = n;
      S.blk_rows = Mp;
      if (n == 0) {
        S.v = P->X; S.out = P->Y; S.write_out = 0; S.read_w = 0; S.a = 0.0; S.b = 0.0;
        S.velocity = true; S.vel = P->Y; S.vdir = p->alpha; S.vel_scale = -1.0; S.blk_src = 1;
      } else if (n == 1) {
        S.v = P->Y; S.out = P->X; S.read_w = 0; S.a = 1.0; S.b = 0.0;
      } else {
        const bool even = (n & 1) == 0;
        S.v = even ? P->X : P->Y;
        S.w = even ? P->Y : P->X;
        S.out = even ? P->Y : P->X;
      }
      e = plan_launch_step(P, s, S);
      g_stats.chain_bytes += step_bytes(S);
    }
    // R chain: start again from xi; v_0 = xi, v_1 = H~ v_0, v_{m+1} = 2 H~ v_m - v_{m-1}
    // (in place), with R_m = h~^b v_m from the same pass stored K-blocked in Rblk.
    if (e == hipSuccess && !sweep_chains) e = plan_launch_prep(P, s);
    for (int m = 0; m < M && e == hipSuccess && !sweep_chains; ++m) {
      StepLaunch S;
      S.dots = 0;
      S.velocity = true;
      S.vdir = p->beta;
      S.vel_scale = 1.0;
      S.blk = Rblk;
      S.blk_lo = Rlo;
      S.blk_src = 1;
      S.blk_row = m;
      S.blk_rows = Mp;
      if (m == 0) {
        S.v = P->X; S.out = P->Y; S.read_w = 0; S.a = 1.0; S.b = 0.0;
      } else {
        const bool odd = (m & 1) != 0;
        S.v = odd ? P->Y : P->X;
        S.w = odd ? P->X : P->Y;
        S.out = odd ? P->X : P->Y;
      }
      S.write_out = (m < M - 1) ? 1 : 0;
      e = plan_launch_step(P, s, S);
      g_stats.chain_bytes += step_bytes(S);
    }
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e != hipSuccess) { fail(e, "Chebyshev chains"); break; }
    // Flops: 2 real GEMMs (Re, Im) of M x M over 2 vec_elems/2 reals = 4 M^2 vec_elems.
    g_stats.gemm_useful_flops += 4.0 * M * (double)M * (double)row_elems;
    g_stats.gemm_mfma_flops += (p->gamma_mode == KPM_GAMMA_SPLIT_BF16 ? 3.0 : 1.0) * 4.0 * M * (double)M * row_elems;
    g_stats.gemm_operand_bytes += 2.0 * M * (double)row_elems * 4.0;
    if (p->gamma_mode == KPM_GAMMA_SPLIT_BF16) {
      e = gamma_accumulate_bf16((const __bf16*)Lb, (const __bf16*)Llo, (const __bf16*)Rblk, (const __bf16*)Rlo, M,
                                Mp, kpad, KS, part, acc, s);
    } else if (p->precision == KPM_FP32) {
      e = gamma_accumulate_fp64<float>((const float*)Lb, (const float*)Rblk, M, Mp, kpad, KS, part, acc, s);
    } else {
      e = gamma_accumulate_fp64<double>((const double*)Lb, (const double*)Rblk, M, Mp, kpad, KS, part, acc, s);
    }
    if (e == hipSuccess) e = hipEventRecord(ev[2], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
    float ms_c = 0.f, ms_g = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_c, ev[0], ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_g, ev[1], ev[2]);
    g_stats.chain_ms += ms_c;
    g_stats.gemm_ms += ms_g;
    if (e != hipSuccess) fail(e, "Gamma GEMM");
  }
  if (st == KPM_OK) {
    hipLaunchKernelGGL(gamma_scale_kernel, dim3((unsigned)ceil_div((int64_t)M * M * 2, 256)), dim3(256), 0, s, acc, M,
                       Rtot, P->active, gout);
    e = ::kpm::launch_status();
    if (e == hipSuccess && !on_dev)
      e = hipMemcpyAsync(gamma, gdev, (size_t)M * M * 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) fail(e, "Gamma output");
  } else {
    (void)hipStreamSynchronize(s);
  }
  if (st == KPM_OK) {
    float ms_t = 0.f;
    if (hipEventRecord(ev[2], s) == hipSuccess && hipEventSynchronize(ev[2]) == hipSuccess &&
        hipEventElapsedTime(&ms_t, ev[3], ev[2]) == hipSuccess)
      g_stats.total_ms = ms_t;
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  for (void* ptr : {Lb, Rblk, Llo, Rlo, (void*)acc, (void*)part, (void*)gdev})
    if (ptr) (void)::kpm::dev_free(ptr);
  chain_plan_free(&C);
  plan_free(P);
  delete P;
  return st;
}

// Rank-1 tensor Gamma_n^{ab} = Tr[h~^{ab} T_n(H~)] / (N (1 + d_n0)) (paper eq.
// Gammanm family, rank 1), h~^{ab} = [r^a, [r^b, H]] Hermitian, with the
// stochastic trace: (1/(R N)) sum_r <T_n(H~) r | h~^{ab} r>.  u = h~^{ab} r comes
// from one velocity-only launch of the step kernel (second-order weights);
// the recursion then runs in place over two buffers and each step's dot
// product <v_n | u> is summed per workgroup in FP64 and reduced in a fixed
// order at the end.
constexpr int kDotBlocks = 1024;

template <typename T>
__global__ void dot_partial_kernel(const T* __restrict__ v, const T* __restrict__ u, int64_t n_cplx,
                                   double* __restrict__ part) {
  __shared__ double sr[256], si[256];
  double ar = 0.0, ai = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_cplx; i += (int64_t)gridDim.x * blockDim.x) {
    const double vr = v[2 * i], vi = v[2 * i + 1], ur = u[2 * i], ui = u[2 * i + 1];
    ar += vr * ur + vi * ui;   // conj(v) u
    ai += vr * ui - vi * ur;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      sr[threadIdx.x] += sr[threadIdx.x + st];
      si[threadIdx.x] += si[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr[0];
    part[2 * blockIdx.x + 1] = si[0];
  }
}

__global__ void gamma1_finish_kernel(const double* part, int M, int R, const unsigned long long* active, double* out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= M) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < kDotBlocks; ++b) {
    re += part[((int64_t)n * kDotBlocks + b) * 2];
    im += part[((int64_t)n * kDotBlocks + b) * 2 + 1];
  }
  const double sc = 1.0 / ((double)R * (double)active[0] * (n == 0 ? 2.0 : 1.0));
  out[2 * n] = re * sc;
  out[2 * n + 1] = im * sc;
}

static int gamma1_run(const kpm_lattice_t* lat, const kpm_cond_params_t* p, double* g1, int32_t on_dev,
                      void* stream) {
  KPM_CHECK_ARG(lat && p && g1, "NULL argument");
  KPM_CHECK_ARG(p->num_moments >= 1, "num_moments must be >= 1");
  KPM_CHECK_ARG(p->num_random >= 1, "num_random must be >= 1");
  KPM_CHECK_ARG((p->alpha == 0 || p->alpha == 1) && (p->beta == 0 || p->beta == 1), "alpha, beta must be 0 (x) or 1 (y)");
  KPM_CHECK_ARG(p->precision == KPM_FP32 || p->precision == KPM_FP64, "precision must be KPM_FP32 or KPM_FP64");
  hipStream_t s = (hipStream_t)stream;
  const int M = p->num_moments, R = p->num_random;
  kpm_dos_params_t dp;
  std::memset(&dp, 0, sizeof(dp));
  dp.num_moments = std::max(2, M);
  dp.num_random = R;
  dp.vector_seed = p->vector_seed;
  dp.precision = p->precision;
  dp.start = KPM_START_RANDOM_PHASE;
  kpm_tune_t tune;
  std::memset(&tune, 0, sizeof(tune));
  tune.use_graph = 0;
  tune.kernel = 2;
  kpm_plan* P = nullptr;
  KPM_TRY(plan_create(lat, 1, &dp, &tune, &P));
  const int64_t n_cplx = P->n_orb * P->Rp;
  void* U = nullptr;
  double *part = nullptr, *gdev = nullptr;
  int st = KPM_OK;
  hipError_t e = ::kpm::dev_malloc(&U, (size_t)n_cplx * 2 * P->tsize);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&part, (size_t)M * kDotBlocks * 2 * sizeof(double));
  if (e == hipSuccess && !on_dev) e = ::kpm::dev_malloc(&gdev, (size_t)M * 2 * sizeof(double));
  if (e == hipSuccess) st = plan_set_vector_base(P, 0);
  if (e == hipSuccess && st == KPM_OK) e = plan_launch_prep(P, s);
  auto dot = [&](const void* v, int n) {
    if (P->prec == KPM_FP32)
      hipLaunchKernelGGL(dot_partial_kernel<float>, dim3(kDotBlocks), dim3(256), 0, s, (const float*)v, (const float*)U,
                         n_cplx, part + (int64_t)n * kDotBlocks * 2);
    else
      hipLaunchKernelGGL(dot_partial_kernel<double>, dim3(kDotBlocks), dim3(256), 0, s, (const double*)v,
                         (const double*)U, n_cplx, part + (int64_t)n * kDotBlocks * 2);
    return ::kpm::launch_status();
  };
  if (e == hipSuccess && st == KPM_OK) {
    // u = h~^{ab} xi (velocity-only launch: no output vector, no dots).
    StepLaunch S;
    S.v = P->X; S.out = P->Y; S.write_out = 0; S.read_w = 0; S.dots = 0; S.a = 0.0; S.b = 0.0;
    S.velocity = true; S.vel = U; S.vdir = 2 + p->alpha + p->beta; S.vel_scale = 1.0;
    e = plan_launch_step(P, s, S);
  }
  void* cur = P->X;
  void* prev = P->Y;
  for (int n = 0; n < M && e == hipSuccess && st == KPM_OK; ++n) {
    if (n == 1) {
      StepLaunch S;
      S.v = P->X; S.out = P->Y; S.read_w = 0; S.a = 1.0; S.b = 0.0; S.dots = 0;
      e = plan_launch_step(P, s, S);
      cur = P->Y;
      prev = P->X;
    } else if (n >= 2) {
      StepLaunch S;
      S.v = cur; S.w = prev; S.out = prev; S.dots = 0;   // v_n over v_{n-2}, in place
      e = plan_launch_step(P, s, S);
      std::swap(cur, prev);
    }
    if (e == hipSuccess) e = dot(cur, n);
  }
  if (e == hipSuccess && st == KPM_OK) {
    double* out = on_dev ? g1 : gdev;
    hipLaunchKernelGGL(gamma1_finish_kernel, dim3((unsigned)ceil_div(M, 256)), dim3(256), 0, s, part, M, R, P->active,
                       out);
    e = ::kpm::launch_status();
    if (e == hipSuccess && !on_dev) e = hipMemcpyAsync(g1, gdev, (size_t)M * 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  } else {
    (void)hipStreamSynchronize(s);
  }
  if (e != hipSuccess && st == KPM_OK) {
    set_error("kpm_moments_gamma1: %s", hipGetErrorString(e));
    st = (e == hipErrorOutOfMemory) ? KPM_E_NOMEM : KPM_E_DEVICE;
  }
  for (void* ptr : {U, (void*)part, (void*)gdev})
    if (ptr) (void)::kpm::dev_free(ptr);
  plan_free(P);
  delete P;
  return st;
}

// ---------------------------------------------------------------------------
// Single-shot Fermi-surface DC conductivity (the paper's 'single-shot'
// algorithm, Sec. 3(b), which avoids the double recursion of eq. Gammanm):
//   sigma_ab(E)/(e^2/h) = -2 pi^2 (1/Omega) Tr[h~^a d_eta(E-H) h~^b d_eta(E-H)],
//   d_eta(E - H) = sum_n c_n(E) T_n(H~),  c_n = -Im g_n(z~)/(pi de- (1 + d_n0))
// (CPGF coefficients of eq. green_function_cheb_expansionb at z~ = eps + i eta~),
// with the stochastic trace -(1/R) sum_r <a|b>, a = d_eta h~^a r, b = h~^b d_eta r.
// Two recursions per vector serve every energy: the accumulators
// A_k = sum_n c_n(E_k) T_n(H~) h~^a r and B_k = sum_n c_n(E_k) T_n(H~) r.
// Each recursion writes T_n x into slot n mod B of a history of B vectors;
// every B steps one pass reads the B vectors once and adds their weighted sum
// to each accumulator (read and written once per B steps instead of once per
// step: per step 1 + 2 K / B vectors move instead of 2 K).  B (<= 64) and the
// energies per batch are sized to the free device memory.
// ---------------------------------------------------------------------------
constexpr int kMaxHist = 64;    // history vectors per flush
constexpr int kAccGroup = 16;   // energies per flush pass (FP64 sums in registers)

template <typename T>
struct HistPtrs {
  const T* v[kMaxHist];
};

// acc_k[i] += sum_{b < nb} coef[b ldc + k] v_b[i] for k < kk <= kAccGroup; the
// coefficient rows hold kAccGroup valid entries (zero padded).  One element per
// thread, its kAccGroup sums in FP64, the accumulator rounded once per flush.
template <typename T>
__global__ void accumulate_block_kernel(HistPtrs<T> H, int nb, int64_t n_elems, T* __restrict__ acc, int64_t stride,
                                        const double* __restrict__ coef, int ldc, int kk) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_elems; i += (int64_t)gridDim.x * blockDim.x) {
    double a[kAccGroup];
#pragma unroll
    for (int k = 0; k < kAccGroup; ++k) a[k] = 0.0;
#pragma unroll 4
    for (int b = 0; b < nb; ++b) {
      const double x = (double)H.v[b][i];
      const double* c = coef + (int64_t)b * ldc;
#pragma unroll
      for (int k = 0; k < kAccGroup; ++k) a[k] += c[k] * x;
    }
#pragma unroll
    for (int k = 0; k < kAccGroup; ++k)
      if (k < kk) acc[k * stride + i] = (T)((double)acc[k * stride + i] + a[k]);
  }
}

template <typename T>
__global__ void zero_kernel(T* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (T)0;
}

__global__ void singleshot_finish_kernel(const double* part, int K, double scale, double* sigma) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double re = 0.0;
  for (int b = 0; b < kDotBlocks; ++b) re += part[((int64_t)k * kDotBlocks + b) * 2];
  sigma[k] = scale * re;
}

static int singleshot_run(const kpm_lattice_t* lat, const kpm_cond_params_t* p, const double* energies_ev, int32_t K,
                          double eta_ev, double* sigma, int32_t on_dev, void* stream) {
  KPM_CHECK_ARG(lat && p && energies_ev && sigma, "NULL argument");
  KPM_CHECK_ARG(p->num_moments >= 2, "num_moments must be >= 2");
  KPM_CHECK_ARG(p->num_random >= 1, "num_random must be >= 1");
  KPM_CHECK_ARG(K >= 1 && K <= 4096, "need 1 <= K <= 4096 energies");
  KPM_CHECK_ARG(eta_ev > 0.0 && std::isfinite(eta_ev), "eta must be > 0");
  KPM_CHECK_ARG((p->alpha == 0 || p->alpha == 1) && (p->beta == 0 || p->beta == 1), "alpha, beta must be 0 (x) or 1 (y)");
  KPM_CHECK_ARG(p->precision == KPM_FP32 || p->precision == KPM_FP64, "precision must be KPM_FP32 or KPM_FP64");
  hipStream_t s = (hipStream_t)stream;
  const int M = p->num_moments, R = p->num_random;
  std::vector<double> en((size_t)K);
  if (on_dev) {
    KPM_TRY_HIP(hipMemcpyAsync(en.data(), energies_ev, sizeof(double) * K, hipMemcpyDeviceToHost, s));
    KPM_TRY_SYNC(hipStreamSynchronize(s));
  } else {
    std::memcpy(en.data(), energies_ev, sizeof(double) * K);
  }
  // Coefficients c_n(E_k) (host, FP64): g_n(z) = -2i w^n / sqrt(1 - z^2), w = exp(-i arccos z)
  // the root of w^2 - 2 z w + 1 inside the unit circle, sqrt(1 - z^2) = i (w - z).
  const double de_p = 0.5 * (lat->e_max + lat->e_min), de_m = 0.5 * (lat->e_max - lat->e_min);
  // [n][Kp], Kp = K rounded up to kAccGroup, zero padded, plus kAccGroup zeros at
  // the end: a flush pass reads kAccGroup entries of a row from any energy
  // offset (a batch need not start at a multiple of kAccGroup), and uses kk.
  const int Kp = (int)ceil_div(K, kAccGroup) * kAccGroup;
  std::vector<double> coef((size_t)Kp * M + kAccGroup, 0.0);
  for (int k = 0; k < K; ++k) {
    typedef std::complex<double> cd;
    const cd z((en[k] - de_p) / de_m, eta_ev / de_m);
    const cd r = std::sqrt(z * z - 1.0);
    const cd outer = std::abs(z + r) >= std::abs(z - r) ? z + r : z - r;
    const cd w = 1.0 / outer;
    const cd pre = -2.0 / (w - z);   // g_n = pre w^n
    cd pw(1.0, 0.0);
    for (int n = 0; n < M; ++n) {
      coef[(size_t)n * Kp + k] = -std::imag(pre * pw) / (M_PI * de_m) / (n == 0 ? 2.0 : 1.0);
      pw *= w;
    }
  }
  kpm_dos_params_t dp;
  std::memset(&dp, 0, sizeof(dp));
  dp.num_moments = M;
  dp.num_random = R;
  dp.vector_seed = p->vector_seed;
  dp.precision = p->precision;
  dp.start = KPM_START_RANDOM_PHASE;
  kpm_tune_t tune;
  std::memset(&tune, 0, sizeof(tune));
  tune.use_graph = 0;
  tune.kernel = 2;
  kpm_plan* P = nullptr;
  KPM_TRY(plan_create(lat, 1, &dp, &tune, &P));
  const int64_t n_elems = P->n_orb * P->Rp * 2;
  const size_t vec_b = (size_t)n_elems * P->tsize;
  size_t free_b = 0, total_b = 0;
  int st = KPM_OK;
  hipError_t e = hipMemGetInfo(&free_b, &total_b);
  // Room in vectors besides the start copy and a scratch vector: the history
  // takes up to a third of it (3 <= B <= 64, no more than M), each energy of a
  // batch two accumulators.
  const double room = std::floor((0.85 * (double)free_b - 2.0 * vec_b - 1.0e9) / (double)vec_b);
  const int B = (int)std::max(3.0, std::min<double>(std::min(kMaxHist, M), std::floor(room / 3.0)));
  const int kb = (int)std::min<double>(K, std::floor((room - B) / 2.0));
  if (e == hipSuccess && kb < 1) {
    set_error("not enough device memory for the single-shot history and accumulators (%.1f GB per vector, %d + 2 "
              "needed)", vec_b / 1e9, B);
    plan_free(P);
    delete P;
    return KPM_E_NOMEM;
  }
  void *V0 = nullptr, *Sc = nullptr, *acc = nullptr, *hist = nullptr;
  double *dcoef = nullptr, *part = nullptr, *dsig = nullptr;
  if (e == hipSuccess) e = ::kpm::dev_malloc(&V0, vec_b);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&Sc, vec_b);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&acc, 2 * vec_b * (size_t)kb);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&hist, vec_b * (size_t)B);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&dcoef, sizeof(double) * coef.size());
  if (e == hipSuccess) e = ::kpm::dev_malloc(&part, sizeof(double) * 2 * kDotBlocks * (size_t)K);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&dsig, sizeof(double) * K);
  if (e == hipSuccess) e = hipMemcpyAsync(dcoef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) st = plan_set_vector_base(P, 0);
  const bool f32 = P->prec == KPM_FP32;
  const dim3 eg(2048), eb(256);
  // T_n x0: x0 itself for n = 0, history slot n mod B otherwise.
  auto hvec = [&](void* x0, int n) -> void* { return n == 0 ? x0 : (char*)hist + vec_b * (size_t)(n % B); };
  // Accumulators k0 .. k0 + kk - 1 (at A) += sum over steps n0 .. n0 + nb - 1 of c_n(E_k) T_n x0.
  auto flush = [&](void* x0, void* A, int n0, int nb, int k0, int kk) {
    hipError_t er = hipSuccess;
    for (int g = 0; g < kk && er == hipSuccess; g += kAccGroup) {
      const int kg = std::min(kAccGroup, kk - g);
      const double* c = dcoef + (size_t)n0 * Kp + k0 + g;
      char* Ag = (char*)A + vec_b * (size_t)g;
      if (f32) {
        HistPtrs<float> H;
        for (int b = 0; b < nb; ++b) H.v[b] = (const float*)hvec(x0, n0 + b);
        hipLaunchKernelGGL(accumulate_block_kernel<float>, eg, eb, 0, s, H, nb, n_elems, (float*)Ag, n_elems, c, Kp,
                           kg);
      } else {
        HistPtrs<double> H;
        for (int b = 0; b < nb; ++b) H.v[b] = (const double*)hvec(x0, n0 + b);
        hipLaunchKernelGGL(accumulate_block_kernel<double>, eg, eb, 0, s, H, nb, n_elems, (double*)Ag, n_elems, c,
                           Kp, kg);
      }
      er = ::kpm::launch_status();
    }
    return er;
  };
  // One recursion from x0 into the history, flushed every B steps (a slot is
  // rewritten only after its vector has been flushed).
  auto chain = [&](void* x0, void* A, int k0, int kk) {
    hipError_t er = hipSuccess;
    int n0 = 0;   // first step not yet flushed
    for (int n = 1; n < M && er == hipSuccess; ++n) {
      StepLaunch S;
      S.dots = 0;
      S.v = hvec(x0, n - 1);
      S.out = hvec(x0, n);
      if (n == 1) {
        S.read_w = 0; S.a = 1.0; S.b = 0.0;
      } else {
        S.w = hvec(x0, n - 2);
      }
      er = plan_launch_step(P, s, S);
      if (er == hipSuccess && n + 1 - n0 == B) {
        er = flush(x0, A, n0, B, k0, kk);
        n0 = n + 1;
      }
    }
    if (er == hipSuccess && n0 < M) er = flush(x0, A, n0, M - n0, k0, kk);
    return er;
  };
  for (int k0 = 0; k0 < K && e == hipSuccess && st == KPM_OK; k0 += kb) {
    const int kk = std::min(kb, K - k0);
    char* Ab = (char*)acc;
    char* Bb = (char*)acc + vec_b * (size_t)kb;
    if (f32)
      hipLaunchKernelGGL(zero_kernel<float>, eg, eb, 0, s, (float*)acc, 2 * n_elems * (int64_t)kb);
    else
      hipLaunchKernelGGL(zero_kernel<double>, eg, eb, 0, s, (double*)acc, 2 * n_elems * (int64_t)kb);
    // r into X; x0 = h~^a r into V0 (velocity-only launch).
    e = plan_launch_prep(P, s);
    if (e == hipSuccess) {
      StepLaunch S;
      S.v = P->X; S.out = P->Y; S.write_out = 0; S.read_w = 0; S.dots = 0; S.a = 0.0; S.b = 0.0;
      S.velocity = true; S.vel = V0; S.vdir = p->alpha; S.vel_scale = 1.0;
      e = plan_launch_step(P, s, S);
    }
    if (e == hipSuccess) e = chain(V0, Ab, k0, kk);     // A_k = d_eta(E_k) h~^a r
    if (e == hipSuccess) e = chain(P->X, Bb, k0, kk);   // B_k = d_eta(E_k) r
    for (int k = 0; k < kk && e == hipSuccess; ++k) {
      // b_k = h~^b B_k into the scratch vector, then <A_k | b_k>.
      StepLaunch S;
      S.v = Bb + vec_b * (size_t)k; S.out = P->Y; S.write_out = 0; S.read_w = 0; S.dots = 0; S.a = 0.0; S.b = 0.0;
      S.velocity = true; S.vel = Sc; S.vdir = p->beta; S.vel_scale = 1.0;
      e = plan_launch_step(P, s, S);
      if (e != hipSuccess) break;
      double* pk = part + (size_t)(k0 + k) * kDotBlocks * 2;
      if (f32)
        hipLaunchKernelGGL(dot_partial_kernel<float>, dim3(kDotBlocks), dim3(256), 0, s,
                           (const float*)(Ab + vec_b * (size_t)k), (const float*)Sc, n_elems / 2, pk);
      else
        hipLaunchKernelGGL(dot_partial_kernel<double>, dim3(kDotBlocks), dim3(256), 0, s,
                           (const double*)(Ab + vec_b * (size_t)k), (const double*)Sc, n_elems / 2, pk);
      e = ::kpm::launch_status();
    }
  }
  if (e == hipSuccess && st == KPM_OK) {
    const double omega = (double)lat->L1 * lat->L2 * cell_area_nm2(lat->kind);
    double* out = on_dev ? sigma : dsig;
    hipLaunchKernelGGL(singleshot_finish_kernel, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, s, part, K,
                       2.0 * M_PI * M_PI / (omega * R), out);
    e = ::kpm::launch_status();
    if (e == hipSuccess && !on_dev) e = hipMemcpyAsync(sigma, dsig, sizeof(double) * K, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  } else {
    (void)hipStreamSynchronize(s);
  }
  if (e != hipSuccess && st == KPM_OK) {
    set_error("kpm_sigma_singleshot: %s", hipGetErrorString(e));
    st = (e == hipErrorOutOfMemory) ? KPM_E_NOMEM : KPM_E_DEVICE;
  }
  for (void* ptr : {V0, Sc, acc, hist, (void*)dcoef, (void*)part, (void*)dsig})
    if (ptr) (void)::kpm::dev_free(ptr);
  plan_free(P);
  delete P;
  return st;
}

}  // namespace kpm

extern "C" int kpm_sigma_singleshot(const kpm_lattice_t* lat, const kpm_cond_params_t* p, const double* energies_ev,
                                    int32_t K, double eta_ev, double* sigma, int32_t on_device, void* hip_stream) {
  try {
    kpm::clear_error();
    return kpm::singleshot_run(lat, p, energies_ev, K, eta_ev, sigma, on_device, hip_stream);
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_sigma_singleshot");
    return KPM_E_DEVICE;
  }
}

extern "C" int kpm_moments_gamma1(const kpm_lattice_t* lat, const kpm_cond_params_t* p, double* gamma1,
                                  int32_t out_on_device, void* hip_stream) {
  try {
    kpm::clear_error();
    return kpm::gamma1_run(lat, p, gamma1, out_on_device, hip_stream);
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_moments_gamma1");
    return KPM_E_DEVICE;
  }
}

extern "C" int kpm_cond_last_stats(kpm_cond_stats_t* out) {
  if (!out) {
    kpm::set_error("NULL argument");
    return KPM_E_INVALID;
  }
  *out = kpm::g_stats;
  return KPM_OK;
}

extern "C" int kpm_moments_cond(const kpm_lattice_t* lat, const kpm_cond_params_t* p, double* gamma,
                                int32_t out_on_device, void* hip_stream) {
  try {
    kpm::clear_error();
    return kpm::cond_run(lat, p, gamma, out_on_device, hip_stream);
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_moments_cond");
    return KPM_E_DEVICE;
  }
}
