// Wave-packet time evolution (the paper's spintronics example, Sec. 4).
//
// Propagator: the time-evolution operator exp(-i H dt / hbar) of the
// time-independent Hamiltonian, expanded in Chebyshev polynomials of the
// rescaled H~ = (H - de+)/de- (Tal-Ezer and Kosloff):
//   U(dt) = exp(-i de+ dt/hbar) sum_{n < M} (2 - d_n0) (-i)^n J_n(de- dt/hbar) T_n(H~).
// The paper prints the coefficient as (-1)^n J_n; the Jacobi-Anger expansion
// exp(-i x cos th) = J_0(x) + 2 sum (-i)^n J_n(x) cos(n th) gives (-i)^n, the
// only choice that makes the series unitary.
//
// One time step runs the M - 1 recursion steps T_{n+1} = 2 H~ T_n - T_{n-1} of
// the plan's single-step kernel from psi(t), writing T_n psi into slot n mod B
// of a history of B (<= 32) vectors; every B steps one pass folds the history
// into psi(t + dt) with the complex coefficients (per step about 1 + 2/B
// vectors of traffic besides the recursion's three, instead of three for a
// per-step update; 32 keeps the footprint at a third of what 64 would take for
// under 1 % more traffic).
//
// The Gaussian packet psi(0, r) = exp(-|r - r_c|^2/(2 sigma^2)) sum_j
// exp(i k_j.r) spinor_j (the printed exponent is garbled; sigma is read as the
// envelope's standard deviation) is built on the device, zero on vacant sites
// and normalised.  Observables per time point and packet: the norm, <x>, <y>,
// <x^2>, <y^2> (nm, nm^2) and <sigma_x,y,z> (hbar/2), divided by the norm;
// FP64 sums in a fixed order.
#include "kpm_geometry.h"
#include "kpm_internal.h"
#include "kpm_plan.h"

#include <cmath>
#include <complex>
#include <cstring>
#include <type_traits>
#include <vector>

namespace kpm {

// hbar in eV fs from the exact SI constants h and e.
constexpr double kHbarEvFs = 6.62607015e-34 / (2.0 * 3.14159265358979323846 * 1.602176634e-19) * 1e15;
constexpr int kEvoHist = 32;      // history vectors per flush
constexpr int kObsBlocks = 512;   // partial sums per packet in the observables reduction

static thread_local kpm_evolve_stats_t g_evo_stats;

struct CellGeom {
  double a1x, a1y, a2x, a2y;
  double tx[2], ty[2];   // sublattice offsets
  int L1, L2, n_sub, n_spin;
};

static CellGeom cell_geom(const kpm_lattice_t& L) {
  CellGeom g;
  g.L1 = L.L1;
  g.L2 = L.L2;
  g.tx[0] = g.tx[1] = g.ty[0] = g.ty[1] = 0.0;
  if (L.kind == KPM_SQUARE) {
    g.a1x = kASq; g.a1y = 0.0; g.a2x = 0.0; g.a2y = kASq;
    g.n_sub = 1;
    g.n_spin = 1;
  } else {
    g.a1x = kAHc; g.a1y = 0.0; g.a2x = 0.5 * kAHc; g.a2y = 0.5 * std::sqrt(3.0) * kAHc;
    g.ty[0] = -0.5 * kAccHc;
    g.ty[1] = 0.5 * kAccHc;
    g.n_sub = 2;
    g.n_spin = L.kind == KPM_HONEYCOMB_SPIN ? 2 : 1;
  }
  return g;
}

// Position (nm) of the site of orbital o = ((n2 L1 + n1) n_sub + s) n_spin + spin,
// and the orbital's component within its cell (s n_spin + spin).
__device__ inline void orbital_xy(const CellGeom& g, int64_t o, double& x, double& y, int& comp) {
  const int per = g.n_sub * g.n_spin;
  const int64_t cell = o / per;
  comp = (int)(o - cell * per);
  const int s = comp / g.n_spin;
  const int64_t n2 = cell / g.L1;
  const int64_t n1 = cell - n2 * g.L1;
  x = (double)n1 * g.a1x + (double)n2 * g.a2x + g.tx[s];
  y = (double)n1 * g.a1y + (double)n2 * g.a2y + g.ty[s];
}

__global__ void wavepacket_kernel(CellGeom g, int64_t n_orb, int n_k, const double* __restrict__ kv,
                                  const double* __restrict__ spin, double inv_2s2, double xc, double yc,
                                  const uint8_t* __restrict__ mask, double* __restrict__ psi) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_orb) return;
  double x, y;
  int comp;
  orbital_xy(g, o, x, y, comp);
  double re = 0.0, im = 0.0;
  if (!mask || mask[o / g.n_spin]) {
    const int per = g.n_sub * g.n_spin;
    const double env = exp(-((x - xc) * (x - xc) + (y - yc) * (y - yc)) * inv_2s2);
    for (int j = 0; j < n_k; ++j) {
      double sn, cs;
      sincos(kv[2 * j] * x + kv[2 * j + 1] * y, &sn, &cs);
      const double sr = spin[2 * (j * per + comp)], si = spin[2 * (j * per + comp) + 1];
      re += cs * sr - sn * si;
      im += cs * si + sn * sr;
    }
    re *= env;
    im *= env;
  }
  psi[2 * o] = re;
  psi[2 * o + 1] = im;
}

// part[b] = sum of |psi|^2 over a fixed slice (one workgroup per slice).
__global__ void evo_sumsq_kernel(const double* __restrict__ psi, int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void evo_sum_kernel(const double* part, int n, double* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < n; ++b) s += part[b];
    *out = s;
  }
}

__global__ void evo_scale_kernel(double* psi, int64_t n, double f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) psi[i] *= f;
}

// Plan layout [orbital][Rp] complex (T) <-> caller layout [R][n_orb] complex (FP64);
// the copy in zeroes vacant orbitals (the model has no such states).
template <typename T>
__global__ void evolve_copy_in_kernel(const double* __restrict__ src, int64_t n_orb, int R, int Rp, int n_spin,
                                      const uint8_t* __restrict__ mask, T* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_orb * Rp) return;
  const int64_t o = i / Rp;
  const int r = (int)(i - o * Rp);
  double re = 0.0, im = 0.0;
  if (r < R && (!mask || mask[o / n_spin])) {
    re = src[2 * ((int64_t)r * n_orb + o)];
    im = src[2 * ((int64_t)r * n_orb + o) + 1];
  }
  dst[2 * i] = (T)re;
  dst[2 * i + 1] = (T)im;
}

template <typename T>
__global__ void evolve_copy_out_kernel(const T* __restrict__ src, int64_t n_orb, int R, int Rp, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_orb * R) return;
  const int r = (int)(i / n_orb);
  const int64_t o = i - (int64_t)r * n_orb;
  dst[2 * i] = (double)src[2 * (o * Rp + r)];
  dst[2 * i + 1] = (double)src[2 * (o * Rp + r) + 1];
}

template <typename T>
struct EvoHist {
  const T* v[kEvoHist];
};

// acc[i] (=, first; += otherwise) sum_{b < nb} coef[b] v_b[i] over complex elements,
// the sum in FP64.
template <typename T>
__global__ void evolve_flush_kernel(EvoHist<T> H, int nb, int64_t n_cplx, const double2* __restrict__ coef, int first,
                                    T* __restrict__ acc) {
  using V2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_cplx; i += (int64_t)gridDim.x * blockDim.x) {
    double ar = 0.0, ai = 0.0;
#pragma unroll 4
    for (int b = 0; b < nb; ++b) {
      const V2 x = reinterpret_cast<const V2*>(H.v[b])[i];
      const double2 c = coef[b];
      ar += c.x * (double)x.x - c.y * (double)x.y;
      ai += c.x * (double)x.y + c.y * (double)x.x;
    }
    V2* a = reinterpret_cast<V2*>(acc) + i;
    if (!first) {
      const V2 o = *a;
      ar += (double)o.x;
      ai += (double)o.y;
    }
    V2 out;
    out.x = (T)ar;
    out.y = (T)ai;
    *a = out;
  }
}

// Per packet r = blockIdx.y: partial sums over a fixed slice of sites of
// |psi|^2 weighted by 1, x, y, x^2, y^2, and the spin numerators
// 2 Re(u* d), 2 Im(u* d), |u|^2 - |d|^2 (spinful lattices).
template <typename T>
__global__ void observables_partial_kernel(CellGeom g, const T* __restrict__ psi, int64_t n_sites, int Rp,
                                           double* __restrict__ part) {
  __shared__ double red[8][256];
  const int r = blockIdx.y;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  for (int64_t st = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; st < n_sites; st += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = st * g.n_spin;
    double x, y;
    int comp;
    orbital_xy(g, o, x, y, comp);
    const double ur = (double)psi[2 * (o * Rp + r)], ui = (double)psi[2 * (o * Rp + r) + 1];
    double p = ur * ur + ui * ui;
    if (g.n_spin == 2) {
      const double dr = (double)psi[2 * ((o + 1) * Rp + r)], di = (double)psi[2 * ((o + 1) * Rp + r) + 1];
      const double pd = dr * dr + di * di;
      acc[5] += 2.0 * (ur * dr + ui * di);   // u* d = (ur - i ui)(dr + i di)
      acc[6] += 2.0 * (ur * di - ui * dr);
      acc[7] += p - pd;
      p += pd;
    }
    acc[0] += p;
    acc[1] += p * x;
    acc[2] += p * y;
    acc[3] += p * x * x;
    acc[4] += p * y * y;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 8) part[((int64_t)r * gridDim.x + blockIdx.x) * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// out[r][q] for one time point: the sums over the slices in a fixed order, all but
// the norm divided by it.
__global__ void observables_finish_kernel(const double* __restrict__ part, int R, int n_blocks, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double s[8];
  for (int q = 0; q < 8; ++q) s[q] = 0.0;
  for (int b = 0; b < n_blocks; ++b)
    for (int q = 0; q < 8; ++q) s[q] += part[((int64_t)r * n_blocks + b) * 8 + q];
  out[(int64_t)r * 8] = s[0];
  for (int q = 1; q < 8; ++q) out[(int64_t)r * 8 + q] = s[0] > 0.0 ? s[q] / s[0] : 0.0;
}

// A plan over one lattice with the single-step ring kernel and R vectors (its
// model build gives the vacancy mask and the on-site terms).
static int evolve_plan(const kpm_lattice_t* lat, int R, int precision, hipStream_t s, kpm_plan** out) {
  kpm_dos_params_t dp;
  std::memset(&dp, 0, sizeof(dp));
  dp.num_moments = 2;
  dp.num_random = R;
  dp.vector_seed = 1;
  dp.precision = precision;
  dp.start = KPM_START_RANDOM_PHASE;
  kpm_tune_t tune;
  std::memset(&tune, 0, sizeof(tune));
  tune.kernel = 2;
  tune.use_graph = 0;
  kpm_plan* P = nullptr;
  KPM_TRY(plan_create(lat, 1, &dp, &tune, &P));
  const hipError_t e = plan_launch_prep(P, s);
  if (e != hipSuccess) {
    plan_free(P);
    delete P;
    set_error("model build: %s", hipGetErrorString(e));
    return ::kpm::hip_status(e);
  }
  *out = P;
  return KPM_OK;
}

static int wavepacket_run(const kpm_lattice_t* lat, int32_t n_k, const double* k_vectors, const double* spinors,
                          double width_nm, const double* center_cells, double* psi, int32_t on_dev, void* stream) {
  KPM_CHECK_ARG(lat && k_vectors && spinors && center_cells && psi, "NULL argument");
  KPM_CHECK_ARG(n_k >= 1 && n_k <= 4096, "need 1 <= n_k <= 4096");
  KPM_CHECK_ARG(width_nm > 0.0 && std::isfinite(width_nm), "width must be > 0");
  KPM_CHECK_ARG(std::isfinite(center_cells[0]) && std::isfinite(center_cells[1]), "centre must be finite");
  hipStream_t s = (hipStream_t)stream;
  const CellGeom g = cell_geom(*lat);
  const int per = g.n_sub * g.n_spin;
  for (int i = 0; i < 2 * n_k; ++i) KPM_CHECK_ARG(std::isfinite(k_vectors[i]), "k vectors must be finite");
  kpm_plan* P = nullptr;
  KPM_TRY(evolve_plan(lat, 1, KPM_FP64, s, &P));
  const int64_t n = P->n_orb;
  double *dk = nullptr, *dsp = nullptr, *part = nullptr, *dpsi = nullptr;
  hipError_t e = ::kpm::dev_malloc(&dk, sizeof(double) * 2 * n_k);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&dsp, sizeof(double) * 2 * (size_t)n_k * per);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&part, sizeof(double) * 1025);
  if (e == hipSuccess && !on_dev) e = ::kpm::dev_malloc(&dpsi, sizeof(double) * 2 * (size_t)n);
  if (e == hipSuccess) e = hipMemcpyAsync(dk, k_vectors, sizeof(double) * 2 * n_k, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dsp, spinors, sizeof(double) * 2 * (size_t)n_k * per, hipMemcpyHostToDevice, s);
  double* out = on_dev ? psi : dpsi;
  double norm = 0.0;
  if (e == hipSuccess) {
    const double xc = center_cells[0] * g.a1x + center_cells[1] * g.a2x;
    const double yc = center_cells[0] * g.a1y + center_cells[1] * g.a2y;
    hipLaunchKernelGGL(wavepacket_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, g, n, n_k, dk, dsp,
                       0.5 / (width_nm * width_nm), xc, yc, (const uint8_t*)P->mask, out);
    hipLaunchKernelGGL(evo_sumsq_kernel, dim3(1024), dim3(256), 0, s, out, n, part);
    hipLaunchKernelGGL(evo_sum_kernel, dim3(1), dim3(64), 0, s, part, 1024, part + 1024);
    e = ::kpm::launch_status();
    if (e == hipSuccess) e = hipMemcpyAsync(&norm, part + 1024, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  int st = KPM_OK;
  if (e == hipSuccess && !(norm > 0.0 && std::isfinite(norm))) {
    set_error("the wave packet has zero or non-finite norm on this lattice");
    st = KPM_E_INVALID;
  }
  if (e == hipSuccess && st == KPM_OK) {
    hipLaunchKernelGGL(evo_scale_kernel, dim3((unsigned)ceil_div(2 * n, 256)), dim3(256), 0, s, out, 2 * n,
                       1.0 / std::sqrt(norm));
    e = ::kpm::launch_status();
    if (e == hipSuccess && !on_dev) e = hipMemcpyAsync(psi, dpsi, sizeof(double) * 2 * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  } else {
    (void)hipStreamSynchronize(s);
  }
  if (e != hipSuccess) {
    set_error("kpm_wavepacket_gaussian: %s", hipGetErrorString(e));
    st = ::kpm::hip_status(e);
  }
  for (void* ptr : {(void*)dk, (void*)dsp, (void*)part, (void*)dpsi})
    if (ptr) (void)::kpm::dev_free(ptr);
  plan_free(P);
  delete P;
  return st;
}

template <typename T>
static hipError_t evolve_loop(kpm_plan* P, const kpm_evolve_params_t* p, const CellGeom& g, const double2* dcoef,
                              int B, void* hist, double* part, double* obs, hipStream_t s) {
  const int M = p->num_moments, R = p->num_packets;
  const int64_t n_cplx = P->n_orb * P->Rp;
  const size_t vec_b = (size_t)n_cplx * 2 * sizeof(T);
  const int64_t n_sites = P->n_orb / g.n_spin;
  const dim3 fg(2048), fb(256);
  void* psi = P->X;
  void* nxt = P->Y;
  auto observe = [&](int k) {
    hipLaunchKernelGGL(observables_partial_kernel<T>, dim3(kObsBlocks, R), dim3(256), 0, s, g, (const T*)psi, n_sites,
                       P->Rp, part);
    hipLaunchKernelGGL(observables_finish_kernel, dim3((unsigned)ceil_div(R, 64)), dim3(64), 0, s, part, R, kObsBlocks,
                       obs + (size_t)k * R * 8);
    return ::kpm::launch_status();
  };
  // T_n psi: psi itself for n = 0, history slot n mod B otherwise.
  auto hvec = [&](int n) -> void* { return n == 0 ? psi : (char*)hist + vec_b * (size_t)(n % B); };
  auto flush = [&](int n0, int nb, int first) {
    EvoHist<T> H;
    for (int b = 0; b < nb; ++b) H.v[b] = (const T*)hvec(n0 + b);
    hipLaunchKernelGGL(evolve_flush_kernel<T>, fg, fb, 0, s, H, nb, n_cplx, dcoef + n0, first, (T*)nxt);
    return ::kpm::launch_status();
  };
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipError_t e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  if (e == hipSuccess) e = hipEventRecord(ev0, s);
  if (e == hipSuccess) e = observe(0);
  // Algorithmic bytes: a recursion step reads v_n (neighbours from cache) and
  // v_(n-1), writes v_(n+1), reads the per-site arrays; a flush reads its
  // history vectors and writes psi(t + dt) (reading it too after the first).
  const double site_b = (double)n_sites * ((P->has_onsite ? (double)sizeof(T) : 0.0) + (P->has_mask ? 1.0 : 0.0));
  const int n_flush = (M + B - 1) / B;
  const double step_b = (double)(M - 1) * (3.0 * (double)vec_b + site_b) + ((double)M + 2.0 * n_flush - 1.0) * (double)vec_b;
  for (int k = 1; k < p->num_points && e == hipSuccess; ++k) {
    int n0 = 0, first = 1;
    for (int n = 1; n < M && e == hipSuccess; ++n) {
      StepLaunch S;
      S.dots = 0;
      S.v = hvec(n - 1);
      S.out = hvec(n);
      if (n == 1) {
        S.read_w = 0; S.a = 1.0; S.b = 0.0;
      } else {
        S.w = hvec(n - 2);
      }
      e = plan_launch_step(P, s, S);
      if (e == hipSuccess && n + 1 - n0 == B) {
        e = flush(n0, B, first);
        first = 0;
        n0 = n + 1;
      }
    }
    if (e == hipSuccess && n0 < M) e = flush(n0, M - n0, first);
    std::swap(psi, nxt);
    if (e == hipSuccess) e = observe(k);
  }
  if (e == hipSuccess) e = hipEventRecord(ev1, s);
  if (e == hipSuccess) e = hipEventSynchronize(ev1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  g_evo_stats.history = B;
  g_evo_stats.time_steps = p->num_points - 1;
  g_evo_stats.loop_ms = ms;
  g_evo_stats.bytes = step_b * (p->num_points - 1);
  // The final state ends in X (copied out by the caller).
  if (e == hipSuccess && psi != P->X) e = hipMemcpyAsync(P->X, psi, vec_b, hipMemcpyDeviceToDevice, s);
  return e;
}

static int evolve_run(const kpm_lattice_t* lat, const kpm_evolve_params_t* p, double* psi, double* observables,
                      int32_t on_dev, void* stream) {
  KPM_CHECK_ARG(lat && p && psi && observables, "NULL argument");
  KPM_CHECK_ARG(p->num_moments >= 2 && p->num_moments <= (1 << 20), "num_moments must be in [2, 2^20]");
  KPM_CHECK_ARG(p->num_points >= 1 && p->num_points <= (1 << 20), "num_points must be in [1, 2^20]");
  KPM_CHECK_ARG(p->num_packets >= 1 && p->num_packets <= 4096, "num_packets must be in [1, 4096]");
  KPM_CHECK_ARG(p->precision == KPM_FP32 || p->precision == KPM_FP64, "precision must be KPM_FP32 or KPM_FP64");
  KPM_CHECK_ARG(std::isfinite(p->dt_fs) && p->dt_fs != 0.0, "dt must be finite and nonzero");
  hipStream_t s = (hipStream_t)stream;
  std::memset(&g_evo_stats, 0, sizeof(g_evo_stats));
  const int M = p->num_moments, R = p->num_packets;
  // Coefficients phase (2 - d_n0) (-i)^n J_n(x), x = de- dt/hbar (J_n(-x) = (-1)^n J_n(x)).
  const double de_p = 0.5 * (lat->e_max + lat->e_min), de_m = 0.5 * (lat->e_max - lat->e_min);
  const double x = de_m * p->dt_fs / kHbarEvFs;
  typedef std::complex<double> cd;
  const cd phase = std::exp(cd(0.0, -de_p * p->dt_fs / kHbarEvFs));
  std::vector<double2> coef((size_t)M);
  cd mi(1.0, 0.0);
  for (int n = 0; n < M; ++n) {
    double j = std::cyl_bessel_j((double)n, std::fabs(x));
    if (x < 0.0 && (n & 1)) j = -j;
    const cd c = phase * mi * (n == 0 ? 1.0 : 2.0) * j;
    coef[(size_t)n] = make_double2(c.real(), c.imag());
    mi *= cd(0.0, -1.0);
  }
  kpm_plan* P = nullptr;
  KPM_TRY(evolve_plan(lat, R, p->precision, s, &P));
  const CellGeom g = cell_geom(*lat);
  const int64_t n_orb = P->n_orb;
  const size_t vec_b = (size_t)n_orb * P->Rp * 2 * P->tsize;
  size_t free_b = 0, total_b = 0;
  hipError_t e = hipMemGetInfo(&free_b, &total_b);
  // History: up to 32 vectors (no more than M), in the free memory.
  const double room = std::floor((0.85 * (double)free_b - 1.0e9) / (double)vec_b);
  const int B = (int)std::min<double>(std::min(kEvoHist, std::max(3, M)), room);
  if (e == hipSuccess && B < 3) {
    set_error("not enough device memory for the evolution history (3 vectors of %.1f GB)", vec_b / 1e9);
    plan_free(P);
    delete P;
    return KPM_E_NOMEM;
  }
  const size_t n_psi = (size_t)R * n_orb * 2, n_obs = (size_t)p->num_points * R * 8;
  void* hist = nullptr;
  double2* dcoef = nullptr;
  double *part = nullptr, *dpsi = nullptr, *dobs = nullptr;
  if (e == hipSuccess) e = ::kpm::dev_malloc(&hist, vec_b * (size_t)B);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&dcoef, sizeof(double2) * M);
  if (e == hipSuccess) e = ::kpm::dev_malloc(&part, sizeof(double) * 8 * (size_t)kObsBlocks * R);
  if (e == hipSuccess && !on_dev) e = ::kpm::dev_malloc(&dpsi, sizeof(double) * n_psi);
  if (e == hipSuccess && !on_dev) e = ::kpm::dev_malloc(&dobs, sizeof(double) * n_obs);
  if (e == hipSuccess) e = hipMemcpyAsync(dcoef, coef.data(), sizeof(double2) * M, hipMemcpyHostToDevice, s);
  double* sp = on_dev ? psi : dpsi;
  double* so = on_dev ? observables : dobs;
  if (e == hipSuccess && !on_dev) e = hipMemcpyAsync(dpsi, psi, sizeof(double) * n_psi, hipMemcpyHostToDevice, s);
  const bool f32 = P->prec == KPM_FP32;
  if (e == hipSuccess) {
    const unsigned gi = (unsigned)ceil_div(n_orb * P->Rp, 256), go = (unsigned)ceil_div(n_orb * R, 256);
    if (f32) {
      hipLaunchKernelGGL(evolve_copy_in_kernel<float>, dim3(gi), dim3(256), 0, s, sp, n_orb, R, P->Rp, g.n_spin,
                         (const uint8_t*)P->mask, (float*)P->X);
      e = ::kpm::launch_status();
      if (e == hipSuccess) e = evolve_loop<float>(P, p, g, dcoef, B, hist, part, so, s);
      if (e == hipSuccess)
        hipLaunchKernelGGL(evolve_copy_out_kernel<float>, dim3(go), dim3(256), 0, s, (const float*)P->X, n_orb, R,
                           P->Rp, sp);
    } else {
      hipLaunchKernelGGL(evolve_copy_in_kernel<double>, dim3(gi), dim3(256), 0, s, sp, n_orb, R, P->Rp, g.n_spin,
                         (const uint8_t*)P->mask, (double*)P->X);
      e = ::kpm::launch_status();
      if (e == hipSuccess) e = evolve_loop<double>(P, p, g, dcoef, B, hist, part, so, s);
      if (e == hipSuccess)
        hipLaunchKernelGGL(evolve_copy_out_kernel<double>, dim3(go), dim3(256), 0, s, (const double*)P->X, n_orb, R,
                           P->Rp, sp);
    }
    if (e == hipSuccess) e = ::kpm::launch_status();
  }
  if (e == hipSuccess && !on_dev) e = hipMemcpyAsync(psi, dpsi, sizeof(double) * n_psi, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && !on_dev) e = hipMemcpyAsync(observables, dobs, sizeof(double) * n_obs, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  else (void)hipStreamSynchronize(s);
  int st = KPM_OK;
  if (e != hipSuccess) {
    set_error("kpm_time_evolve: %s", hipGetErrorString(e));
    st = (e == hipErrorOutOfMemory) ? KPM_E_NOMEM : KPM_E_DEVICE;
  }
  for (void* ptr : {hist, (void*)dcoef, (void*)part, (void*)dpsi, (void*)dobs})
    if (ptr) (void)::kpm::dev_free(ptr);
  plan_free(P);
  delete P;
  return st;
}

}  // namespace kpm

extern "C" int kpm_wavepacket_gaussian(const kpm_lattice_t* lat, int32_t n_k, const double* k_vectors,
                                       const double* spinors, double width_nm, const double* center_cells, double* psi,
                                       int32_t on_device, void* hip_stream) {
  try {
    kpm::clear_error();
    return kpm::wavepacket_run(lat, n_k, k_vectors, spinors, width_nm, center_cells, psi, on_device, hip_stream);
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_wavepacket_gaussian");
    return KPM_E_DEVICE;
  }
}

extern "C" int kpm_evolve_last_stats(kpm_evolve_stats_t* stats) {
  if (!stats) return KPM_E_INVALID;
  *stats = kpm::g_evo_stats;
  return KPM_OK;
}

extern "C" int kpm_time_evolve(const kpm_lattice_t* lat, const kpm_evolve_params_t* p, double* psi,
                               double* observables, int32_t on_device, void* hip_stream) {
  try {
    kpm::clear_error();
    return kpm::evolve_run(lat, p, psi, observables, on_device, hip_stream);
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_time_evolve");
    return KPM_E_DEVICE;
  }
}
