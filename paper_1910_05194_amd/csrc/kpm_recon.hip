// DOS reconstructions from Chebyshev moments, FP64 throughout.
//
// KPM (paper eqs. e7 and delta_function_cheb_expansion) with a damping kernel:
//   rho(E) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(eps)] / (pi sqrt(1 - eps^2) de-),
// g_n the Jackson kernel (Weisse et al. 2006, which the paper cites) or the
// Lorentz kernel the paper prints (Sec. 2(a)).  One workgroup stages
// c_n = g_n mu_n (x2 for n >= 1) in LDS in chunks; each thread owns one energy
// and runs the scalar Chebyshev recursion in eps.
//
// CPGF (eqs. green_function_cheb_expansion(b)): the retarded resolvent
//   (1/N) Tr 1/(E - H + i eta) = (1/de-) sum_n g_n(z) mu_n / (1 + delta_n0),
//   g_n(z) = -2 i w^n / sqrt(1 - z^2),  z = eps + i eta/de-,  w = exp(-i arccos z).
// w is the root of w^2 - 2 z w + 1 = 0 inside the unit circle (taken as the
// reciprocal of the outer root, which has no cancellation), and with that
// branch sqrt(1 - z^2) = i (w - z), so g_n = -2 w^n / (w - z).

#include "kpm_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace kpm {

enum { kKernelJackson = 0, kKernelLorentz = 1 };

__device__ inline double damping(int kernel, int n, int M, double lam) {
  if (kernel == kKernelLorentz) return sinh(lam * (1.0 - (double)n / M)) / sinh(lam);
  const double q = M_PI / (M + 1);
  return ((M - n + 1) * cos(q * n) + sin(q * n) / tan(q)) / (M + 1);
}

__global__ void kernel_dos_kernel(const double* mu, int M, const double* energies, int K, double e_min,
                                  double e_max, int kernel, double lam, double* rho) {
  __shared__ double coef[1024];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const double de_p = 0.5 * (e_max + e_min), de_m = 0.5 * (e_max - e_min);
  const double eps = (k < K) ? (energies[k] - de_p) / de_m : 0.0;
  const bool inside = (k < K) && fabs(eps) < 1.0;
  double tm1 = 1.0, t0 = eps, acc = 0.0;   // T_{n-1}, T_n as the recursion advances
  for (int base = 0; base < M; base += 1024) {
    __syncthreads();
    for (int i = threadIdx.x; i < 1024 && base + i < M; i += blockDim.x) {
      const int n = base + i;
      coef[i] = (n == 0 ? 1.0 : 2.0) * damping(kernel, n, M, lam) * mu[n];
    }
    __syncthreads();
    const int cnt = min(1024, M - base);
    for (int i = 0; i < cnt; ++i) {
      const int n = base + i;
      double tn;
      if (n == 0) tn = 1.0;
      else if (n == 1) tn = eps;
      else {
        tn = 2.0 * eps * t0 - tm1;
        tm1 = t0;
        t0 = tn;
      }
      acc += coef[i] * tn;
    }
  }
  if (k < K) rho[k] = inside ? acc / (M_PI * sqrt(1.0 - eps * eps) * de_m) : 0.0;
}

struct cplx {
  double re, im;
};
__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm (scaled by the larger component of b).
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
// Principal square root.
__device__ inline cplx csqrt_p(cplx z) {
  const double m = hypot(z.re, z.im);
  if (m == 0.0) return {0.0, 0.0};
  if (z.re >= 0.0) {
    const double p = sqrt(0.5 * (m + z.re));
    return {p, z.im / (2.0 * p)};
  }
  const double q = copysign(sqrt(0.5 * (m - z.re)), z.im);
  return {z.im / (2.0 * q), q};
}

__global__ void cpgf_kernel(const double* mu, int M, const double* energies, int K, double e_min, double e_max,
                            double eta_ev, double* rho, double* green) {
  __shared__ double cm[1024];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const double de_p = 0.5 * (e_max + e_min), de_m = 0.5 * (e_max - e_min);
  const cplx z = {(k < K) ? (energies[k] - de_p) / de_m : 0.0, eta_ev / de_m};
  // Roots of w^2 - 2 z w + 1: z +- sqrt(z^2 - 1); the outer one has |.| > 1.
  const cplx s = csqrt_p({z.re * z.re - z.im * z.im - 1.0, 2.0 * z.re * z.im});
  const cplx wp = {z.re + s.re, z.im + s.im}, wm = {z.re - s.re, z.im - s.im};
  const cplx outer = (hypot(wp.re, wp.im) >= hypot(wm.re, wm.im)) ? wp : wm;
  const cplx w = cdiv({1.0, 0.0}, outer);
  cplx pw = {1.0, 0.0};   // w^n
  cplx acc = {0.0, 0.0};  // sum_n mu_n w^n / (1 + delta_n0)
  for (int base = 0; base < M; base += 1024) {
    __syncthreads();
    for (int i = threadIdx.x; i < 1024 && base + i < M; i += blockDim.x) {
      const int n = base + i;
      cm[i] = (n == 0 ? 0.5 : 1.0) * mu[n];
    }
    __syncthreads();
    const int cnt = min(1024, M - base);
    for (int i = 0; i < cnt; ++i) {
      acc.re += cm[i] * pw.re;
      acc.im += cm[i] * pw.im;
      pw = cmul(pw, w);
    }
  }
  // G = -2 acc / ((w - z) de-).
  const cplx g = cdiv({-2.0 * acc.re / de_m, -2.0 * acc.im / de_m}, {w.re - z.re, w.im - z.im});
  if (k < K) {
    rho[k] = -g.im / M_PI;
    if (green) {
      green[2 * k] = g.re;
      green[2 * k + 1] = g.im;
    }
  }
}

// T=0 longitudinal conductivity from Gamma (Kubo-Greenwood limit of the
// first-order formula, with eq. delta_function_cheb_expansion for both deltas):
//   sigma(E) = -2 pi^2 (N/Omega) / de-^2  sum_nm g_n g_m D_n(eps) D_m(eps) Re Gamma_nm   [e^2/h],
//   D_n(eps) = 2 T_n(eps) / (pi sqrt(1 - eps^2)).
// One workgroup per energy; w_n = g_n D_n(eps) staged in LDS.
__global__ void sigma_kernel(const double* gamma, int M, const double* energies, int K, double e_min, double e_max,
                             double density, double* sigma) {
  extern __shared__ double w[];
  __shared__ double red[256];
  const int k = blockIdx.x;
  const double de_p = 0.5 * (e_max + e_min), de_m = 0.5 * (e_max - e_min);
  const double eps = (energies[k] - de_p) / de_m;
  if (!(fabs(eps) < 1.0)) {
    if (threadIdx.x == 0) sigma[k] = 0.0;
    return;
  }
  const double th = acos(eps);
  const double pref = 2.0 / (M_PI * sqrt(1.0 - eps * eps));
  for (int n = threadIdx.x; n < M; n += blockDim.x) w[n] = damping(kKernelJackson, n, M, 0.0) * pref * cos(n * th);
  __syncthreads();
  double acc = 0.0;
  for (int n = threadIdx.x; n < M; n += blockDim.x) {
    const double* row = gamma + (int64_t)n * M * 2;
    double rs = 0.0;
    for (int m = 0; m < M; ++m) rs += row[2 * m] * w[m];
    acc += w[n] * rs;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[k] = -2.0 * M_PI * M_PI * density / (de_m * de_m) * red[0];
}

}  // namespace kpm

extern "C" int kpm_reconstruct_sigma(const double* gamma, int32_t M, const double* energies_ev, int32_t K,
                                     double e_min, double e_max, double orbitals_per_nm2, double* sigma,
                                     int32_t on_device, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(gamma && energies_ev && sigma, "NULL argument");
  KPM_CHECK_ARG(M >= 1 && M <= 8192 && K >= 1, "need 1 <= M <= 8192 and K >= 1");
  KPM_CHECK_ARG(std::isfinite(e_min) && std::isfinite(e_max) && e_min < e_max, "need e_min < e_max");
  KPM_CHECK_ARG(orbitals_per_nm2 > 0.0, "orbitals_per_nm2 must be > 0");
  hipStream_t s = (hipStream_t)hip_stream;
  const double* dg = gamma;
  const double* den = energies_ev;
  double* dsig = sigma;
  double* tmp = nullptr;
  const size_t gn = (size_t)M * M * 2;
  hipError_t e = hipSuccess;
  if (!on_device) {
    e = ::kpm::dev_malloc(&tmp, sizeof(double) * (gn + 2 * (size_t)K));
    if (e == hipSuccess) e = KPM_HIP(hipMemcpyAsync(tmp, gamma, sizeof(double) * gn, hipMemcpyHostToDevice, s));
    if (e == hipSuccess)
      e = KPM_HIP(hipMemcpyAsync(tmp + gn, energies_ev, sizeof(double) * K, hipMemcpyHostToDevice, s));
    dg = tmp;
    den = tmp + gn;
    dsig = tmp + gn + K;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(sigma_kernel, dim3(K), dim3(256), sizeof(double) * M, s, dg, M, den, K, e_min, e_max,
                       orbitals_per_nm2, dsig);
    e = ::kpm::launch_status();
  }
  if (e == hipSuccess && !on_device) {
    e = hipMemcpyAsync(sigma, dsig, sizeof(double) * K, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (tmp) (void)::kpm::dev_free(tmp);
  if (e != hipSuccess) {
    set_error("kpm_reconstruct_sigma: %s", hipGetErrorString(e));
    return ::kpm::hip_status(e);
  }
  return KPM_OK;
}

namespace kpm {
// Shared driver: stages host inputs, launches one of the DOS kernels, copies
// the outputs back.  green (CPGF only) may be NULL.
static int reconstruct(const char* name, int which, const double* mu, int32_t M, const double* energies_ev,
                       int32_t K, double e_min, double e_max, double param, double* rho, double* green,
                       int32_t on_device, void* hip_stream) {
  KPM_CHECK_ARG(mu && energies_ev && rho, "NULL argument");
  KPM_CHECK_ARG(M >= 1 && K >= 1, "need M >= 1 and K >= 1");
  KPM_CHECK_ARG(std::isfinite(e_min) && std::isfinite(e_max) && e_min < e_max, "need e_min < e_max");
  hipStream_t s = (hipStream_t)hip_stream;
  const double* dmu = mu;
  const double* den = energies_ev;
  double* drho = rho;
  double* dg = green;
  double* tmp = nullptr;
  hipError_t e = hipSuccess;
  if (!on_device) {
    e = ::kpm::dev_malloc(&tmp, sizeof(double) * ((size_t)M + 4 * (size_t)K));
    if (e == hipSuccess) e = KPM_HIP(hipMemcpyAsync(tmp, mu, sizeof(double) * M, hipMemcpyHostToDevice, s));
    if (e == hipSuccess)
      e = KPM_HIP(hipMemcpyAsync(tmp + M, energies_ev, sizeof(double) * K, hipMemcpyHostToDevice, s));
    dmu = tmp;
    den = tmp + M;
    drho = tmp + M + K;
    dg = green ? tmp + M + 2 * (size_t)K : nullptr;
  }
  if (e == hipSuccess) {
    const dim3 grid((unsigned)ceil_div(K, 256)), block(256);
    if (which == 2)
      hipLaunchKernelGGL(cpgf_kernel, grid, block, 0, s, dmu, M, den, K, e_min, e_max, param, drho, dg);
    else
      hipLaunchKernelGGL(kernel_dos_kernel, grid, block, 0, s, dmu, M, den, K, e_min, e_max, which, param, drho);
    e = ::kpm::launch_status();
  }
  if (e == hipSuccess && !on_device) {
    e = hipMemcpyAsync(rho, drho, sizeof(double) * K, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && green) e = hipMemcpyAsync(green, dg, sizeof(double) * 2 * K, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (tmp) (void)::kpm::dev_free(tmp);
  if (e != hipSuccess) {
    set_error("%s: %s", name, hipGetErrorString(e));
    return ::kpm::hip_status(e);
  }
  return KPM_OK;
}
}  // namespace kpm

namespace kpm {
__global__ void kernel_factors_kernel(int kernel, int M, double lam, int n0, int count, double* g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) g[i] = damping(kernel, n0 + i, M, lam);
}
}  // namespace kpm

extern "C" int kpm_kernel_factors(int32_t kernel, int32_t M, double lambda, int32_t n0, int32_t count, double* g,
                                  int32_t on_device, void* hip_stream) {
  kpm::clear_error();
  KPM_CHECK_ARG(kernel == kpm::kKernelJackson || kernel == kpm::kKernelLorentz, "kernel must be 0 (Jackson) or 1 (Lorentz)");
  KPM_CHECK_ARG(M >= 1 && n0 >= 0 && count >= 1 && (int64_t)n0 + count <= M, "need 0 <= n0 < n0 + count <= M");
  KPM_CHECK_ARG(kernel == kpm::kKernelJackson || (std::isfinite(lambda) && lambda > 0.0), "lambda must be > 0");
  KPM_CHECK_ARG(g != nullptr, "NULL argument");
  hipStream_t s = (hipStream_t)hip_stream;
  double* dg = g;
  if (!on_device) KPM_TRY_HIP(::kpm::dev_malloc(&dg, sizeof(double) * (size_t)count));
  hipLaunchKernelGGL(kpm::kernel_factors_kernel, dim3((unsigned)kpm::ceil_div(count, 256)), dim3(256), 0, s, kernel, M,
                     lambda, n0, count, dg);
  hipError_t e = ::kpm::launch_status();
  if (e == hipSuccess && !on_device) {
    e = hipMemcpyAsync(g, dg, sizeof(double) * (size_t)count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (!on_device) (void)::kpm::dev_free(dg);
  if (e != hipSuccess) {
    kpm::set_error("kpm_kernel_factors: %s", hipGetErrorString(e));
    return ::kpm::hip_status(e);
  }
  return KPM_OK;
}

extern "C" int kpm_reconstruct_jackson(const double* mu, int32_t M, const double* energies_ev, int32_t K,
                                       double e_min, double e_max, double* rho, int32_t on_device,
                                       void* hip_stream) {
  kpm::clear_error();
  return kpm::reconstruct("kpm_reconstruct_jackson", kpm::kKernelJackson, mu, M, energies_ev, K, e_min, e_max, 0.0,
                          rho, nullptr, on_device, hip_stream);
}

extern "C" int kpm_reconstruct_lorentz(const double* mu, int32_t M, const double* energies_ev, int32_t K,
                                       double e_min, double e_max, double lambda, double* rho, int32_t on_device,
                                       void* hip_stream) {
  kpm::clear_error();
  if (!(std::isfinite(lambda) && lambda > 0.0)) {
    kpm::set_error("kpm_reconstruct_lorentz: need lambda > 0");
    return KPM_E_INVALID;
  }
  return kpm::reconstruct("kpm_reconstruct_lorentz", kpm::kKernelLorentz, mu, M, energies_ev, K, e_min, e_max, lambda,
                          rho, nullptr, on_device, hip_stream);
}

extern "C" int kpm_reconstruct_cpgf(const double* mu, int32_t M, const double* energies_ev, int32_t K, double e_min,
                                    double e_max, double eta_ev, double* rho, double* green, int32_t on_device,
                                    void* hip_stream) {
  kpm::clear_error();
  if (!(std::isfinite(eta_ev) && eta_ev > 0.0)) {
    kpm::set_error("kpm_reconstruct_cpgf: need eta > 0");
    return KPM_E_INVALID;
  }
  return kpm::reconstruct("kpm_reconstruct_cpgf", 2, mu, M, energies_ev, K, e_min, e_max, eta_ev, rho, green,
                          on_device, hip_stream);
}

namespace kpm {

// ---------------------------------------------------------------------------
// Kubo-Bastin conductivity from Gamma^{ab} (the static limit of the
// first-order formula, eq. cond 1st order, written with eq.
// delta_function_cheb_expansion for the delta function and the CPGF
// coefficients of eqs. green_function_cheb_expansion(b) for the resolvents,
// contracted with Gamma as in eq. conductivity_1st_order):
//   sigma_ab(mu) = Re{ -2 pi i (N/Omega)/de-^2 int_{-1}^{1} d eps f(eps)
//                  sum_nm Gamma_nm [Delta_n(eps) g'^R_m(eps) - g'^A_n(eps) Delta_m(eps)] }  [e^2/h],
// f the Fermi function at chemical potential mu and temperature T.
// With eps = cos(theta), Delta_n d eps = (2/pi) cos(n theta) d theta, so the
// integrand in theta is F(theta) = sum_n D_n(theta) W_n(theta),
//   D_n = (2/pi) cos(n theta),   W_n = sum_m (g'^R_m Gamma_nm - g'^A_m Gamma_mn),
// and g'^A = conj(g'^R) for real eps.  The retarded derivative, with
// z = eps + i eta~, w = exp(-i arccos z) (the inner root, as above) and
// s = sqrt(1 - z^2) = i (w - z):
//   g'^R_n = -2 i w^n (i n / s^2 + z / s^3).
// theta runs over Q equal cells of [0, pi]: the integrand apart from f at each
// cell's midpoint, times the cell's occupation weight int_cell f(cos theta)
// d theta (occ_weight).
// Kernels: the g'^R and -g'^A tables [Q][Mp]; the contraction on 64 x 64
// (q, n) tiles with FP64 partial sums per n tile; one workgroup per Fermi
// energy for the weighted sum, all in a fixed order (deterministic).
// ---------------------------------------------------------------------------
constexpr int kBT = 64;   // q and n tile
constexpr int kBK = 8;    // m chunk

// Table of CPGF coefficients at z_q = cos(theta_q) + shift + i eta (retarded
// branch), for n < M (zero for M <= n < Mp): deriv = 0 gives g_n = -2 w^n/(w - z),
// deriv = 1 gives d g_n/d eps; xform 0 stores the value, 1 its conjugate (the
// advanced coefficient at the conjugate point), 2 minus its conjugate.
__global__ void cpgf_table_kernel(int Q, int M, int Mp, double shift, double eta, int deriv, int xform,
                                  double2* out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  const double th = (q + 0.5) * M_PI / Q;
  const cplx z = {cos(th) + shift, eta};
  const cplx r = csqrt_p({z.re * z.re - z.im * z.im - 1.0, 2.0 * z.re * z.im});
  const cplx wp = {z.re + r.re, z.im + r.im}, wm = {z.re - r.re, z.im - r.im};
  const cplx outer = (hypot(wp.re, wp.im) >= hypot(wm.re, wm.im)) ? wp : wm;
  const cplx w = cdiv({1.0, 0.0}, outer);
  const cplx s = {-(w.im - z.im), w.re - z.re};            // i (w - z) = sqrt(1 - z^2)
  const cplx s2 = cmul(s, s);
  const cplx inv_s2 = cdiv({1.0, 0.0}, s2);
  const cplx zs3 = cdiv(z, cmul(s2, s));
  const cplx m2_wz = cdiv({-2.0, 0.0}, {w.re - z.re, w.im - z.im});   // -2/(w - z)
  cplx pw = {1.0, 0.0};
  double2* row = out + (int64_t)q * Mp;
  for (int n = 0; n < Mp; ++n) {
    if (n < M) {
      cplx v;
      if (deriv) {
        // -2 i w^n (i n / s^2 + z / s^3)
        const cplx c = cmul(pw, {-n * inv_s2.im + zs3.re, n * inv_s2.re + zs3.im});
        v = {2.0 * c.im, -2.0 * c.re};
      } else {
        v = cmul(pw, m2_wz);
      }
      if (xform == 1) v.im = -v.im;
      if (xform == 2) v.re = -v.re;
      row[n] = make_double2(v.re, v.im);
      pw = cmul(pw, w);
    } else {
      row[n] = make_double2(0.0, 0.0);
    }
  }
}

// gam: Gamma padded to [Mp][Mp] complex.  W_n(theta_q) = sum_m (ta[q][m] Gamma_nm + tb[q][m] Gamma_mn);
// part[nt][q] = sum_{n in tile nt} D_n(theta_q) W_n(theta_q).
__global__ void __launch_bounds__(256) bastin_contract_kernel(const double2* __restrict__ ta,
                                                              const double2* __restrict__ tb,
                                                              const double2* __restrict__ gam, int Q, int Mp,
                                                              double2* __restrict__ part) {
  __shared__ double2 sa[kBT][kBK + 1];    // ta[q][m]
  __shared__ double2 sb[kBT][kBK + 1];    // tb[q][m]
  __shared__ double2 sr[kBT][kBK + 1];    // Gamma[n][m]
  __shared__ double2 sc[kBK][kBT + 1];    // Gamma[m][n]
  __shared__ double2 red[16][kBT + 1];
  const int tq = threadIdx.x / 16, tn = threadIdx.x % 16;   // 16 x 16 threads, 4 x 4 outputs each
  const int q0 = blockIdx.x * kBT, n0 = blockIdx.y * kBT;
  cplx acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = {0.0, 0.0};
  for (int m0 = 0; m0 < Mp; m0 += kBK) {
    __syncthreads();
    for (int e = threadIdx.x; e < kBT * kBK; e += 256) {
      const int a = e / kBK, b = e % kBK;
      const int q = q0 + a;
      sa[a][b] = (q < Q) ? ta[(int64_t)q * Mp + m0 + b] : make_double2(0.0, 0.0);
      sb[a][b] = (q < Q) ? tb[(int64_t)q * Mp + m0 + b] : make_double2(0.0, 0.0);
      sr[a][b] = gam[(int64_t)(n0 + a) * Mp + m0 + b];
    }
    for (int e = threadIdx.x; e < kBT * kBK; e += 256) {
      const int b = e / kBT, a = e % kBT;
      sc[b][a] = gam[(int64_t)(m0 + b) * Mp + n0 + a];
    }
    __syncthreads();
#pragma unroll 2
    for (int k = 0; k < kBK; ++k) {
      cplx ga[4], gb[4], r[4], c[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double2 va = sa[tq * 4 + i][k], vb = sb[tq * 4 + i][k];
        ga[i] = {va.x, va.y};
        gb[i] = {vb.x, vb.y};
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 x = sr[tn * 4 + j][k], y = sc[k][tn * 4 + j];
        r[j] = {x.x, x.y};
        c[j] = {y.x, y.y};
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j].re += ga[i].re * r[j].re - ga[i].im * r[j].im + gb[i].re * c[j].re - gb[i].im * c[j].im;
          acc[i][j].im += ga[i].re * r[j].im + ga[i].im * r[j].re + gb[i].re * c[j].im + gb[i].im * c[j].re;
        }
    }
  }
  // Weight by D_n(theta_q) and sum this thread's four n; then over the 16 n-threads.
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = q0 + tq * 4 + i;
    const double th = (q + 0.5) * M_PI / Q;
    cplx t = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double d = 2.0 / M_PI * cos((double)(n0 + tn * 4 + j) * th);
      t.re += d * acc[i][j].re;
      t.im += d * acc[i][j].im;
    }
    red[tn][tq * 4 + i] = make_double2(t.re, t.im);
  }
  __syncthreads();
  if (threadIdx.x < kBT) {
    const int a = threadIdx.x;
    double sre = 0.0, sim = 0.0;
    for (int j = 0; j < 16; ++j) {
      sre += red[j][a].x;
      sim += red[j][a].y;
    }
    const int q = q0 + a;
    if (q < Q) part[(int64_t)blockIdx.y * Q + q] = make_double2(sre, sim);
  }
}

// Occupation weight of theta-cell q of Q: int_cell f(cos theta) d theta, f the
// Fermi function 1/(1 + exp((eps - mu~)/kT~)) in rescaled energies.  kT~ = 0:
// the length of the cell inside [theta_mu, pi] (theta_mu = arccos mu~, 0 or pi
// outside the spectrum); kT~ > 0: midpoint sum over kFermiSub equal sub-cells.
constexpr int kFermiSub = 32;

__device__ inline double occ_weight(int q, int Q, double mut, double kTt) {
  const double h = M_PI / Q;
  const double lo = q * h;
  if (kTt == 0.0) {
    const double th_mu = (mut >= 1.0) ? 0.0 : (mut <= -1.0 ? M_PI : acos(mut));
    return fmin(fmax(lo + h - fmax(lo, th_mu), 0.0), h);
  }
  const double hs = h / kFermiSub;
  double acc = 0.0;
  for (int j = 0; j < kFermiSub; ++j) {
    const double x = (cos(lo + (j + 0.5) * hs) - mut) / kTt;
    const double ex = exp(-fabs(x));   // no overflow on either side of mu
    acc += (x > 0.0) ? ex / (1.0 + ex) : 1.0 / (1.0 + ex);
  }
  return acc * hs;
}

__global__ void bastin_sigma_kernel(const double2* part, int n_tiles, int Q, const double* energies, int K,
                                    double e_min, double e_max, double kTt, double pref_im, double* sigma) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const double de_p = 0.5 * (e_max + e_min), de_m = 0.5 * (e_max - e_min);
  const double mut = (energies[k] - de_p) / de_m;
  double acc = 0.0;   // Im of sum_q F_q w_q (pref is purely imaginary: Re(pref F) = -pref_im Im F)
  for (int q = threadIdx.x; q < Q; q += blockDim.x) {
    const double wq = occ_weight(q, Q, mut, kTt);
    if (wq > 0.0) {
      double fi = 0.0;
      for (int t = 0; t < n_tiles; ++t) fi += part[(int64_t)t * Q + q].y;
      acc += fi * wq;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma[k] = -pref_im * red[0];
}

__global__ void pad_gamma_kernel(const double* gamma, int M, int Mp, double2* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)Mp * Mp) return;
  const int n = (int)(i / Mp), m = (int)(i % Mp);
  out[i] = (n < M && m < M) ? make_double2(gamma[2 * ((int64_t)n * M + m)], gamma[2 * ((int64_t)n * M + m) + 1])
                            : make_double2(0.0, 0.0);
}

}  // namespace kpm

extern "C" int kpm_reconstruct_sigma_bastin(const double* gamma, int32_t M, const double* energies_ev, int32_t K,
                                            double e_min, double e_max, double eta_ev, double kT_ev,
                                            double orbitals_per_nm2, int32_t n_theta, double* sigma,
                                            int32_t on_device, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(gamma && energies_ev && sigma, "NULL argument");
  KPM_CHECK_ARG(M >= 1 && M <= 16384 && K >= 1, "need 1 <= M <= 16384 and K >= 1");
  KPM_CHECK_ARG(std::isfinite(e_min) && std::isfinite(e_max) && e_min < e_max, "need e_min < e_max");
  KPM_CHECK_ARG(eta_ev > 0.0 && std::isfinite(eta_ev), "eta must be > 0");
  KPM_CHECK_ARG(kT_ev >= 0.0 && std::isfinite(kT_ev), "kT must be >= 0");
  KPM_CHECK_ARG(orbitals_per_nm2 > 0.0, "orbitals_per_nm2 must be > 0");
  KPM_CHECK_ARG(n_theta >= 0 && n_theta <= (1 << 20), "n_theta must be in [0, 2^20]");
  const int Q = n_theta > 0 ? n_theta : 4 * M;
  const int Mp = (int)ceil_div(M, kBT) * kBT;
  const int Qp = (int)ceil_div(Q, kBT) * kBT;
  const int n_tiles = Mp / kBT;
  hipStream_t s = (hipStream_t)hip_stream;
  const double de_m = 0.5 * (e_max - e_min);
  // Workspace: padded Gamma, the g'^R table, the partial sums, and staged host data.
  const size_t b_gam = sizeof(double2) * (size_t)Mp * Mp;
  const size_t b_tab = 2 * sizeof(double2) * (size_t)Qp * Mp;
  const size_t b_part = sizeof(double2) * (size_t)n_tiles * Q;
  const size_t gn = (size_t)M * M * 2;
  const size_t b_host = on_device ? 0 : sizeof(double) * (gn + 2 * (size_t)K);
  char* ws = nullptr;
  KPM_TRY_HIP(::kpm::dev_malloc(&ws, b_gam + b_tab + b_part + b_host));
  double2* gam = (double2*)ws;
  double2* tab = (double2*)(ws + b_gam);
  double2* part = (double2*)(ws + b_gam + b_tab);
  const double* dg = gamma;
  const double* den = energies_ev;
  double* dsig = sigma;
  hipError_t e = hipSuccess;
  if (!on_device) {
    double* h = (double*)(ws + b_gam + b_tab + b_part);
    e = hipMemcpyAsync(h, gamma, sizeof(double) * gn, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + gn, energies_ev, sizeof(double) * K, hipMemcpyHostToDevice, s);
    dg = h;
    den = h + gn;
    dsig = h + gn + K;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(pad_gamma_kernel, dim3((unsigned)ceil_div((int64_t)Mp * Mp, 256)), dim3(256), 0, s, dg, M, Mp,
                       gam);
    // Table rows q >= Q stay unused (the contraction zero-fills them).  ta = g'^R,
    // tb = -g'^A = -conj(g'^R).
    hipLaunchKernelGGL(cpgf_table_kernel, dim3((unsigned)ceil_div(Q, 256)), dim3(256), 0, s, Q, M, Mp, 0.0,
                       eta_ev / de_m, 1, 0, tab);
    hipLaunchKernelGGL(cpgf_table_kernel, dim3((unsigned)ceil_div(Q, 256)), dim3(256), 0, s, Q, M, Mp, 0.0,
                       eta_ev / de_m, 1, 2, tab + (size_t)Qp * Mp);
    hipLaunchKernelGGL(bastin_contract_kernel, dim3(Qp / kBT, n_tiles), dim3(256), 0, s, tab,
                       tab + (size_t)Qp * Mp, gam, Q, Mp, part);
    // pref = -2 pi i (N/Omega)/de-^2 is imaginary: Re(pref F) = -Im(pref) Im(F).
    hipLaunchKernelGGL(bastin_sigma_kernel, dim3(K), dim3(256), 0, s, part, n_tiles, Q, den, K, e_min, e_max,
                       kT_ev / de_m, -2.0 * M_PI * orbitals_per_nm2 / (de_m * de_m), dsig);
    e = ::kpm::launch_status();
  }
  if (e == hipSuccess && !on_device) {
    e = hipMemcpyAsync(sigma, dsig, sizeof(double) * K, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)::kpm::dev_free(ws);
  if (e != hipSuccess) {
    set_error("kpm_reconstruct_sigma_bastin: %s", hipGetErrorString(e));
    return ::kpm::hip_status(e);
  }
  return KPM_OK;
}

namespace kpm {

// ---------------------------------------------------------------------------
// Optical conductivity sigma_ab(omega) at chemical potential mu and
// temperature T (eq. cond 1st order, rank-1 and rank-2 Gamma of eq. Gammanm,
// Lambda_n and Lambda_nm(omega), combined as in eq. conductivity_1st_order):
//   sigma(w)/(e^2/h) = (-2 pi i (N/Omega)/E_w) [ sum_n Gamma_n L_n + (1/de-) sum_nm Gamma_nm L_nm(w) ],
//   L_n = int f Delta_n,  L_nm(w) = int f [g^R_n(eps + w~) Delta_m + Delta_n g^A_m(eps - w~)],
// in theta with the quadrature and occupation weights of the Kubo-Bastin
// reconstruction.  The
// rank-2 part is the same contraction with ta = g^A(eps - w~) and
// tb = g^R(eps + w~): sum_n D_n sum_m (g^A_m Gamma_nm + g^R_m Gamma_mn).
// ---------------------------------------------------------------------------
// out = sum_q w_q sum_n Gamma1_n D_n(theta_q) (one workgroup, fixed order).
__global__ void optical_rank1_kernel(const double* g1, int M, int Q, double mut, double kTt, double* out) {
  __shared__ double sr[256], si[256];
  double ar = 0.0, ai = 0.0;
  for (int q = threadIdx.x; q < Q; q += blockDim.x) {
    const double wq = occ_weight(q, Q, mut, kTt);
    if (wq <= 0.0) continue;
    const double th = (q + 0.5) * M_PI / Q;
    double cr = 0.0, ci = 0.0;
    for (int n = 0; n < M; ++n) {
      const double d = 2.0 / M_PI * cos((double)n * th);
      cr += d * g1[2 * n];
      ci += d * g1[2 * n + 1];
    }
    ar += wq * cr;
    ai += wq * ci;
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
    out[0] = sr[0];
    out[1] = si[0];
  }
}

// para = sum_q w_q sum_t part[t][q] (one workgroup, fixed order).
__global__ void optical_para_kernel(const double2* part, int n_tiles, int Q, double mut, double kTt, double* para) {
  __shared__ double sr[256], si[256];
  double ar = 0.0, ai = 0.0;
  for (int q = threadIdx.x; q < Q; q += blockDim.x) {
    const double wq = occ_weight(q, Q, mut, kTt);
    if (wq <= 0.0) continue;
    double fr = 0.0, fi = 0.0;
    for (int t = 0; t < n_tiles; ++t) {
      fr += part[(int64_t)t * Q + q].x;
      fi += part[(int64_t)t * Q + q].y;
    }
    ar += wq * fr;
    ai += wq * fi;
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
    para[0] = sr[0];
    para[1] = si[0];
  }
}

// sigma[k] = -2 pi i (N/Omega)/E_k (lam + para_k / de-), stored (re, im).
__global__ void optical_final_kernel(const double* para, const double* lam, const double* omegas, int K, double de_m,
                                     double opn, double* sigma) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double xr = lam[0] + para[2 * k] / de_m, xi = lam[1] + para[2 * k + 1] / de_m;
  const double c = 2.0 * M_PI * opn / omegas[k];
  sigma[2 * k] = c * xi;        // -i (xr + i xi) = xi - i xr
  sigma[2 * k + 1] = -c * xr;
}

}  // namespace kpm

extern "C" int kpm_reconstruct_sigma_optical(const double* gamma_nm, const double* gamma_n, int32_t M,
                                             const double* omegas_ev, int32_t K, double mu_ev, double e_min,
                                             double e_max, double eta_ev, double kT_ev, double orbitals_per_nm2,
                                             int32_t n_theta, double* sigma, int32_t on_device, void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(gamma_nm && gamma_n && omegas_ev && sigma, "NULL argument");
  KPM_CHECK_ARG(M >= 1 && M <= 16384 && K >= 1 && K <= 65536, "need 1 <= M <= 16384 and 1 <= K <= 65536");
  KPM_CHECK_ARG(std::isfinite(e_min) && std::isfinite(e_max) && e_min < e_max, "need e_min < e_max");
  KPM_CHECK_ARG(std::isfinite(mu_ev), "mu must be finite");
  KPM_CHECK_ARG(eta_ev > 0.0 && std::isfinite(eta_ev), "eta must be > 0");
  KPM_CHECK_ARG(kT_ev >= 0.0 && std::isfinite(kT_ev), "kT must be >= 0");
  KPM_CHECK_ARG(orbitals_per_nm2 > 0.0, "orbitals_per_nm2 must be > 0");
  KPM_CHECK_ARG(n_theta >= 0 && n_theta <= (1 << 20), "n_theta must be in [0, 2^20]");
  hipStream_t s = (hipStream_t)hip_stream;
  // The frequencies set the table shifts: they are needed on the host.
  std::vector<double> om;
  try {
    om.resize((size_t)K);
  } catch (...) {
    set_error("kpm_reconstruct_sigma_optical: out of host memory");
    return KPM_E_NOMEM;
  }
  if (on_device) {
    KPM_TRY_HIP(hipMemcpyAsync(om.data(), omegas_ev, sizeof(double) * K, hipMemcpyDeviceToHost, s));
    KPM_TRY_SYNC(hipStreamSynchronize(s));
  } else {
    std::memcpy(om.data(), omegas_ev, sizeof(double) * K);
  }
  for (double w : om) KPM_CHECK_ARG(w > 0.0 && std::isfinite(w), "every frequency must be > 0 (hbar omega in eV)");
  const int Q = n_theta > 0 ? n_theta : 4 * M;
  const int Mp = (int)ceil_div(M, kBT) * kBT;
  const int Qp = (int)ceil_div(Q, kBT) * kBT;
  const int n_tiles = Mp / kBT;
  const double de_p = 0.5 * (e_max + e_min), de_m = 0.5 * (e_max - e_min);
  const double mut = (mu_ev - de_p) / de_m;
  const double kTt = kT_ev / de_m;
  const size_t b_gam = sizeof(double2) * (size_t)Mp * Mp;
  const size_t b_tab = 2 * sizeof(double2) * (size_t)Qp * Mp;
  const size_t b_part = sizeof(double2) * (size_t)n_tiles * Q;
  const size_t b_small = sizeof(double) * (2 * (size_t)K + 2);
  const size_t gn = (size_t)M * M * 2;
  const size_t b_host = on_device ? 0 : sizeof(double) * (gn + 2 * (size_t)M + (size_t)K + 2 * (size_t)K);
  char* ws = nullptr;
  KPM_TRY_HIP(::kpm::dev_malloc(&ws, b_gam + b_tab + b_part + b_small + b_host));
  double2* gam = (double2*)ws;
  double2* ta = (double2*)(ws + b_gam);
  double2* tb = ta + (size_t)Qp * Mp;
  double2* part = (double2*)(ws + b_gam + b_tab);
  double* para = (double*)(ws + b_gam + b_tab + b_part);
  double* lam = para + 2 * (size_t)K;
  const double* dgnm = gamma_nm;
  const double* dgn = gamma_n;
  const double* dom = omegas_ev;
  double* dsig = sigma;
  hipError_t e = hipSuccess;
  if (!on_device) {
    double* h = (double*)(ws + b_gam + b_tab + b_part + b_small);
    e = hipMemcpyAsync(h, gamma_nm, sizeof(double) * gn, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + gn, gamma_n, sizeof(double) * 2 * M, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + gn + 2 * M, omegas_ev, sizeof(double) * K, hipMemcpyHostToDevice, s);
    dgnm = h;
    dgn = h + gn;
    dom = h + gn + 2 * M;
    dsig = h + gn + 2 * M + K;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(pad_gamma_kernel, dim3((unsigned)ceil_div((int64_t)Mp * Mp, 256)), dim3(256), 0, s, dgnm, M,
                       Mp, gam);
    hipLaunchKernelGGL(optical_rank1_kernel, dim3(1), dim3(256), 0, s, dgn, M, Q, mut, kTt, lam);
    const double eta = eta_ev / de_m;
    for (int k = 0; k < K && e == hipSuccess; ++k) {
      const double wt = om[k] / de_m;
      hipLaunchKernelGGL(cpgf_table_kernel, dim3((unsigned)ceil_div(Q, 256)), dim3(256), 0, s, Q, M, Mp, -wt, eta, 0,
                         1, ta);   // g^A(eps - w~) = conj(g^R(eps - w~ + i eta))
      hipLaunchKernelGGL(cpgf_table_kernel, dim3((unsigned)ceil_div(Q, 256)), dim3(256), 0, s, Q, M, Mp, wt, eta, 0, 0,
                         tb);   // g^R(eps + w~)
      hipLaunchKernelGGL(bastin_contract_kernel, dim3(Qp / kBT, n_tiles), dim3(256), 0, s, ta, tb, gam, Q, Mp, part);
      hipLaunchKernelGGL(optical_para_kernel, dim3(1), dim3(256), 0, s, part, n_tiles, Q, mut, kTt,
                         para + 2 * k);
      e = ::kpm::launch_status();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(optical_final_kernel, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, s, para, lam, dom, K,
                         de_m, orbitals_per_nm2, dsig);
      e = ::kpm::launch_status();
    }
  }
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(sigma, dsig, sizeof(double) * 2 * K, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)::kpm::dev_free(ws);
  if (e != hipSuccess) {
    set_error("kpm_reconstruct_sigma_optical: %s", hipGetErrorString(e));
    return ::kpm::hip_status(e);
  }
  return KPM_OK;
}
