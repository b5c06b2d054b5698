// Jackson-damped DOS reconstruction (paper eqs. e7 and
// delta_function_cheb_expansion; Jackson kernel of Weisse et al. 2006, which
// the paper cites for KPM damping).  FP64 throughout.
//
//   rho(E) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(eps)] / (pi sqrt(1 - eps^2) de-)
//
// One workgroup stages c_n = g_n mu_n (x2 for n >= 1) in LDS in chunks; each
// thread owns one energy and runs the scalar Chebyshev recursion in x.

#include "kpm_internal.h"

#include <cmath>
#include <vector>

namespace kpm {

__device__ inline double jackson_g(int n, int M) {
  const double q = M_PI / (M + 1);
  return ((M - n + 1) * cos(q * n) + sin(q * n) / tan(q)) / (M + 1);
}

__global__ void jackson_dos_kernel(const double* mu, int M, const double* energies, int K, double e_min,
                                   double e_max, double* rho) {
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
      coef[i] = (n == 0 ? 1.0 : 2.0) * jackson_g(n, M) * mu[n];
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
  for (int n = threadIdx.x; n < M; n += blockDim.x) w[n] = jackson_g(n, M) * pref * cos(n * th);
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
  if (!on_device) {
    KPM_TRY_HIP(hipMalloc(&tmp, sizeof(double) * (gn + 2 * (size_t)K)));
    KPM_TRY_HIP(hipMemcpyAsync(tmp, gamma, sizeof(double) * gn, hipMemcpyHostToDevice, s));
    KPM_TRY_HIP(hipMemcpyAsync(tmp + gn, energies_ev, sizeof(double) * K, hipMemcpyHostToDevice, s));
    dg = tmp;
    den = tmp + gn;
    dsig = tmp + gn + K;
  }
  hipLaunchKernelGGL(sigma_kernel, dim3(K), dim3(256), sizeof(double) * M, s, dg, M, den, K, e_min, e_max,
                     orbitals_per_nm2, dsig);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !on_device) {
    e = hipMemcpyAsync(sigma, dsig, sizeof(double) * K, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) {
    set_error("kpm_reconstruct_sigma: %s", hipGetErrorString(e));
    return KPM_E_DEVICE;
  }
  return KPM_OK;
}

extern "C" int kpm_reconstruct_jackson(const double* mu, int32_t M, const double* energies_ev, int32_t K,
                                       double e_min, double e_max, double* rho, int32_t on_device,
                                       void* hip_stream) {
  using namespace kpm;
  clear_error();
  KPM_CHECK_ARG(mu && energies_ev && rho, "NULL argument");
  KPM_CHECK_ARG(M >= 1 && K >= 1, "need M >= 1 and K >= 1");
  KPM_CHECK_ARG(std::isfinite(e_min) && std::isfinite(e_max) && e_min < e_max, "need e_min < e_max");
  hipStream_t s = (hipStream_t)hip_stream;
  const double* dmu = mu;
  const double* den = energies_ev;
  double* drho = rho;
  double* tmp = nullptr;
  if (!on_device) {
    KPM_TRY_HIP(hipMalloc(&tmp, sizeof(double) * ((size_t)M + 2 * (size_t)K)));
    KPM_TRY_HIP(hipMemcpyAsync(tmp, mu, sizeof(double) * M, hipMemcpyHostToDevice, s));
    KPM_TRY_HIP(hipMemcpyAsync(tmp + M, energies_ev, sizeof(double) * K, hipMemcpyHostToDevice, s));
    dmu = tmp;
    den = tmp + M;
    drho = tmp + M + K;
  }
  hipLaunchKernelGGL(jackson_dos_kernel, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, s, dmu, M, den, K, e_min,
                     e_max, drho);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !on_device) {
    e = hipMemcpyAsync(rho, drho, sizeof(double) * K, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) {
    set_error("kpm_reconstruct_jackson: %s", hipGetErrorString(e));
    return KPM_E_DEVICE;
  }
  return KPM_OK;
}
