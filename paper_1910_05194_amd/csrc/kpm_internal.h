// Internal helpers of libkpm: status handling, the counter-based RNG and
// 16-byte vector packs.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/kpm.h"

namespace kpm {

void set_error(const char* fmt, ...);
void clear_error();

// Fault injection for the error-path tests (kpm_debug_inject_failure).  While
// it is armed, a countdown runs over the library's checked HIP operations;
// the operation that takes it to zero reports the injected error.  An
// allocation or a call wrapped in KPM_TRY_HIP is then skipped; a
// synchronising call (KPM_TRY_SYNC) and a kernel launch (launch_status) run
// and only their status is replaced, as when a real failure is reported by
// a later call.
bool fault_due();
hipError_t fault_error();

// Library status of a failed HIP call.
inline int hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? KPM_E_NOMEM : KPM_E_DEVICE; }
inline hipError_t after_call(hipError_t e) { return (e == hipSuccess && fault_due()) ? fault_error() : e; }
// Status of the kernel launches issued since the last check.
inline hipError_t launch_status() { return after_call(hipGetLastError()); }

// Device allocations of the library: hipMalloc behind the fault countdown,
// with a count of live allocations (kpm_debug_live_allocations) so that the
// error-path tests can see every buffer released.
void live_add(int64_t d);
template <typename T>
inline hipError_t dev_malloc(T** p, size_t bytes) {
  if (fault_due()) {
    *p = nullptr;
    return fault_error();
  }
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e == hipSuccess) live_add(1);
  else *p = nullptr;
  return e;
}
inline hipError_t dev_free(void* p) {
  if (!p) return hipSuccess;
  live_add(-1);
  return hipFree(p);
}

#define KPM_TRY_HIP_STATUS_(expr, text)                                                    \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      ::kpm::set_error("%s failed: %s (%s:%d)", text, hipGetErrorString(e_), __FILE__,     \
                       __LINE__);                                                           \
      (void)hipGetLastError();                                                              \
      return (e_ == hipErrorOutOfMemory) ? KPM_E_NOMEM : KPM_E_DEVICE;                      \
    }                                                                                       \
  } while (0)
// A HIP call behind the fault countdown (skipped when the injected failure falls on it).
#define KPM_HIP(call) (::kpm::fault_due() ? ::kpm::fault_error() : (call))
#define KPM_TRY_HIP(call) KPM_TRY_HIP_STATUS_(KPM_HIP(call), #call)
#define KPM_TRY_SYNC(call) KPM_TRY_HIP_STATUS_(::kpm::after_call(call), #call)

#define KPM_TRY(call)          \
  do {                         \
    int s_ = (call);           \
    if (s_ != KPM_OK) return s_; \
  } while (0)

#define KPM_CHECK_ARG(cond, ...)          \
  do {                                    \
    if (!(cond)) {                        \
      ::kpm::set_error(__VA_ARGS__);      \
      return KPM_E_INVALID;               \
    }                                     \
  } while (0)

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), counter-based form:
//   x_i = mix(key + (i+1) G), u_i = (x_i >> 11) 2^-53.
// ---------------------------------------------------------------------------
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPurposePhase = 1, kPurposeAnderson = 2, kPurposeVacancy = 3;

__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t sm_key(uint64_t purpose, uint64_t seed, uint64_t a, uint64_t b) {
  uint64_t k = sm_mix(seed + purpose * kGolden);
  k = sm_mix(k + a * kGolden);
  return sm_mix(k + b * kGolden);
}

__host__ __device__ inline double sm_uniform(uint64_t key, uint64_t i) {
  return (double)(sm_mix(key + (i + 1) * kGolden) >> 11) * (1.0 / 9007199254740992.0);
}

// A 16-byte pack of NC = 8/sizeof(T) complex values (re, im interleaved).
template <typename T>
struct alignas(16) Pack {
  static constexpr int NC = 8 / (int)sizeof(T);
  T v[2 * NC];
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline Pack<T> ld_pack(const T* p) {
  return __builtin_bit_cast(Pack<T>, *reinterpret_cast<const u32x4*>(p));
}
// Streaming (nontemporal) forms: data touched once per step.
template <typename T>
__device__ inline Pack<T> ld_pack_nt(const T* p) {
  return __builtin_bit_cast(Pack<T>, __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p)));
}
template <typename T>
__device__ inline void st_pack(T* p, const Pack<T>& v) {
  *reinterpret_cast<u32x4*>(p) = __builtin_bit_cast(u32x4, v);
}
template <typename T>
__device__ inline void st_pack_nt(T* p, const Pack<T>& v) {
  __builtin_nontemporal_store(__builtin_bit_cast(u32x4, v), reinterpret_cast<u32x4*>(p));
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// K blocking of the stored Chebyshev blocks of the conductivity path: element
// (row n, complex k) lives at complex index ((k / kBlkK) * rows + n) * kBlkK + k % kBlkK.
// One row chunk is 1 KiB per BF16 plane, so each recursion step writes whole
// DRAM-page-sized pieces, and the Gamma GEMM reads whole 128-byte lines.
constexpr int kBlkK = 256;
// Row padding of the stored blocks (zero rows), a multiple of every Gamma GEMM tile.
constexpr int kGammaRowAlign = 256;

}  // namespace kpm
