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

#define KPM_TRY_HIP(call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      ::kpm::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,   \
                       __LINE__);                                                           \
      return (e_ == hipErrorOutOfMemory) ? KPM_E_NOMEM : KPM_E_DEVICE;                      \
    }                                                                                       \
  } while (0)

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
