// Device-side pieces shared by the Chebyshev step kernels (kpm_dos.hip) and
// the multi-step sweep kernels (kpm_sweep.hip).  Not part of the ABI.
#pragma once

#include "kpm_internal.h"

#include <type_traits>

namespace kpm {

// Per-lattice constants seen by the kernels.
template <typename T>
struct LatDev {
  int32_t L1, L2;
  int64_t site_off;     // first site of the lattice in the batch per-site arrays
  int64_t vec_off;      // first T element of the lattice's block in a vector buffer
  int64_t phase_off;    // first complex entry of its [L1][3] Peierls table
  T onsite_const;       // -de+/de- (used when there is no per-site array)
  T hop;                // t/de-
  T blk[3][8];          // spin lattice: H_{A,B'} / de- for bond class k (2x2 complex, row-major), no phase
  T vc[5][2][4];        // velocity weights for [dir][sublattice of i][neighbour k]: dir 0, 1 = x, y:
                        // (r_i - r_j)_dir * de-; dir 2, 3, 4 = xx, xy, yy: the product of two components * de-
  T exch;               // spin lattice: Delta_ex / de- (+ on spin up, - on spin down)
};

// Largest step workgroup.  Two waves per SIMD leave each wave 256 VGPRs, which
// the spinful (2x2 hopping) kernels need to run without scratch spills.
constexpr int kMaxStepBlock = 512;

// Workgroup barrier for LDS data: waits for this wave's LDS operations only.
// __syncthreads() also drains the global loads in flight, which would defeat
// the one-row-ahead register prefetch of the step kernels.  The memory clobber keeps the
// compiler from moving LDS accesses across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int KIND>
struct KindTraits;
template <>
struct KindTraits<KPM_HONEYCOMB> { static constexpr int NSUB = 2, NSPIN = 1, NNB = 3; };
template <>
struct KindTraits<KPM_HONEYCOMB_SPIN> { static constexpr int NSUB = 2, NSPIN = 2, NNB = 3; };
template <>
struct KindTraits<KPM_SQUARE> { static constexpr int NSUB = 1, NSPIN = 1, NNB = 4; };

template <typename T>
__device__ inline void cmul_acc(T& ore, T& oim, T are, T aim, T bre, T bim) {
  // Four FMAs (a sum of products would compile to a multiply, an FMA and an
  // add per real part: the compiler may not reassociate it).
  ore = fma(are, bre, ore);
  ore = fma(-aim, bim, ore);
  oim = fma(are, bim, oim);
  oim = fma(aim, bre, oim);
}

// Reduce the per-thread dot products of one moment slot over the workgroup
// (fixed-order LDS tree) and write them to part[slot].
template <int NC>
__device__ inline void flush_slot(double* lds, double* part, int slot, int tid, int Ew, int grp, int n_grp,
                                  double* vv, double* wv) {
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    lds[tid * 2 * NC + 2 * j] = vv[j];
    lds[tid * 2 * NC + 2 * j + 1] = wv[j];
    vv[j] = wv[j] = 0.0;
  }
  __syncthreads();
  int p2 = 1;
  while (p2 < n_grp) p2 <<= 1;
  for (int st = p2 >> 1; st > 0; st >>= 1) {
    if (grp < st && grp + st < n_grp) {
#pragma unroll
      for (int q = 0; q < 2 * NC; ++q) lds[tid * 2 * NC + q] += lds[(tid + st * Ew) * 2 * NC + q];
    }
    __syncthreads();
  }
  if (tid < Ew) {
    double* dst = part + ((int64_t)slot * Ew * NC + tid * NC) * 2;
#pragma unroll
    for (int q = 0; q < 2 * NC; ++q) dst[q] = lds[tid * 2 * NC + q];
  }
  __syncthreads();
}

// Memory access through buffer resources (the sweep kernels).  A resource covers one lattice row
// (its base is uniform; num_records = the row's bytes, < 2^31); an access at
// an offset >= num_records is dropped by the hardware's range check (a store
// writes nothing, a load returns zeros).  Threads without data for an access
// pass kOOB instead of branching around it, so every wave issues the same
// memory instructions in every row: the in-order vector-memory counter then
// lets a row wait for its own loads without also waiting for the previous
// row's stores (a branch around a store would make the compiler assume none
// was issued and drain the counter).
constexpr uint32_t kOOB = 0x80000000u;
constexpr int kRsrcFlags = 0x00020000;   // dword 3 of a gfx9 raw buffer resource

__device__ inline __amdgpu_buffer_rsrc_t row_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcFlags);
}
// Start of row y of a row-major array whose rows hold row_bytes bytes: the
// offset is formed as an unsigned 32 x 32 -> 64-bit product (y >= 0), two
// scalar instructions instead of a signed 64-bit multiply.
template <typename P>
__device__ inline P* row_ptr(P* base, int y, uint32_t row_bytes) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(base) + (uint64_t)(uint32_t)y * (uint64_t)row_bytes);
}
template <typename T>
__device__ inline Pack<T> buf_ld_pack(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(Pack<T>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <typename T>
__device__ inline void buf_st_pack(__amdgpu_buffer_rsrc_t r, uint32_t off, const Pack<T>& v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, 0);
}
template <typename T>
__device__ inline T buf_ld_scalar(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
}

// Multi-step sweep kernels (kpm_sweep.hip): at most kMaxSweep Chebyshev steps per launch.
constexpr int kMaxSweep = 5;

template <typename T>
struct SweepArgs {
  const LatDev<T>* __restrict__ lats;
  const int4* __restrict__ tiles;   // (lattice, r-group, x0, y0), x0 the first interior column
  const int* __restrict__ slot_of;
  int n_tiles;
  const T* __restrict__ v;          // v_n
  const T* __restrict__ w;          // v_{n-1} (read when read_w1)
  T* __restrict__ out_a;            // v_{n+nlev-1} (nlev >= 2)
  T* __restrict__ out_b;            // v_{n+nlev}
  const T* __restrict__ onsite;
  const uint8_t* __restrict__ mask;
  const T* __restrict__ phase;      // Peierls table [L1][3] complex per lattice (PHASE)
  double* part[kMaxSweep];          // slot partials of steps n .. n+nlev-1
  T a1, b1;
  int read_w1, nlev;
  int Tx, Ty, E, Ew, Rp;            // Tx = thread columns (interior + 2 (KS - 1))
};

// The sweep kernel instance for a precision (KPM_FP32 / KPM_FP64), lattice kind,
// steps per sweep (2..kMaxSweep), the optional per-site arrays and Peierls
// table, and the launch's workgroup size, thread columns and chunks per site.
void* sweep_kernel_fn(int prec, int kind, int ks, bool onsite, bool mask, bool phase, int block, int tx, int ew);

}  // namespace kpm
