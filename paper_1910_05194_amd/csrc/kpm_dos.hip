// DOS / LDOS Chebyshev moments on gfx950.
//
// Paper passages: eq. e6 (matrix Chebyshev recursion), eq. e8 and Sec. 2(c)
// (stochastic trace, random vectors), Sec. 3(a) (matrix-free pattern-rule
// Hamiltonian with disorder fused into the multiplication), Sec. 3(b) (tiles
// of the lattice processed as a unit), eq. PcomplexityFactor (R vectors, S
// realisations).
//
// Data layout in HBM: one batch buffer per Chebyshev vector, lattice after
// lattice; inside a lattice [n2][n1][sublattice][spin][r] complex, r fastest,
// R padded to a multiple of the 16-byte pack (2 complex64 or 1 complex128).
// Each thread owns one (site, 16-byte chunk of r) column of a tile and walks
// the tile's rows along a2, so the neighbour rows it reads were loaded by the
// same workgroup one row earlier (L1/L2 hits) and every vector element crosses
// HBM once per step: read v_n, read v_{n-1}, write v_{n+1} in place of v_{n-1}.
//
// Moments use the product identities T_{2n} = 2 T_n^2 - T_0 and
// T_{2n+1} = 2 T_{n+1} T_n - T_1 (from T_m T_n = (T_{m+n} + T_{|m-n|})/2), so
// one step yields two moments from <v_n|v_n> and <v_{n+1}|v_n>, accumulated in
// FP64 in registers (products of FP32 values are exact in FP64), reduced per
// workgroup in LDS and across workgroups by a fixed-order tree: results are
// bitwise reproducible.

#include "kpm_geometry.h"
#include "kpm_internal.h"
#include "kpm_plan.h"
#include "kpm_stencil.h"

// Cache policy of the step kernel's streams: bit 0 = nontemporal store of
// v_{n+1}, bit 1 = nontemporal load of v_{n-1} (both are touched once per step).
#ifndef KPM_STEP_NT
#define KPM_STEP_NT 0
#endif

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

namespace kpm {

static thread_local std::string g_err;

// Fault injection state (kpm_debug_inject_failure) and the live-allocation count.
static std::atomic<int64_t> g_fault_countdown{0};
static std::atomic<int32_t> g_fault_kind{0};
static std::atomic<int32_t> g_fault_fired{0};
static std::atomic<int64_t> g_live_allocs{0};

bool fault_due() {
  int64_t c = g_fault_countdown.load(std::memory_order_relaxed);
  while (c > 0) {
    if (g_fault_countdown.compare_exchange_weak(c, c - 1, std::memory_order_relaxed)) {
      if (c == 1) {
        g_fault_fired.fetch_add(1, std::memory_order_relaxed);
        return true;
      }
      return false;
    }
  }
  return false;
}

hipError_t fault_error() {
  return g_fault_kind.load(std::memory_order_relaxed) == 0 ? hipErrorOutOfMemory : hipErrorLaunchFailure;
}

void live_add(int64_t d) { g_live_allocs.fetch_add(d, std::memory_order_relaxed); }

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------
// Geometry (paper Sec. 3(d) listing; the constants are in kpm_geometry.h).
// ---------------------------------------------------------------------------
// Honeycomb bond classes: A(n) - B(n + d_k).
constexpr int kBondD1[3] = {0, 1, 0};
constexpr int kBondD2[3] = {0, -1, -1};

struct Geometry {
  double a1[2], a2[2], tauA[2], tauB[2];
  double fA[2], fB[2];   // fractional coordinates of the sublattice positions
};

// Area of one unit cell (nm^2): a^2 sqrt(3)/2 (honeycomb), a^2 (square).
double cell_area_nm2(int kind) {
  return kind == KPM_SQUARE ? kASq * kASq : kAHc * kAHc * std::sqrt(3.0) / 2.0;
}

static Geometry honeycomb_geometry() {
  Geometry g;
  g.a1[0] = kAHc; g.a1[1] = 0.0;
  g.a2[0] = kAHc / 2.0; g.a2[1] = kAHc * std::sqrt(3.0) / 2.0;
  g.tauA[0] = 0.0; g.tauA[1] = -kAccHc / 2.0;
  g.tauB[0] = 0.0; g.tauB[1] = kAccHc / 2.0;
  auto frac = [&](const double* r, double* f) {
    // Solve r = f0 a1 + f1 a2 (a1 has no y component).
    f[1] = r[1] / g.a2[1];
    f[0] = (r[0] - f[1] * g.a2[0]) / g.a1[0];
  };
  frac(g.tauA, g.fA);
  frac(g.tauB, g.fB);
  return g;
}

template <typename T>
struct StepArgs {
  const LatDev<T>* lats;
  const int4* tiles;      // (lattice, r-group, x0, y0)
  const int* slot_of;     // moment slot of each tile
  int n_tiles;
  const T* __restrict__ v;
  const T* __restrict__ w;   // v_{n-1} (read when read_w)
  T* __restrict__ out;       // v_{n+1} (may equal w: in place)
  T* __restrict__ vel;       // velocity output h~^dir v_n (VEL; may be null)
  T* __restrict__ blk;       // K-blocked copy of out (blk_src 0) or vel (blk_src 1), may be null
  __bf16* __restrict__ blk_lo;   // split-BF16 store: blk holds the hi plane (as __bf16), blk_lo the lo plane
  const T* onsite;
  const uint8_t* mask;
  const T* phase;         // complex interleaved
  double* part;           // [n_slots][Rw][2] for this step
  T a, b;                 // v_{n+1} = a H~ v_n - b v_{n-1}
  T vel_scale;            // vel = vel_scale * [r^dir, H] v_n  (physical units, eV nm)
  int read_w, write_out, dots, vdir, blk_src;
  int64_t blk_row, blk_rows;   // row of this vector in the blocked [K/kBlkK][rows][kBlkK] store
  int Tx, Ty, E, Ew, Rp;
};

// ---------------------------------------------------------------------------
// Per-site arithmetic of one Chebyshev step (shared by both step kernels).
// ---------------------------------------------------------------------------
template <typename T, int KIND>
struct LatRegs {
  int64_t site_off, vec_off, phase_off;
  T onsite_const, hop, exch;
  T blk[3][8];
  int L1, L2;
};

template <typename T, int KIND>
__device__ inline void load_lat(const LatDev<T>& Lg, LatRegs<T, KIND>& L) {
  L.site_off = Lg.site_off;
  L.vec_off = Lg.vec_off;
  L.phase_off = Lg.phase_off;
  L.onsite_const = Lg.onsite_const;
  L.hop = Lg.hop;
  L.L1 = Lg.L1;
  L.L2 = Lg.L2;
  L.exch = Lg.exch;
  if constexpr (KIND == KPM_HONEYCOMB_SPIN) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int q = 0; q < 8; ++q) L.blk[k][q] = Lg.blk[k][q];
  }
}

// Hopping coefficients of column n1 for sublattice s (Peierls phases depend on
// n1 only; the table is indexed by the A site's cell, the B' image unwrapped).
template <typename T, int KIND, bool PHASE>
__device__ inline void column_coefficients(const StepArgs<T>& A, const LatRegs<T, KIND>& L, int s, int n1, int n1m,
                                           T* hre, T* him) {
  constexpr int NNB = KindTraits<KIND>::NNB;
#pragma unroll
  for (int k = 0; k < NNB; ++k) {
    hre[k] = L.hop;
    him[k] = (T)0;
  }
  if constexpr (PHASE) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int na = (s == 0) ? n1 : ((k == 1) ? n1m : n1);
      const T pre = A.phase[2 * (L.phase_off + (int64_t)na * 3 + k)];
      const T pim = A.phase[2 * (L.phase_off + (int64_t)na * 3 + k) + 1];
      hre[k] = pre;
      him[k] = (s == 0) ? pim : -pim;   // B side: conjugate
      if constexpr (KIND != KPM_HONEYCOMB_SPIN) {
        hre[k] *= L.hop;
        him[k] *= L.hop;
      }
    }
  }
}

// out = a (H~ v)_i - b w_i, vel = vel_scale [r^dir, H] v at one site (all
// spins, all complex values of the pack), and the doubling dot products.
template <typename T, int KIND, bool PHASE, bool VEL>
__device__ inline void site_update(const StepArgs<T>& A, const LatRegs<T, KIND>& L, int s, const T* hre,
                                   const T* him, const T* vcs, T ons, bool alive,
                                   const Pack<T> (&vo)[KindTraits<KIND>::NSPIN],
                                   const Pack<T> (&wo)[KindTraits<KIND>::NSPIN],
                                   const Pack<T> (&vn)[KindTraits<KIND>::NNB][KindTraits<KIND>::NSPIN],
                                   Pack<T> (&out)[KindTraits<KIND>::NSPIN], Pack<T> (&vout)[KindTraits<KIND>::NSPIN],
                                   double* vv, double* wv) {
  constexpr int NC = Pack<T>::NC;
  constexpr int NSPIN = KindTraits<KIND>::NSPIN;
  constexpr int NNB = KindTraits<KIND>::NNB;
#pragma unroll
  for (int sp = 0; sp < NSPIN; ++sp) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      // On-site term; the spin lattice adds the exchange field +-Delta_ex.
      T onsp = ons;
      if constexpr (KIND == KPM_HONEYCOMB_SPIN) onsp = ons + (sp == 0 ? L.exch : -L.exch);
      T hr = onsp * vo[sp].v[2 * j], hi = onsp * vo[sp].v[2 * j + 1];
      T gr = 0, gi = 0;   // velocity accumulator
#pragma unroll
      for (int k = 0; k < NNB; ++k) {
        // term_k = (hop from neighbour k) applied to v_k, rescaled units.
        T tr = 0, ti = 0;
        if constexpr (KIND == KPM_HONEYCOMB_SPIN) {
          // A side: B_k[sigma][s'] v_k,s';  B side: conj(B_k[s'][sigma]) v_k,s'.
          T br = 0, bi = 0;
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            T er, ei;
            if (s == 0) {
              er = L.blk[k][2 * (sp * 2 + s2)];
              ei = L.blk[k][2 * (sp * 2 + s2) + 1];
            } else {
              er = L.blk[k][2 * (s2 * 2 + sp)];
              ei = -L.blk[k][2 * (s2 * 2 + sp) + 1];
            }
            cmul_acc(br, bi, er, ei, vn[k][s2].v[2 * j], vn[k][s2].v[2 * j + 1]);
          }
          if constexpr (PHASE) cmul_acc(tr, ti, hre[k], him[k], br, bi);
          else { tr = br; ti = bi; }
        } else {
          if constexpr (PHASE) {
            cmul_acc(tr, ti, hre[k], him[k], vn[k][0].v[2 * j], vn[k][0].v[2 * j + 1]);
          } else {
            tr = L.hop * vn[k][0].v[2 * j];
            ti = L.hop * vn[k][0].v[2 * j + 1];
          }
        }
        hr += tr;
        hi += ti;
        if constexpr (VEL) {
          gr += vcs[k] * tr;
          gi += vcs[k] * ti;
        }
      }
      T orr = A.a * hr, oi = A.a * hi;
      if (A.read_w) {
        orr -= A.b * wo[sp].v[2 * j];
        oi -= A.b * wo[sp].v[2 * j + 1];
      }
      if (!alive) { orr = 0; oi = 0; gr = 0; gi = 0; }
      out[sp].v[2 * j] = orr;
      out[sp].v[2 * j + 1] = oi;
      if constexpr (VEL) {
        vout[sp].v[2 * j] = A.vel_scale * gr;
        vout[sp].v[2 * j + 1] = A.vel_scale * gi;
      }
      const double xr = (double)vo[sp].v[2 * j], xi = (double)vo[sp].v[2 * j + 1];
      vv[j] += xr * xr + xi * xi;
      wv[j] += (double)orr * xr + (double)oi * xi;
    }
  }
}

template <typename T, int KIND, bool VEL>
__device__ inline void store_site(const StepArgs<T>& A, T* ob, T* velb, int64_t vec_off_c, int64_t site, int64_t coff,
                                  const Pack<T> (&out)[KindTraits<KIND>::NSPIN],
                                  const Pack<T> (&vout)[KindTraits<KIND>::NSPIN]) {
  constexpr int NSPIN = KindTraits<KIND>::NSPIN;
#pragma unroll
  for (int sp = 0; sp < NSPIN; ++sp) {
    const int64_t eo = (site * NSPIN + sp) * A.Rp * 2 + coff;
    if (A.write_out) {
      if constexpr ((KPM_STEP_NT & 1) != 0) st_pack_nt(ob + eo, out[sp]);
      else st_pack(ob + eo, out[sp]);
    }
    if constexpr (VEL) {
      if (velb) {
        if constexpr ((KPM_STEP_NT & 1) != 0) st_pack_nt(velb + eo, vout[sp]);
        else st_pack(velb + eo, vout[sp]);
      }
    }
    if (A.blk) {
      const int64_t e = eo / 2 + vec_off_c;   // complex index in the batch vector
      const int64_t b = (e / kBlkK) * A.blk_rows * kBlkK + A.blk_row * kBlkK + (e % kBlkK);
      // Select values, not a reference: a runtime choice between the two
      // private arrays would place both in scratch memory.
      Pack<T> src = out[sp];
      if constexpr (VEL) {
        if (A.blk_src == 1) src = vout[sp];
      }
      if (A.blk_lo == nullptr) {
        st_pack(A.blk + 2 * b, src);
      } else if constexpr (sizeof(T) == 4) {
        // x = hi + lo with hi = bf16(x), lo = bf16(x - hi): 4 reals -> 4 + 4 bf16.
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 hi, lo;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          hi[q] = (__bf16)src.v[q];
          lo[q] = (__bf16)(src.v[q] - (float)hi[q]);
        }
        *reinterpret_cast<bf16x4*>(reinterpret_cast<__bf16*>(A.blk) + 2 * b) = hi;
        *reinterpret_cast<bf16x4*>(A.blk_lo + 2 * b) = lo;
      }
    }
  }
}

template <typename T, int KIND>
__device__ inline void load_w(const StepArgs<T>& A, const T* wb, int64_t site, int64_t coff,
                              Pack<T> (&wo)[KindTraits<KIND>::NSPIN]) {
  constexpr int NSPIN = KindTraits<KIND>::NSPIN;
#pragma unroll
  for (int sp = 0; sp < NSPIN; ++sp) {
    if (A.read_w) {
      if constexpr ((KPM_STEP_NT & 2) != 0) wo[sp] = ld_pack_nt(wb + (site * NSPIN + sp) * A.Rp * 2 + coff);
      else wo[sp] = ld_pack(wb + (site * NSPIN + sp) * A.Rp * 2 + coff);
    }
  }
}

// Neighbour sites of (n1, y, s): honeycomb A(n) <- B(n), B(n+(1,-1)), B(n+(0,-1));
// B(n) <- A(n), A(n-(1,-1)), A(n-(0,-1)); square: (+-1, 0), (0, +-1).
template <int KIND>
__device__ inline void neighbours(int s, int n1, int n1p, int n1m, int y, int ym, int yp, int L1, int64_t* nb) {
  if constexpr (KIND == KPM_SQUARE) {
    nb[0] = (int64_t)y * L1 + n1p;
    nb[1] = (int64_t)y * L1 + n1m;
    nb[2] = (int64_t)yp * L1 + n1;
    nb[3] = (int64_t)ym * L1 + n1;
  } else {
    if (s == 0) {
      nb[0] = ((int64_t)y * L1 + n1) * 2 + 1;
      nb[1] = ((int64_t)ym * L1 + n1p) * 2 + 1;
      nb[2] = ((int64_t)ym * L1 + n1) * 2 + 1;
    } else {
      nb[0] = ((int64_t)y * L1 + n1) * 2;
      nb[1] = ((int64_t)yp * L1 + n1m) * 2;
      nb[2] = ((int64_t)yp * L1 + n1) * 2;
    }
  }
}

// ---------------------------------------------------------------------------
// The Chebyshev step: one launch = one grid-wide step of eq. e6 over every
// tile of every lattice in the batch, with the two doubling dot products.
//
// Variant 1 (direct): each thread reads its neighbours from global memory;
// the row-by-row walk makes them L1/L2 hits in the common case.
// ---------------------------------------------------------------------------
template <typename T, int KIND, bool ONSITE, bool MASK, bool PHASE, bool VEL>
__global__ void __launch_bounds__(kMaxStepBlock) step_kernel(StepArgs<T> A) {
  using P = Pack<T>;
  constexpr int NC = P::NC;
  constexpr int NSUB = KindTraits<KIND>::NSUB;
  constexpr int NSPIN = KindTraits<KIND>::NSPIN;
  constexpr int NNB = KindTraits<KIND>::NNB;
  extern __shared__ double lds[];

  const int tid = threadIdx.x;
  const int Ew = A.Ew;
  const int cl = tid % Ew;
  const int grp = tid / Ew;               // index of this thread among those sharing cl
  const int n_grp = blockDim.x / Ew;
  const int s = grp % NSUB;
  const int xl = grp / NSUB;
  const int Rp = A.Rp;

  // XCD-aware static schedule: workgroup b runs on XCD b % 8; XCD x owns the
  // contiguous tile range [x*T/8, (x+1)*T/8) so that neighbouring tiles share
  // an L2.
  const int xcd = blockIdx.x & 7;
  const int jx = blockIdx.x >> 3;
  const int gx = gridDim.x >> 3;
  const int t_begin = (int)(((int64_t)xcd * A.n_tiles) >> 3);
  const int t_end = (int)(((int64_t)(xcd + 1) * A.n_tiles) >> 3);

  double vv[NC], wv[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) vv[j] = wv[j] = 0.0;

  for (int ti = t_begin + jx; ti < t_end; ti += gx) {
    const int4 tl = A.tiles[ti];
    LatRegs<T, KIND> L;
    load_lat<T, KIND>(A.lats[tl.x], L);
    T vcs[NNB];
    if constexpr (VEL) {
#pragma unroll
      for (int k = 0; k < NNB; ++k) vcs[k] = A.lats[tl.x].vc[A.vdir][s][k];
    }
    const int L1 = L.L1, L2 = L.L2;
    const int n1 = tl.z + xl;
    const int c = tl.y * Ew + cl;
    const bool act = (grp < n_grp) && (xl < A.Tx) && (n1 < L1) && (c < A.E);
    if (act) {
      const T* __restrict__ vb = A.v + L.vec_off;
      const T* __restrict__ wb = A.w + L.vec_off;
      T* __restrict__ ob = A.out + L.vec_off;
      T* __restrict__ velb = (VEL && A.vel) ? A.vel + L.vec_off : nullptr;
      const int n1p = (n1 + 1 == L1) ? 0 : n1 + 1;
      const int n1m = (n1 == 0) ? L1 - 1 : n1 - 1;
      T hre[NNB], him[NNB];
      column_coefficients<T, KIND, PHASE>(A, L, s, n1, n1m, hre, him);
      const int yend = min(tl.w + A.Ty, L2);
      const int64_t coff = (int64_t)c * NC * 2;
      for (int y = tl.w; y < yend; ++y) {
        const int ym = (y == 0) ? L2 - 1 : y - 1;
        const int yp = (y + 1 == L2) ? 0 : y + 1;
        const int64_t site = ((int64_t)y * L1 + n1) * NSUB + s;
        int64_t nb[NNB];
        neighbours<KIND>(s, n1, n1p, n1m, y, ym, yp, L1, nb);
        P vo[NSPIN], wo[NSPIN], vn[NNB][NSPIN];
#pragma unroll
        for (int sp = 0; sp < NSPIN; ++sp) {
          vo[sp] = ld_pack(vb + (site * NSPIN + sp) * Rp * 2 + coff);
#pragma unroll
          for (int k = 0; k < NNB; ++k) vn[k][sp] = ld_pack(vb + (nb[k] * NSPIN + sp) * Rp * 2 + coff);
        }
        load_w<T, KIND>(A, wb, site, coff, wo);
        T ons = L.onsite_const;
        if constexpr (ONSITE) ons = A.onsite[L.site_off + site];
        bool alive = true;
        if constexpr (MASK) alive = A.mask[L.site_off + site] != 0;
        P out[NSPIN], vout[NSPIN];
        site_update<T, KIND, PHASE, VEL>(A, L, s, hre, him, vcs, ons, alive, vo, wo, vn, out, vout, vv, wv);
        store_site<T, KIND, VEL>(A, ob, velb, L.vec_off / 2, site, coff, out, vout);
      }
    }
    // Flush the accumulators when the next tile of this workgroup belongs to
    // another moment slot (another lattice / r-group) or this was the last.
    const int tn = ti + gx;
    const int slot = A.dots ? A.slot_of[ti] : 0;
    if (A.dots && (tn >= t_end || A.slot_of[tn] != slot)) flush_slot<NC>(lds, A.part, slot, tid, Ew, grp, n_grp, vv, wv);
  }
}

// ---------------------------------------------------------------------------
// Variant 2 (LDS ring): the workgroup streams its tile row by row through a
// four-slot ring of rows in LDS (cells x0-1 .. x0+Tx, both sublattices), so
// every element of v_n is fetched from HBM once per tile and all neighbour
// reads are LDS reads.  A-sites of row y need B rows y and y-1 (already in the
// ring); B-sites need A rows y and y+1, so the walk loads row y+1 before
// updating row y.  One barrier per row: the slot written at row y+1 was last
// read two rows earlier.
// ---------------------------------------------------------------------------
template <typename T, int KIND, bool ONSITE, bool MASK, bool PHASE, bool VEL>
__global__ void __launch_bounds__(kMaxStepBlock) step_kernel_ring(StepArgs<T> A) {
  using P = Pack<T>;
  constexpr int NC = P::NC;
  constexpr int NSUB = KindTraits<KIND>::NSUB;
  constexpr int NSPIN = KindTraits<KIND>::NSPIN;
  constexpr int NNB = KindTraits<KIND>::NNB;
  extern __shared__ double lds[];

  const int tid = threadIdx.x;
  const int Ew = A.Ew;
  const int cl = tid % Ew;
  const int grp = tid / Ew;
  const int n_grp = blockDim.x / Ew;
  const int s = grp % NSUB;
  const int xl = grp / NSUB;
  const int Rp = A.Rp;
  const int Tx = A.Tx;
  // Ring layout: ring[slot][cell = xl + 1 in 0 .. Tx+1][sub][spin][chunk cl] as packs.
  P* ring = reinterpret_cast<P*>(lds + (size_t)blockDim.x * 2 * NC);
  const int row_packs = (Tx + 2) * NSUB * NSPIN * Ew;
  auto ring_at = [&](int slot, int cell, int sub, int sp, int ch) -> P& {
    return ring[(size_t)slot * row_packs + (((size_t)cell * NSUB + sub) * NSPIN + sp) * Ew + ch];
  };

  const int xcd = blockIdx.x & 7;
  const int jx = blockIdx.x >> 3;
  const int gx = gridDim.x >> 3;
  const int t_begin = (int)(((int64_t)xcd * A.n_tiles) >> 3);
  const int t_end = (int)(((int64_t)(xcd + 1) * A.n_tiles) >> 3);

  double vv[NC], wv[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) vv[j] = wv[j] = 0.0;

  for (int ti = t_begin + jx; ti < t_end; ti += gx) {
    const int4 tl = A.tiles[ti];
    LatRegs<T, KIND> L;
    load_lat<T, KIND>(A.lats[tl.x], L);
    T vcs[NNB];
    if constexpr (VEL) {
#pragma unroll
      for (int k = 0; k < NNB; ++k) vcs[k] = A.lats[tl.x].vc[A.vdir][s][k];
    }
    const int L1 = L.L1, L2 = L.L2;
    const int x0 = tl.z, y0 = tl.w;
    const int tx_eff = min(Tx, L1 - x0);          // valid cells of this tile column
    const int n1 = x0 + xl;
    const int c = tl.y * Ew + cl;
    const bool lane_ok = (grp < n_grp) && (c < A.E);
    const bool act = lane_ok && (xl < tx_eff);
    const int64_t coff = (int64_t)c * NC * 2;
    const T* __restrict__ vb = A.v + L.vec_off;
    const T* __restrict__ wb = A.w + L.vec_off;
    T* __restrict__ ob = A.out + L.vec_off;
    T* __restrict__ velb = (VEL && A.vel) ? A.vel + L.vec_off : nullptr;
    // Halo cells: the left neighbour column x0-1 and the right one x0+tx_eff
    // (both wrapped).  They are loaded by the threads of the first and last
    // valid cell column (one extra load each per row).
    const int hl = (x0 == 0) ? L1 - 1 : x0 - 1;
    const int hr = (x0 + tx_eff == L1) ? 0 : x0 + tx_eff;
    // Honeycomb: only B-sites read the left column (sublattice A) and only
    // A-sites read the right column (sublattice B).
    const bool load_left = lane_ok && (xl == 0) && (KIND == KPM_SQUARE || s == 0);
    const bool load_right = lane_ok && (xl == tx_eff - 1) && (KIND == KPM_SQUARE || s == 1);
    // Rows go through registers one iteration ahead of their use (two sets,
    // the loop unrolled by two), together with the site data of the row
    // being formed, so that a row's HBM latency overlaps the previous row's
    // work; the barrier covers LDS only.
    struct RowSet {
      P own[NSPIN], left[NSPIN], right[NSPIN], w[NSPIN];
      T ons;
      bool alive;
    };
    RowSet sa, sb;
    auto fetch_row = [&](RowSet& S, int yy) {
      // yy in [0, L2): this thread's own cell and, for edge threads, one halo cell.
      if (act) {
        const int64_t site = ((int64_t)yy * L1 + n1) * NSUB + s;
#pragma unroll
        for (int sp = 0; sp < NSPIN; ++sp) S.own[sp] = ld_pack(vb + (site * NSPIN + sp) * Rp * 2 + coff);
      }
      if (load_left) {
        const int64_t site = ((int64_t)yy * L1 + hl) * NSUB + s;
#pragma unroll
        for (int sp = 0; sp < NSPIN; ++sp) S.left[sp] = ld_pack(vb + (site * NSPIN + sp) * Rp * 2 + coff);
      }
      if (load_right) {
        const int64_t site = ((int64_t)yy * L1 + hr) * NSUB + s;
#pragma unroll
        for (int sp = 0; sp < NSPIN; ++sp) S.right[sp] = ld_pack(vb + (site * NSPIN + sp) * Rp * 2 + coff);
      }
    };
    auto store_row = [&](const RowSet& S, int slot) {
#pragma unroll
      for (int sp = 0; sp < NSPIN; ++sp) {
        if (act) ring_at(slot, xl + 1, s, sp, cl) = S.own[sp];
        if (load_left) ring_at(slot, 0, s, sp, cl) = S.left[sp];
        if (load_right) ring_at(slot, tx_eff + 1, s, sp, cl) = S.right[sp];
      }
    };
    auto fetch_site = [&](RowSet& S, int yy) {
      S.ons = L.onsite_const;
      S.alive = true;
      if (act) {
        const int64_t site = ((int64_t)yy * L1 + n1) * NSUB + s;
        if (A.read_w) load_w<T, KIND>(A, wb, site, coff, S.w);
        if constexpr (ONSITE) S.ons = A.onsite[L.site_off + site];
        if constexpr (MASK) S.alive = A.mask[L.site_off + site] != 0;
      }
    };
    const int n1m = (n1 == 0) ? L1 - 1 : n1 - 1;
    T hre[NNB], him[NNB];
    column_coefficients<T, KIND, PHASE>(A, L, s, act ? n1 : 0, act ? n1m : 0, hre, him);
    const int yend = min(y0 + A.Ty, L2);
    // Row y = y0 + k from the ring (rows y - 1, y, y + 1) and cur's site data.
    auto compute_row = [&](int k, const RowSet& cur) {
      const int y = y0 + k;
      const int sy = k & 3, sm = (k + 3) & 3, sp1 = (k + 1) & 3;
      if (act) {
        const int64_t site = ((int64_t)y * L1 + n1) * NSUB + s;
        P vo[NSPIN], vn[NNB][NSPIN];
#pragma unroll
        for (int sp = 0; sp < NSPIN; ++sp) {
          vo[sp] = ring_at(sy, xl + 1, s, sp, cl);
          if constexpr (KIND == KPM_SQUARE) {
            vn[0][sp] = ring_at(sy, xl + 2, 0, sp, cl);
            vn[1][sp] = ring_at(sy, xl, 0, sp, cl);
            vn[2][sp] = ring_at(sp1, xl + 1, 0, sp, cl);
            vn[3][sp] = ring_at(sm, xl + 1, 0, sp, cl);
          } else if (s == 0) {
            vn[0][sp] = ring_at(sy, xl + 1, 1, sp, cl);
            vn[1][sp] = ring_at(sm, xl + 2, 1, sp, cl);
            vn[2][sp] = ring_at(sm, xl + 1, 1, sp, cl);
          } else {
            vn[0][sp] = ring_at(sy, xl + 1, 0, sp, cl);
            vn[1][sp] = ring_at(sp1, xl, 0, sp, cl);
            vn[2][sp] = ring_at(sp1, xl + 1, 0, sp, cl);
          }
        }
        P out[NSPIN], vout[NSPIN];
        site_update<T, KIND, PHASE, VEL>(A, L, s, hre, him, vcs, cur.ons, cur.alive, vo, cur.w, vn, out, vout, vv,
                                         wv);
        store_site<T, KIND, VEL>(A, ob, velb, L.vec_off / 2, site, coff, out, vout);
      }
    };
    // Prologue: rows y0-1 and y0 into slots 3 and 0 (slot of row y0+k is k & 3).
    fetch_row(sa, y0 == 0 ? L2 - 1 : y0 - 1);
    store_row(sa, 3);
    fetch_row(sa, y0);
    store_row(sa, 0);
    // The spinful FP64 kernel has no registers for a second set: it loads
    // each row right before its use.
    constexpr bool kPrefetch = !(KIND == KPM_HONEYCOMB_SPIN && sizeof(T) == 8);
    if constexpr (kPrefetch) {
      // One row: cur holds v_n row y + 1 and the site data of row y.
      auto row = [&](int k, const RowSet& cur, RowSet& nxt) {
        const int y = y0 + k;
        // All of cur has arrived (vmcnt(0); expcnt and lgkmcnt left at their
        // maxima), so no later use of it waits for the loads issued below.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        store_row(cur, (k + 1) & 3);
        __builtin_amdgcn_sched_barrier(0);
        if (y + 1 < yend) {
          fetch_row(nxt, y + 2 >= L2 ? y + 2 - L2 : y + 2);
          fetch_site(nxt, y + 1);
        }
        lds_barrier();
        compute_row(k, cur);
      };
      fetch_row(sa, y0 + 1 == L2 ? 0 : y0 + 1);
      fetch_site(sa, y0);
      int k = 0;
      for (; y0 + k + 1 < yend; k += 2) {
        row(k, sa, sb);
        row(k + 1, sb, sa);
      }
      if (y0 + k < yend) row(k, sa, sb);
    } else {
      for (int k = 0; y0 + k < yend; ++k) {
        const int y = y0 + k;
        fetch_row(sa, y + 1 == L2 ? 0 : y + 1);
        fetch_site(sa, y);
        store_row(sa, (k + 1) & 3);
        lds_barrier();
        compute_row(k, sa);
      }
    }
    __syncthreads();   // the next tile reuses the ring
    const int tn = ti + gx;
    const int slot = A.dots ? A.slot_of[ti] : 0;
    if (A.dots && (tn >= t_end || A.slot_of[tn] != slot)) flush_slot<NC>(lds, A.part, slot, tid, Ew, grp, n_grp, vv, wv);
  }
}

// ---------------------------------------------------------------------------
// Model build: Anderson potential, vacancy mask, active-orbital count.
// ---------------------------------------------------------------------------
struct ModelLat {
  int64_t site_off, n_sites;
  double W, p, de_p, de_m;
  uint64_t key_anderson, key_vacancy;
  int n_spin;
};

template <typename T>
__global__ void model_kernel(const ModelLat* ml, int lat, T* onsite, uint8_t* mask,
                             unsigned long long* active) {
  const ModelLat m = ml[lat];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool alive = true;
  if (i < m.n_sites) {
    double V = 0.0;
    if (m.W != 0.0) V = m.W * (sm_uniform(m.key_anderson, (uint64_t)i) - 0.5);
    if (m.p > 0.0) alive = !(sm_uniform(m.key_vacancy, (uint64_t)i) < m.p);
    if (onsite) onsite[m.site_off + i] = (T)((V - m.de_p) / m.de_m);
    if (mask) mask[m.site_off + i] = alive ? 1 : 0;
  }
  // Count active orbitals: wave-level ballot, one atomic per wave.
  const bool contrib = (i < m.n_sites) && alive;
  const unsigned long long bal = __ballot(contrib);
  if ((threadIdx.x & 63) == 0 && bal) atomicAdd(active + lat, (unsigned long long)__popcll(bal) * m.n_spin);
}

__global__ void zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Peierls table: theta_k(n1) = 2 pi flux (s1_A + s1_B')/2 (s2_A - s2_B') for the
// hop B' -> A with B' = A + d_k unwrapped (fractional coordinates).
struct PhaseLat {
  int64_t off;
  int L1;
  double flux;
  double fA0, fA1, fB0, fB1;
};

template <typename T>
__global__ void phase_kernel(const PhaseLat* pl, int lat, T* phase) {
  const PhaseLat q = pl[lat];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q.L1 * 3) return;
  const int n1 = i / 3, k = i % 3;
  const int d1 = (k == 1) ? 1 : 0;
  const int d2 = (k == 0) ? 0 : -1;
  const double s1a = n1 + q.fA0, s2a = q.fA1;
  const double s1b = n1 + d1 + q.fB0, s2b = d2 + q.fB1;
  const double th = 2.0 * M_PI * q.flux * 0.5 * (s1a + s1b) * (s2a - s2b);
  phase[2 * (q.off + i)] = (T)cos(th);
  phase[2 * (q.off + i) + 1] = (T)sin(th);
}

// Start vectors: random phases exp(2 pi i u) (FP64, rounded once), zero on
// vacant sites and on padded vectors.
template <typename T>
__global__ void start_phase_kernel(T* x, int64_t vec_off, int64_t n_orb, int n_spin, int R, int Rp,
                                   const uint64_t* keys, const uint8_t* mask, int64_t site_off) {
  using P = Pack<T>;
  constexpr int NC = P::NC;
  const int E = Rp / NC;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_orb * E) return;
  const int64_t o = idx / E;
  const int c = (int)(idx % E);
  const bool alive = mask ? (mask[site_off + o / n_spin] != 0) : true;
  P p;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int r = c * NC + j;
    double cr = 0.0, ci = 0.0;
    if (alive && r < R) {
      const double u = sm_uniform(keys[r], (uint64_t)o);
      sincospi(2.0 * u, &ci, &cr);
    }
    p.v[2 * j] = (T)cr;
    p.v[2 * j + 1] = (T)ci;
  }
  *reinterpret_cast<P*>(x + vec_off + (o * Rp + (int64_t)c * NC) * 2) = p;
}

template <typename T>
__global__ void fill_zero_kernel(T* x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (T)0;
}

template <typename T>
__global__ void start_sites_kernel(T* x, int64_t vec_off, const int64_t* sites, int R, int Rp) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  x[vec_off + (sites[r] * Rp + r) * 2] = (T)1;
}

// ---------------------------------------------------------------------------
// Deterministic reduction of moment slots: dots[lat][r][step][2].
// grid = (steps in chunk, lattice*r-groups, ceil(2*Rw/64)), block = 1024:
// lane -> output, 16 waves -> contiguous slot sub-ranges, fixed-order sums.
// ---------------------------------------------------------------------------
__global__ void reduce_slots_kernel(const double* part, int64_t part_step_stride, int Rw, const int2* ranges,
                                    int n_rg, int Rp, int n_steps, int step0, double* dots) {
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sc = blockIdx.x;                 // step within the chunk
  const int lr = blockIdx.y;
  const int o = blockIdx.z * 64 + lane;      // output index within (r_local, q)
  const int2 rg = ranges[lr];
  const double* pb = part + (int64_t)sc * part_step_stride;
  double acc = 0.0;
  if (o < 2 * Rw) {
    const int per = (rg.y + 15) / 16;
    const int b = rg.x + wave * per;
    const int e = min(rg.x + rg.y, b + per);
    for (int sl = b; sl < e; ++sl) acc += pb[(int64_t)sl * 2 * Rw + o];
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && o < 2 * Rw) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += red[k][lane];
    const int lat = lr / n_rg, g = lr % n_rg;
    const int r = g * Rw + o / 2, q = o & 1;
    if (r < Rp) dots[(((int64_t)lat * Rp + r) * n_steps + step0 + sc) * 2 + q] = s;
  }
}

// mu_0 = <v0|v0>/norm, mu_1 = <v1|v0>/norm, mu_2k = 2<vk|vk>/norm - mu_0,
// mu_2k+1 = 2<vk+1|vk>/norm - mu_1.
__global__ void finish_kernel(const double* dots, int n_lat, int R, int Rp, int n_steps, int M,
                              const unsigned long long* active, int ldos, double* mu, int* flag) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_lat * R * M) return;
  const int n = (int)(idx % M);
  const int64_t lr = idx / M;
  const int r = (int)(lr % R);
  const int lat = (int)(lr / R);
  const double norm = ldos ? 1.0 : (double)active[lat];
  const double* d = dots + ((int64_t)lat * Rp + r) * n_steps * 2;
  const double mu0 = d[0] / norm, mu1 = d[1] / norm;
  double val;
  const int k = n >> 1;
  if (n == 0) val = mu0;
  else if (n == 1) val = mu1;
  else if ((n & 1) == 0) val = 2.0 * d[2 * k] / norm - mu0;
  else val = 2.0 * d[2 * k + 1] / norm - mu1;
  mu[idx] = val;
  if (!(fabs(val) <= 1.0 + 1e-6)) atomicMax(flag, n + 1);
}

__global__ void mean_kernel(const double* mu, int n_lat, int R, int M, double* mean) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_lat * M) return;
  const int n = (int)(idx % M);
  const int lat = (int)(idx / M);
  double s = 0.0;
  for (int r = 0; r < R; ++r) s += mu[((int64_t)lat * R + r) * M + n];
  mean[idx] = s / R;
}

__global__ void zero_int(int* p) { *p = 0; }

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
template <typename T, int KIND, bool ONSITE, bool MASK, bool PHASE, bool VEL>
static void* pick_variant(int variant) {
  if (variant == 2) return (void*)step_kernel_ring<T, KIND, ONSITE, MASK, PHASE, VEL>;
  return (void*)step_kernel<T, KIND, ONSITE, MASK, PHASE, VEL>;
}

template <typename T, int KIND, bool VEL>
static void* pick_step(int variant, bool onsite, bool mask, bool phase) {
  const int k = (onsite ? 4 : 0) | (mask ? 2 : 0) | (phase ? 1 : 0);
  switch (k) {
    case 0: return pick_variant<T, KIND, false, false, false, VEL>(variant);
    case 1: return pick_variant<T, KIND, false, false, true, VEL>(variant);
    case 2: return pick_variant<T, KIND, false, true, false, VEL>(variant);
    case 3: return pick_variant<T, KIND, false, true, true, VEL>(variant);
    case 4: return pick_variant<T, KIND, true, false, false, VEL>(variant);
    case 5: return pick_variant<T, KIND, true, false, true, VEL>(variant);
    case 6: return pick_variant<T, KIND, true, true, false, VEL>(variant);
    default: return pick_variant<T, KIND, true, true, true, VEL>(variant);
  }
}

template <typename T, bool VEL>
static void* pick_step_kind(int kind, int variant, bool onsite, bool mask, bool phase) {
  if (kind == KPM_HONEYCOMB) return pick_step<T, KPM_HONEYCOMB, VEL>(variant, onsite, mask, phase);
  if (kind == KPM_HONEYCOMB_SPIN) return pick_step<T, KPM_HONEYCOMB_SPIN, VEL>(variant, onsite, mask, phase);
  // The square lattice has no Peierls table: only the (onsite, mask) variants exist.
  const int k = (onsite ? 2 : 0) | (mask ? 1 : 0);
  switch (k) {
    case 0: return pick_variant<T, KPM_SQUARE, false, false, false, VEL>(variant);
    case 1: return pick_variant<T, KPM_SQUARE, false, true, false, VEL>(variant);
    case 2: return pick_variant<T, KPM_SQUARE, true, false, false, VEL>(variant);
    default: return pick_variant<T, KPM_SQUARE, true, true, false, VEL>(variant);
  }
}


static int validate_lattice(const kpm_lattice_t& L, int idx) {
  KPM_CHECK_ARG(L.kind == KPM_HONEYCOMB || L.kind == KPM_HONEYCOMB_SPIN || L.kind == KPM_SQUARE,
                "lattice %d: unknown kind %d", idx, L.kind);
  KPM_CHECK_ARG(L.L1 >= 2 && L.L2 >= 2, "lattice %d: L1, L2 must be >= 2 (got %d, %d)", idx, L.L1, L.L2);
  KPM_CHECK_ARG(std::isfinite(L.e_min) && std::isfinite(L.e_max) && L.e_min < L.e_max,
                "lattice %d: need e_min < e_max", idx);
  KPM_CHECK_ARG(std::isfinite(L.t), "lattice %d: t must be finite", idx);
  KPM_CHECK_ARG(L.anderson_w >= 0.0 && std::isfinite(L.anderson_w), "lattice %d: anderson_w must be >= 0", idx);
  KPM_CHECK_ARG(L.vacancy_p >= 0.0 && L.vacancy_p < 1.0, "lattice %d: vacancy_p must be in [0, 1)", idx);
  KPM_CHECK_ARG(L.rashba == 0.0 || L.kind == KPM_HONEYCOMB_SPIN,
                "lattice %d: Rashba coupling needs KPM_HONEYCOMB_SPIN", idx);
  KPM_CHECK_ARG(std::isfinite(L.exchange) && (L.exchange == 0.0 || L.kind == KPM_HONEYCOMB_SPIN),
                "lattice %d: the exchange field needs KPM_HONEYCOMB_SPIN", idx);
  if (L.flux != 0.0) {
    KPM_CHECK_ARG(L.kind != KPM_SQUARE, "lattice %d: flux on the square lattice is not supported", idx);
    const double q = L.flux * L.L1;
    KPM_CHECK_ARG(std::fabs(q - std::round(q)) < 1e-9, "lattice %d: flux*L1 must be an integer (got %.12g)", idx, q);
  }
  // Gershgorin: every eigenvalue lies within G = max_i (|H_ii| + sum_j |H_ij|)
  // = W/2 + |exchange| + Z |t| + 2 |rashba| of zero (Z = 3 bonds per site on
  // the honeycomb lattices, 4 on the square one; a spinful bond's spin-flip
  // entry has magnitude 2 |rashba| / 3; Peierls phases and vacancies do not
  // raise a row sum).  The interval is rarely reached (disorder and spin-orbit
  // terms do not add up at the band edge), so bounds may cut into it by a
  // quarter of their half-width; tighter bounds are detected from the moments
  // themselves (|mu_n| <= 1 must hold when the rescaled spectrum lies in
  // [-1, 1]).
  const double Z = (L.kind == KPM_SQUARE) ? 4.0 : 3.0;
  const double G = 0.5 * L.anderson_w + std::fabs(L.exchange) + Z * std::fabs(L.t) + 2.0 * std::fabs(L.rashba);
  const double slack = 0.125 * (L.e_max - L.e_min);
  KPM_CHECK_ARG(-G >= L.e_min - slack && G <= L.e_max + slack,
                "lattice %d: spectrum bounds [%g, %g] eV cut into the Gershgorin interval [%g, %g] eV by more "
                "than a quarter of their half-width",
                idx, L.e_min, L.e_max, -G, G);
  return KPM_OK;
}

template <typename T>
static void fill_latdev(kpm_plan* P, std::vector<LatDev<T>>& out) {
  const Geometry g = honeycomb_geometry();
  out.resize(P->n_lat);
  for (int l = 0; l < P->n_lat; ++l) {
    const kpm_lattice_t& L = P->lats[l];
    const double de_p = 0.5 * (L.e_max + L.e_min), de_m = 0.5 * (L.e_max - L.e_min);
    LatDev<T>& d = out[l];
    std::memset(&d, 0, sizeof(d));
    d.L1 = L.L1;
    d.L2 = L.L2;
    d.site_off = P->site_off[l];
    d.vec_off = P->vec_off[l];
    d.phase_off = P->phase_off[l];
    d.onsite_const = (T)(-de_p / de_m);
    d.hop = (T)(L.t / de_m);
    d.exch = (T)(L.exchange / de_m);
    // Velocity [r^dir, H]_ij = (r_i - r_j)_dir H_ij; the kernel applies it to the
    // rescaled hop terms, hence the factor de-.
    // The second-order operator [r^a, [r^b, H]]_ij = (r_i - r_j)_a (r_i - r_j)_b H_ij
    // (eq. generalized velocity with two indices) uses the same stencil with
    // the product of the two components (dir 2, 3, 4 = xx, xy, yy).
    const int ab[3][2] = {{0, 0}, {0, 1}, {1, 1}};
    if (L.kind == KPM_SQUARE) {
      const double d_sq[4][2] = {{-kASq, 0.0}, {kASq, 0.0}, {0.0, -kASq}, {0.0, kASq}};
      for (int k = 0; k < 4; ++k) {
        for (int dir = 0; dir < 2; ++dir) d.vc[dir][0][k] = (T)(d_sq[k][dir] * de_m);
        for (int q = 0; q < 3; ++q) d.vc[2 + q][0][k] = (T)(d_sq[k][ab[q][0]] * d_sq[k][ab[q][1]] * de_m);
      }
    } else {
      for (int k = 0; k < 3; ++k) {
        // d_k = r_A(n) - r_B(n + d_k): seen from A (+d_k) and from B (-d_k).
        double dk[2];
        for (int dir = 0; dir < 2; ++dir) {
          dk[dir] = g.tauA[dir] - (kBondD1[k] * g.a1[dir] + kBondD2[k] * g.a2[dir] + g.tauB[dir]);
          d.vc[dir][0][k] = (T)(dk[dir] * de_m);
          d.vc[dir][1][k] = (T)(-dk[dir] * de_m);
        }
        for (int q = 0; q < 3; ++q) {
          d.vc[2 + q][0][k] = (T)(dk[ab[q][0]] * dk[ab[q][1]] * de_m);
          d.vc[2 + q][1][k] = d.vc[2 + q][0][k];
        }
      }
    }
    if (L.kind == KPM_HONEYCOMB_SPIN) {
      typedef std::complex<double> cd;
      const cd I(0.0, 1.0);
      const cd sx[2][2] = {{0.0, 1.0}, {1.0, 0.0}};
      const cd sy[2][2] = {{0.0, -I}, {I, 0.0}};
      for (int k = 0; k < 3; ++k) {
        // Bond vector from B' = B(n + d_k) to A(n) (the hop j -> i with i = A).
        double dv[2];
        for (int ax = 0; ax < 2; ++ax)
          dv[ax] = g.tauA[ax] - (kBondD1[k] * g.a1[ax] + kBondD2[k] * g.a2[ax] + g.tauB[ax]);
        const double nrm = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1]);
        const double dx = dv[0] / nrm, dy = dv[1] / nrm;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            cd e = (a == b ? cd(L.t, 0.0) : cd(0.0, 0.0)) +
                   (2.0 * I / 3.0) * L.rashba * (sx[a][b] * dy - sy[a][b] * dx);
            e /= de_m;
            d.blk[k][2 * (a * 2 + b)] = (T)e.real();
            d.blk[k][2 * (a * 2 + b) + 1] = (T)e.imag();
          }
      }
    }
  }
}

static int plan_alloc(kpm_plan* P, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (P->use_arena) {
    // Caller-provided arena: 256-byte aligned pieces, no device allocation.
    const size_t off = (P->arena_used + 255) & ~(size_t)255;
    if (off > P->arena_cap || bytes > P->arena_cap - off) {
      set_error("workspace of %zu bytes or more exceeds the %zu-byte scratch array", off + bytes, P->arena_cap);
      return KPM_E_INVALID;
    }
    *ptr = P->arena_base + off;
    P->arena_used = off + bytes;
    P->dev_bytes += bytes;
    return KPM_OK;
  }
  hipError_t e = ::kpm::dev_malloc(ptr, bytes);
  if (e != hipSuccess) {
    set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? KPM_E_NOMEM : KPM_E_DEVICE;
  }
  P->dev_bytes += bytes;
  return KPM_OK;
}

void plan_free(kpm_plan* P) {
  void* bufs[] = {P->X, P->Y, P->Z, P->W, P->onsite, P->mask, P->phase, P->latdev, P->tiles, P->slot_of, P->ranges,
                  P->part, P->dots, P->keys, P->d_sites, P->active, P->mlat, P->plat, P->flag,
                  P->mu_dev, P->mean_dev};
  if (!P->use_arena)
    for (void* b : bufs)
      if (b) (void)::kpm::dev_free(b);
  if (P->graph_loop) (void)hipGraphExecDestroy(P->graph_loop);
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  for (auto& e : P->ev)
    if (e) (void)hipEventDestroy(e);
}

int plan_create(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p,
                       const kpm_tune_t* tune, kpm_plan** out, int (*arena_get)(char**), size_t arena_cap) {
  KPM_CHECK_ARG(out != nullptr, "plan output pointer is NULL");
  *out = nullptr;
  // No launch shape given: use the autotune cache (KPM_TUNE_CACHE) if it has one.
  kpm_tune_t cached;
  if (lat != nullptr && n_lat >= 1 && p != nullptr &&
      (!tune || (tune->block == 0 && tune->rows == 0 && tune->grid == 0 && tune->kernel == 0 && tune->chunks == 0))) {
    std::memset(&cached, 0, sizeof(cached));
    cached.use_graph = tune ? tune->use_graph : 1;
    if (tune_cache_lookup(lat, n_lat, p, &cached)) tune = &cached;
  }
  KPM_CHECK_ARG(lat != nullptr && n_lat >= 1, "need at least one lattice");
  KPM_CHECK_ARG(p != nullptr, "params is NULL");
  KPM_CHECK_ARG(p->num_moments >= 2, "num_moments must be >= 2");
  KPM_CHECK_ARG(p->precision == KPM_FP32 || p->precision == KPM_FP64, "precision must be KPM_FP32 or KPM_FP64");
  KPM_CHECK_ARG(p->start == KPM_START_RANDOM_PHASE || p->start == KPM_START_SITES, "unknown start kind");
  for (int l = 0; l < n_lat; ++l) KPM_TRY(validate_lattice(lat[l], l));
  for (int l = 1; l < n_lat; ++l)
    KPM_CHECK_ARG(lat[l].kind == lat[0].kind, "all lattices of a batch must have the same kind");
  int R;
  if (p->start == KPM_START_SITES) {
    KPM_CHECK_ARG(p->sites != nullptr && p->num_sites >= 1, "KPM_START_SITES needs sites");
    R = p->num_sites;
  } else {
    KPM_CHECK_ARG(p->num_random >= 1, "num_random must be >= 1");
    R = p->num_random;
  }
  kpm_plan* P = new kpm_plan();
  P->use_arena = arena_get != nullptr;
  P->arena_cap = P->use_arena ? arena_cap : 0;
  P->lats.assign(lat, lat + n_lat);
  P->p = *p;
  if (p->start == KPM_START_SITES) P->sites.assign(p->sites, p->sites + p->num_sites);
  P->p.sites = nullptr;
  P->n_lat = n_lat;
  P->kind = lat[0].kind;
  P->prec = p->precision;
  P->n_sub = (P->kind == KPM_SQUARE) ? 1 : 2;
  P->n_spin = (P->kind == KPM_HONEYCOMB_SPIN) ? 2 : 1;
  P->M = p->num_moments;
  P->R = R;
  P->tsize = (P->prec == KPM_FP32) ? 4 : 8;
  P->NC = (P->prec == KPM_FP32) ? 2 : 1;
  P->Rp = (int)ceil_div(R, P->NC) * P->NC;
  P->E = P->Rp / P->NC;
  P->n_steps = (P->M + 1) / 2;

  // Per-lattice offsets and which optional arrays are needed.
  int64_t so = 0, po = 0;
  for (int l = 0; l < n_lat; ++l) {
    const kpm_lattice_t& L = lat[l];
    const int64_t ns = (int64_t)L.L1 * L.L2 * P->n_sub;
    P->site_off.push_back(so);
    P->vec_off.push_back(so * P->n_spin * P->Rp * 2);
    P->phase_off.push_back(L.flux != 0.0 ? po : 0);
    if (L.flux != 0.0) po += (int64_t)L.L1 * 3;
    so += ns;
    if (L.anderson_w != 0.0) P->has_onsite = true;
    if (L.vacancy_p > 0.0) P->has_mask = true;
    if (L.flux != 0.0) P->has_phase = true;
  }
  P->n_sites = so;
  P->n_orb = so * P->n_spin;
  P->n_phase = po;
  // A lattice without its own table in a batch that needs one gets a table of
  // flux 0 (all phases 1).
  if (P->has_phase) {
    for (int l = 0; l < n_lat; ++l)
      if (lat[l].flux == 0.0) {
        P->phase_off[l] = P->n_phase;
        P->n_phase += (int64_t)lat[l].L1 * 3;
      }
  }

  // LDOS sites: range and vacancy checks on the host with the same generator.
  if (p->start == KPM_START_SITES) {
    for (int l = 0; l < n_lat; ++l) {
      const int64_t norb = (int64_t)lat[l].L1 * lat[l].L2 * P->n_sub * P->n_spin;
      const uint64_t kv = sm_key(kPurposeVacancy, lat[l].disorder_seed, 0, 0);
      for (int r = 0; r < R; ++r) {
        const int64_t o = P->sites[r];
        if (o < 0 || o >= norb) {
          set_error("LDOS site %lld out of range [0, %lld) for lattice %d", (long long)o, (long long)norb, l);
          delete P;
          return KPM_E_INVALID;
        }
        if (lat[l].vacancy_p > 0.0 && sm_uniform(kv, (uint64_t)(o / P->n_spin)) < lat[l].vacancy_p) {
          set_error("LDOS site %lld of lattice %d is vacant", (long long)o, l);
          delete P;
          return KPM_E_INVALID;
        }
      }
    }
  }

  // Launch shape.
  const bool block_given = tune && tune->block > 0;
  P->block = block_given ? tune->block : 256;
  P->Ty = (tune && tune->rows > 0) ? tune->rows : 64;
  P->use_graph = (tune ? (tune->use_graph != 0) : true) && !P->use_arena;
  if (P->block < 64 || P->block > kMaxStepBlock || (P->block % 64) != 0) {
    set_error("block must be a multiple of 64 in [64, %d]", kMaxStepBlock);
    delete P;
    return KPM_E_INVALID;
  }
  const int chunks = tune ? tune->chunks : 0;
  if (chunks < 0 || chunks > P->block / P->n_sub) {
    set_error("chunks must be in [0, block / sublattices]");
    delete P;
    return KPM_E_INVALID;
  }
  // Kernel variant: 3..6 = 2..5 steps per sweep (spinless lattices, with or
  // without Peierls phases, room for two more vectors), 2 = LDS row ring,
  // 1 = direct loads.  The default (four steps per sweep where eligible)
  // was the fastest on the graphene workloads in FP32 and FP64.
  const int want = (tune && tune->kernel > 0) ? tune->kernel : 5;
  if (want < 1 || want > 6) {
    set_error("kernel must be 0 (default) or 1..6");
    delete P;
    return KPM_E_INVALID;
  }
  P->variant = want;
  if (P->variant >= 3) {
    const double vec_b = (double)P->n_orb * P->Rp * 2 * P->tsize;
    size_t free_b = 0, total_b = 0;
    // Four vectors with 2 GB to spare, or (arena) with a quarter of the arena left for the rest.
    const bool room = P->use_arena ? 4.0 * vec_b <= 0.75 * (double)P->arena_cap
                                    : hipMemGetInfo(&free_b, &total_b) == hipSuccess && (double)free_b > 4.0 * vec_b + 2.0e9;
    // The sweep kernels address a lattice row with 32-bit offsets.
    bool rows_fit = true;
    for (int l = 0; l < n_lat; ++l)
      rows_fit = rows_fit && (int64_t)lat[l].L1 * P->n_sub * P->Rp * 2 * (int64_t)P->tsize < (int64_t(1) << 31);
    if (P->kind == KPM_HONEYCOMB_SPIN || !room || !rows_fit) P->variant = 2;
  }
  if (P->variant >= 3 && !block_given) P->block = kMaxStepBlock;
  int lds_max = 65536;
  {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      lds_max = v;
  }
  // Sweep kernels: by default a tile covers 8 chunks (128 contiguous bytes)
  // of each site, and at least 4 KS thread columns (KS - 1 on each side are
  // halo); the row rings must fit in LDS, otherwise (with the workgroup
  // size left to the library) a smaller workgroup, down to 4 KS thread
  // columns, and then fewer steps per sweep, down to the single-step ring.
  while (P->variant >= 3) {
    const int ks = P->variant - 1;
    if (chunks > 0) {
      P->Ew = (int)std::min<int64_t>(P->E, chunks);
    } else {
      P->Ew = (int)std::min<int64_t>(P->E, 8);
      while (P->Ew > 1 && P->block / (P->n_sub * P->Ew) < 4 * ks) P->Ew >>= 1;
    }
    P->Tx = P->block / (P->n_sub * P->Ew);
    const size_t rings = (4 * (size_t)ks * (P->Tx + 2) + 1) * P->n_sub * P->Ew * 16;
    if (P->Tx >= 2 * ks - 1 && rings <= (size_t)lds_max) break;
    if (!block_given && chunks == 0 && P->block - 64 >= 4 * ks * P->n_sub * P->Ew) {
      P->block -= 64;
      continue;
    }
    P->variant = (ks == 2) ? 2 : P->variant - 1;
  }
  P->sweep = (P->variant >= 3) ? P->variant - 1 : 1;
  if (P->variant < 3) {
    P->Ew = (int)std::min<int64_t>(P->E, chunks > 0 ? chunks : std::max(1, P->block / P->n_sub));
    P->Tx = std::max(1, P->block / (P->n_sub * P->Ew));
  }
  P->n_rg = (int)ceil_div(P->E, P->Ew);
  // Cells a tile owns along n1 (a sweep kernel spends KS - 1 thread columns per side on halos).
  const int xstep = P->Tx - 2 * (P->sweep - 1);
  if (!(tune && tune->rows > 0)) {
    // Default rows per tile: the largest power of two <= 64 (128 for the sweep
    // kernels, whose bands re-read 2 KS halo rows) that still gives at least
    // 2048 tiles (8 per CU), so that small lattices fill the chip.
    int ty = P->variant >= 3 ? 128 : 64;
    while (ty > 1) {
      int64_t nt = 0;
      for (int l = 0; l < n_lat; ++l) nt += ceil_div(lat[l].L1, xstep) * P->n_rg * ceil_div(lat[l].L2, ty);
      if (nt >= 2048) break;
      ty >>= 1;
    }
    P->Ty = ty;
  }

  // Tile work list ordered (lattice, r-group, row band, column band).
  std::vector<int4> tiles;
  for (int l = 0; l < n_lat; ++l)
    for (int g = 0; g < P->n_rg; ++g)
      for (int y0 = 0; y0 < lat[l].L2; y0 += P->Ty)
        for (int x0 = 0; x0 < lat[l].L1; x0 += xstep) tiles.push_back(make_int4(l, g, x0, y0));
  P->n_tiles = (int)tiles.size();
  // Default: a persistent grid of at most 2048 workgroups (8 per CU).
  int grid = (tune && tune->grid > 0) ? tune->grid : (int)std::min<int64_t>(2048, ceil_div(P->n_tiles, 8) * 8);
  if (grid % 8 != 0 || grid < 8) {
    set_error("grid must be a positive multiple of 8");
    delete P;
    return KPM_E_INVALID;
  }
  P->grid = grid;
  // Moment slots: walk each workgroup's static tile sequence; a new slot opens
  // whenever the (lattice, r-group) changes.  Slots are numbered so that those
  // of one (lattice, r-group) are contiguous.
  struct SlotKey { int lr, wg, seq; };
  std::vector<SlotKey> keys_list;
  std::vector<int> tile_slot_tmp(P->n_tiles, -1);
  const int gx = grid / 8;
  for (int b = 0; b < grid; ++b) {
    const int x = b & 7, j = b >> 3;
    const int tb = (int)(((int64_t)x * P->n_tiles) >> 3), te = (int)(((int64_t)(x + 1) * P->n_tiles) >> 3);
    int prev_lr = -1, seq = 0, cur = -1;
    for (int ti = tb + j; ti < te; ti += gx) {
      const int lr = tiles[ti].x * P->n_rg + tiles[ti].y;
      if (lr != prev_lr) {
        cur = (int)keys_list.size();
        keys_list.push_back({lr, b, seq++});
        prev_lr = lr;
      }
      tile_slot_tmp[ti] = cur;
    }
  }
  std::vector<int> order(keys_list.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (keys_list[a].lr != keys_list[b].lr) return keys_list[a].lr < keys_list[b].lr;
    if (keys_list[a].wg != keys_list[b].wg) return keys_list[a].wg < keys_list[b].wg;
    return keys_list[a].seq < keys_list[b].seq;
  });
  std::vector<int> new_id(order.size());
  for (size_t i = 0; i < order.size(); ++i) new_id[order[i]] = (int)i;
  std::vector<int> slot_of(P->n_tiles);
  for (int ti = 0; ti < P->n_tiles; ++ti) slot_of[ti] = new_id[tile_slot_tmp[ti]];
  P->n_slots = (int)order.size();
  std::vector<int2> ranges(n_lat * P->n_rg, make_int2(0, 0));
  for (size_t i = 0; i < order.size(); ++i) {
    const int lr = keys_list[order[i]].lr;
    if (ranges[lr].y == 0) ranges[lr].x = (int)i;
    ranges[lr].y++;
  }
  const int Rw = P->Ew * P->NC;
  const double part_step_bytes = (double)P->n_slots * Rw * 2 * 8;
  // Moment partials: at most 2 GB, or an eighth of a caller-provided arena.
  const double budget = P->use_arena ? (double)P->arena_cap / 8.0 : 2.0e9;
  P->steps_per_chunk = (int)std::max<double>(1.0, std::min<double>(P->n_steps, std::floor(budget / part_step_bytes)));
  // A sweep kernel writes the partials of its KS steps into one chunk.
  if (P->sweep > 1)
    P->steps_per_chunk = std::max(P->sweep, P->steps_per_chunk - P->steps_per_chunk % P->sweep);

  // Algorithmic bytes per step: read v_n and v_{n-1}, write v_{n+1}, per-site
  // arrays; a sweep kernel reads two vectors and the site arrays and writes
  // two vectors per KS steps.
  const double site_arrays =
      (P->has_onsite ? (double)P->n_sites * P->tsize : 0.0) + (P->has_mask ? (double)P->n_sites : 0.0);
  P->bytes_per_step = (P->sweep > 1)
                          ? (4.0 * (double)P->n_orb * P->Rp * 2 * P->tsize + site_arrays) / P->sweep
                          : 3.0 * (double)P->n_orb * P->Rp * 2 * P->tsize + site_arrays;

  // Device allocations.
  const size_t vec_bytes = (size_t)P->n_orb * P->Rp * 2 * P->tsize;
  int st = KPM_OK;
  size_t need = 0;
  bool measure = P->use_arena;
  auto A = [&](void** ptr, size_t bytes) {
    if (measure) need = ((need + 255) & ~(size_t)255) + std::max<size_t>(bytes, 16);
    else if (st == KPM_OK) st = plan_alloc(P, ptr, bytes);
  };
  auto alloc_all = [&]() {
    A(&P->X, vec_bytes);
    A(&P->Y, vec_bytes);
    if (P->sweep > 1) {
      A(&P->Z, vec_bytes);
      A(&P->W, vec_bytes);
    }
    if (P->has_onsite) A(&P->onsite, (size_t)P->n_sites * P->tsize);
    if (P->has_mask) A((void**)&P->mask, (size_t)P->n_sites);
    if (P->has_phase) A(&P->phase, (size_t)P->n_phase * 2 * P->tsize);
    A(&P->latdev, (size_t)n_lat * (P->prec == KPM_FP32 ? sizeof(LatDev<float>) : sizeof(LatDev<double>)));
    A((void**)&P->tiles, tiles.size() * sizeof(int4));
    A((void**)&P->slot_of, slot_of.size() * sizeof(int));
    A((void**)&P->ranges, ranges.size() * sizeof(int2));
    A((void**)&P->part, (size_t)part_step_bytes * P->steps_per_chunk);
    A((void**)&P->dots, (size_t)n_lat * P->Rp * P->n_steps * 2 * sizeof(double));
    A((void**)&P->keys, (size_t)n_lat * P->Rp * sizeof(uint64_t));
    if (!P->sites.empty()) A((void**)&P->d_sites, P->sites.size() * sizeof(int64_t));
    A((void**)&P->active, (size_t)n_lat * sizeof(unsigned long long));
    A((void**)&P->mlat, (size_t)n_lat * sizeof(ModelLat));
    A((void**)&P->plat, (size_t)n_lat * sizeof(PhaseLat));
    A((void**)&P->flag, sizeof(int));
    A((void**)&P->mu_dev, (size_t)n_lat * R * P->M * sizeof(double));
    A((void**)&P->mean_dev, (size_t)n_lat * P->M * sizeof(double));
  };
  if (measure) {
    // Arena: the whole workspace must fit, checked before anything is carved.
    alloc_all();
    if (need > P->arena_cap) {
      set_error("this workload needs %zu bytes of device workspace; the scratch array holds %zu", need,
                P->arena_cap);
      delete P;
      return KPM_E_INVALID;
    }
    measure = false;
    const int ast = arena_get(&P->arena_base);
    if (ast != KPM_OK) {
      delete P;
      return ast;
    }
  }
  alloc_all();
  if (st != KPM_OK) {
    plan_free(P);
    delete P;
    return st;
  }

  // Host-built tables.
  std::vector<uint64_t> keys((size_t)n_lat * P->Rp, 0);
  for (int l = 0; l < n_lat; ++l)
    for (int r = 0; r < P->Rp; ++r) keys[(size_t)l * P->Rp + r] = sm_key(kPurposePhase, p->vector_seed, l, r);
  std::vector<ModelLat> ml(n_lat);
  std::vector<PhaseLat> pl(n_lat);
  const Geometry g = honeycomb_geometry();
  for (int l = 0; l < n_lat; ++l) {
    const kpm_lattice_t& L = lat[l];
    ml[l].site_off = P->site_off[l];
    ml[l].n_sites = (int64_t)L.L1 * L.L2 * P->n_sub;
    ml[l].W = L.anderson_w;
    ml[l].p = L.vacancy_p;
    ml[l].de_p = 0.5 * (L.e_max + L.e_min);
    ml[l].de_m = 0.5 * (L.e_max - L.e_min);
    ml[l].key_anderson = sm_key(kPurposeAnderson, L.disorder_seed, 0, 0);
    ml[l].key_vacancy = sm_key(kPurposeVacancy, L.disorder_seed, 0, 0);
    ml[l].n_spin = P->n_spin;
    pl[l].off = P->phase_off[l];
    pl[l].L1 = L.L1;
    pl[l].flux = L.flux;
    pl[l].fA0 = g.fA[0];
    pl[l].fA1 = g.fA[1];
    pl[l].fB0 = g.fB[0];
    pl[l].fB1 = g.fB[1];
  }
  hipError_t e = hipSuccess;
  auto H2D = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes) e = KPM_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  };
  if (P->prec == KPM_FP32) {
    std::vector<LatDev<float>> ld;
    fill_latdev<float>(P, ld);
    H2D(P->latdev, ld.data(), ld.size() * sizeof(ld[0]));
  } else {
    std::vector<LatDev<double>> ld;
    fill_latdev<double>(P, ld);
    H2D(P->latdev, ld.data(), ld.size() * sizeof(ld[0]));
  }
  H2D(P->tiles, tiles.data(), tiles.size() * sizeof(int4));
  H2D(P->slot_of, slot_of.data(), slot_of.size() * sizeof(int));
  H2D(P->ranges, ranges.data(), ranges.size() * sizeof(int2));
  H2D(P->keys, keys.data(), keys.size() * sizeof(uint64_t));
  if (!P->sites.empty()) H2D(P->d_sites, P->sites.data(), P->sites.size() * sizeof(int64_t));
  H2D(P->mlat, ml.data(), ml.size() * sizeof(ModelLat));
  H2D(P->plat, pl.data(), pl.size() * sizeof(PhaseLat));
  if (!P->use_arena) {
    // The graph-capture stream and the timing events (not in the allocation-free form).
    if (e == hipSuccess) e = KPM_HIP(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    for (auto& ev : P->ev)
      if (e == hipSuccess) e = KPM_HIP(hipEventCreate(&ev));
  }
  if (e != hipSuccess) {
    set_error("plan setup failed: %s", hipGetErrorString(e));
    plan_free(P);
    delete P;
    return ::kpm::hip_status(e);
  }
  // LDS: the ring variant needs 4 rows of (Tx + 2) cells (fall back to direct
  // loads when that exceeds 64 KiB); a sweep kernel its row rings.
  const size_t ring_bytes = (size_t)P->block * 2 * P->NC * sizeof(double) +
                            4 * (size_t)(P->Tx + 2) * P->n_sub * P->n_spin * P->Ew * 16;
  if (P->variant == 2 && ring_bytes > 65536) P->variant = 1;
  if (P->sweep > 1) {
    // v_n ring and one ring per inner level; the moment flush reuses the same LDS between tiles.
    const size_t rings = (4 * (size_t)P->sweep * (P->Tx + 2) + 1) * P->n_sub * P->Ew * 16;
    P->lds_bytes = std::max(rings, (size_t)P->block * 2 * P->NC * sizeof(double));
    P->sweep_fn = sweep_kernel_fn(P->prec, P->kind, P->sweep, P->has_onsite, P->has_mask, P->has_phase, P->block,
                                  P->Tx, P->Ew);
  } else {
    P->lds_bytes = (P->variant == 2) ? ring_bytes : (size_t)P->block * 2 * P->NC * sizeof(double);
  }
  P->step_fn = (P->prec == KPM_FP32)
                   ? pick_step_kind<float, false>(P->kind, P->variant, P->has_onsite, P->has_mask, P->has_phase)
                   : pick_step_kind<double, false>(P->kind, P->variant, P->has_onsite, P->has_mask, P->has_phase);
  P->step_fn_vel = (P->prec == KPM_FP32)
                       ? pick_step_kind<float, true>(P->kind, P->variant, P->has_onsite, P->has_mask, P->has_phase)
                       : pick_step_kind<double, true>(P->kind, P->variant, P->has_onsite, P->has_mask, P->has_phase);
  if (const char* lg = std::getenv("KPM_LOG"); lg && *lg && std::strcmp(lg, "0") != 0) {
    static const char* kKind[] = {"honeycomb", "honeycomb+spin", "square"};
    std::fprintf(stderr,
                 "[kpm] plan: %d lattice(s) %s, %lld orbitals, R=%d (padded %d), M=%d, %s; kernel %d (%d step%s "
                 "per launch), block %d, tile %d cells x %d rows x %d chunks, grid %d, %d tiles, LDS %zu B, "
                 "device %.1f MB%s, %.1f MB per step\n",
                 n_lat, (P->kind >= 0 && P->kind <= 2) ? kKind[P->kind] : "?", (long long)P->n_orb, P->R, P->Rp,
                 P->M, P->prec == KPM_FP32 ? "fp32" : "fp64", P->variant, P->sweep, P->sweep > 1 ? "s" : "",
                 P->block, P->Tx, P->Ty, P->Ew, P->grid, P->n_tiles, P->lds_bytes,
                 (double)P->dev_bytes / 1e6,
                 P->use_arena ? " (scratch array)" : (P->use_graph ? ", graph" : ""), P->bytes_per_step / 1e6);
  }
  *out = P;
  return KPM_OK;
}

template <typename T>
static hipError_t launch_prep(kpm_plan* P, hipStream_t s) {
  T* X = (T*)P->X;
  hipLaunchKernelGGL(zero_u64, dim3(ceil_div(P->n_lat, 256)), dim3(256), 0, s, P->active, P->n_lat);
  for (int l = 0; l < P->n_lat; ++l) {
    const kpm_lattice_t& L = P->lats[l];
    const int64_t ns = (int64_t)L.L1 * L.L2 * P->n_sub;
    hipLaunchKernelGGL(model_kernel<T>, dim3(ceil_div(ns, 256)), dim3(256), 0, s, P->mlat, l, (T*)P->onsite,
                       P->mask, P->active);
    if (P->has_phase)
      hipLaunchKernelGGL(phase_kernel<T>, dim3(ceil_div((int64_t)L.L1 * 3, 256)), dim3(256), 0, s, P->plat, l,
                         (T*)P->phase);
    const int64_t norb = ns * P->n_spin;
    if (P->p.start == KPM_START_RANDOM_PHASE) {
      hipLaunchKernelGGL(start_phase_kernel<T>, dim3(ceil_div(norb * P->E, 256)), dim3(256), 0, s, X,
                         P->vec_off[l], norb, P->n_spin, P->R, P->Rp, P->keys + (size_t)l * P->Rp, P->mask,
                         P->site_off[l]);
    } else {
      const int64_t n = norb * P->Rp * 2;
      hipLaunchKernelGGL(fill_zero_kernel<T>, dim3(ceil_div(n, 256)), dim3(256), 0, s, X + P->vec_off[l], n);
      hipLaunchKernelGGL(start_sites_kernel<T>, dim3(ceil_div(P->R, 256)), dim3(256), 0, s, X, P->vec_off[l],
                         P->d_sites, P->R, P->Rp);
    }
  }
  return ::kpm::launch_status();
}

template <typename T>
static hipError_t launch_step_t(kpm_plan* P, hipStream_t s, const StepLaunch& L) {
  StepArgs<T> a;
  a.lats = (const LatDev<T>*)P->latdev;
  a.tiles = P->tiles;
  a.slot_of = P->slot_of;
  a.n_tiles = P->n_tiles;
  a.onsite = (const T*)P->onsite;
  a.mask = P->mask;
  a.phase = (const T*)P->phase;
  a.Tx = P->Tx;
  a.Ty = P->Ty;
  a.E = P->E;
  a.Ew = P->Ew;
  a.Rp = P->Rp;
  a.v = (const T*)L.v;
  a.w = (const T*)(L.w ? L.w : L.v);
  a.out = (T*)L.out;
  a.vel = (T*)L.vel;
  a.blk = (T*)L.blk;
  a.blk_lo = (__bf16*)L.blk_lo;
  a.blk_src = L.blk_src;
  a.blk_row = L.blk_row;
  a.blk_rows = L.blk_rows;
  a.a = (T)L.a;
  a.b = (T)L.b;
  a.vel_scale = (T)L.vel_scale;
  a.read_w = L.read_w;
  a.write_out = L.write_out;
  a.dots = L.dots;
  a.vdir = L.vdir;
  a.part = L.part;
  void* args[] = {&a};
  return ::kpm::after_call(hipLaunchKernel(L.velocity ? P->step_fn_vel : P->step_fn, dim3(P->grid),
                                           dim3(P->block), args, P->lds_bytes, s));
}

hipError_t plan_launch_step(kpm_plan* P, hipStream_t s, const StepLaunch& L) {
  // Single steps need the single-step tile list (a sweep plan's tiles overlap).
  if (P->sweep > 1) return hipErrorInvalidValue;
  return P->prec == KPM_FP32 ? launch_step_t<float>(P, s, L) : launch_step_t<double>(P, s, L);
}

hipError_t plan_launch_prep(kpm_plan* P, hipStream_t s) {
  return P->prec == KPM_FP32 ? launch_prep<float>(P, s) : launch_prep<double>(P, s);
}

int plan_set_vector_base(kpm_plan* P, int64_t r0) {
  std::vector<uint64_t> keys((size_t)P->n_lat * P->Rp, 0);
  for (int l = 0; l < P->n_lat; ++l)
    for (int r = 0; r < P->Rp; ++r)
      keys[(size_t)l * P->Rp + r] = sm_key(kPurposePhase, P->p.vector_seed, l, (uint64_t)(r0 + r));
  KPM_TRY_HIP(hipMemcpy(P->keys, keys.data(), keys.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
  P->r_base = r0;
  return KPM_OK;
}

// One sweep: steps k .. k + nlev - 1 of the recursion from v = v_k and
// w = v_{k-1}; out_a receives v_{k+nlev-1} (nlev >= 2), out_b v_{k+nlev}.
template <typename T>
static hipError_t launch_sweep_t(kpm_plan* P, hipStream_t s, const void* v, const void* w, void* out_a, void* out_b,
                                 int first, int nlev, double* part0, int64_t part_stride) {
  SweepArgs<T> a;
  a.lats = (const LatDev<T>*)P->latdev;
  a.tiles = P->tiles;
  a.slot_of = P->slot_of;
  a.n_tiles = P->n_tiles;
  a.v = (const T*)v;
  a.w = (const T*)(w ? w : v);
  a.out_a = (T*)out_a;
  a.out_b = (T*)out_b;
  a.onsite = (const T*)P->onsite;
  a.mask = P->mask;
  a.phase = (const T*)P->phase;
  for (int l = 0; l < kMaxSweep; ++l) a.part[l] = (l < nlev) ? part0 + l * part_stride : nullptr;
  a.a1 = first ? (T)1 : (T)2;
  a.b1 = first ? (T)0 : (T)1;
  a.read_w1 = first ? 0 : 1;
  a.nlev = nlev;
  a.Tx = P->Tx;
  a.Ty = P->Ty;
  a.E = P->E;
  a.Ew = P->Ew;
  a.Rp = P->Rp;
  void* args[] = {&a};
  return ::kpm::after_call(hipLaunchKernel(P->sweep_fn, dim3(P->grid), dim3(P->block), args, P->lds_bytes, s));
}

// The DOS recursion with KS steps per launch: v_0 = start, v_1 = H~ v_0,
// v_{k+1} = 2 H~ v_k - v_{k-1}.  A launch reads two buffers and writes the
// other two (four vectors rotate); the last launch runs the remaining steps.
static hipError_t launch_loop_sweep(kpm_plan* P, hipStream_t s) {
  const int Rw = P->Ew * P->NC;
  const int64_t part_stride = (int64_t)P->n_slots * Rw * 2;
  void* cur = P->X;    // v_k
  void* prev = P->W;   // v_{k-1} (unused for k = 0)
  void* fa = P->Y;
  void* fb = P->Z;
  int chunk0 = 0;
  for (int k = 0; k < P->n_steps; k += P->sweep) {
    const int nlev = std::min(P->sweep, P->n_steps - k);
    double* p0 = P->part + (int64_t)(k - chunk0) * part_stride;
    hipError_t le = (P->prec == KPM_FP32)
                        ? launch_sweep_t<float>(P, s, cur, prev, fa, fb, k == 0 ? 1 : 0, nlev, p0, part_stride)
                        : launch_sweep_t<double>(P, s, cur, prev, fa, fb, k == 0 ? 1 : 0, nlev, p0, part_stride);
    if (le != hipSuccess) return le;
    void* oc = cur;
    void* op = prev;
    cur = fb;
    prev = fa;
    fa = oc;
    fb = op;
    const int last = k + nlev - 1;
    if (last - chunk0 + 1 >= P->steps_per_chunk || last == P->n_steps - 1) {
      const int nsc = last - chunk0 + 1;
      hipLaunchKernelGGL(reduce_slots_kernel, dim3(nsc, P->n_lat * P->n_rg, (unsigned)ceil_div(2 * Rw, 64)),
                         dim3(1024), 0, s, P->part, part_stride, Rw, P->ranges, P->n_rg, P->Rp, P->n_steps, chunk0,
                         P->dots);
      chunk0 = last + 1;
    }
  }
  return ::kpm::launch_status();
}

static hipError_t launch_loop(kpm_plan* P, hipStream_t s) {
  if (P->sweep > 1) return launch_loop_sweep(P, s);
  const int Rw = P->Ew * P->NC;
  const int64_t part_stride = (int64_t)P->n_slots * Rw * 2;
  int chunk0 = 0;
  for (int k = 0; k < P->n_steps; ++k) {
    const bool odd = (k & 1) != 0;
    StepLaunch L;
    L.v = odd ? P->Y : P->X;
    L.w = odd ? P->X : P->Y;
    L.out = odd ? P->X : P->Y;
    L.a = (k == 0) ? 1.0 : 2.0;
    L.b = (k == 0) ? 0.0 : 1.0;
    L.read_w = (k == 0) ? 0 : 1;
    L.part = P->part + (int64_t)(k - chunk0) * part_stride;
    hipError_t le = plan_launch_step(P, s, L);
    if (le != hipSuccess) return le;
    if (k - chunk0 + 1 == P->steps_per_chunk || k == P->n_steps - 1) {
      const int nsc = k - chunk0 + 1;
      hipLaunchKernelGGL(reduce_slots_kernel, dim3(nsc, P->n_lat * P->n_rg, (unsigned)ceil_div(2 * Rw, 64)),
                         dim3(1024), 0, s, P->part, part_stride, Rw, P->ranges, P->n_rg, P->Rp, P->n_steps, chunk0,
                         P->dots);
      chunk0 = k + 1;
    }
  }
  return ::kpm::launch_status();
}

static hipError_t launch_finish(kpm_plan* P, hipStream_t s) {
  hipLaunchKernelGGL(zero_int, dim3(1), dim3(1), 0, s, P->flag);
  const int64_t n = (int64_t)P->n_lat * P->R * P->M;
  hipLaunchKernelGGL(finish_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, P->dots, P->n_lat, P->R, P->Rp,
                     P->n_steps, P->M, P->active, P->p.start == KPM_START_SITES ? 1 : 0, P->mu_dev, P->flag);
  hipLaunchKernelGGL(mean_kernel, dim3(ceil_div((int64_t)P->n_lat * P->M, 256)), dim3(256), 0, s, P->mu_dev,
                     P->n_lat, P->R, P->M, P->mean_dev);
  return ::kpm::launch_status();
}

static int plan_run(kpm_plan* P, double* mu_pv, double* mu_mean, int32_t on_dev, void* stream) {
  KPM_CHECK_ARG(P != nullptr, "plan is NULL");
  hipStream_t s = (hipStream_t)stream;
  const bool timed = P->ev[0] != nullptr;
  if (timed) KPM_TRY_HIP(hipEventRecord(P->ev[0], s));
  KPM_TRY_HIP(plan_launch_prep(P, s));
  if (timed) KPM_TRY_HIP(hipEventRecord(P->ev[1], s));
  if (P->use_graph) {
    if (!P->graph_loop) {
      // Capture the step loop once on the plan's private stream.
      hipGraph_t g = nullptr;
      KPM_TRY_HIP(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t le = launch_loop(P, P->cap_stream);
      hipError_t ce = hipStreamEndCapture(P->cap_stream, &g);
      if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        set_error("graph capture failed: %s / %s", hipGetErrorString(le), hipGetErrorString(ce));
        (void)hipGetLastError();
        return ::kpm::hip_status(le != hipSuccess ? le : ce);
      }
      hipError_t ie = hipGraphInstantiate(&P->graph_loop, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        P->graph_loop = nullptr;
        set_error("graph instantiate failed: %s", hipGetErrorString(ie));
        return ::kpm::hip_status(ie);
      }
    }
    KPM_TRY_HIP(hipGraphLaunch(P->graph_loop, s));
  } else {
    KPM_TRY_HIP(launch_loop(P, s));
  }
  if (timed) KPM_TRY_HIP(hipEventRecord(P->ev[2], s));
  KPM_TRY_HIP(launch_finish(P, s));
  const size_t mu_bytes = (size_t)P->n_lat * P->R * P->M * sizeof(double);
  const size_t mean_bytes = (size_t)P->n_lat * P->M * sizeof(double);
  const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (mu_pv) KPM_TRY_HIP(hipMemcpyAsync(mu_pv, P->mu_dev, mu_bytes, kind, s));
  if (mu_mean) KPM_TRY_HIP(hipMemcpyAsync(mu_mean, P->mean_dev, mean_bytes, kind, s));
  if (timed) KPM_TRY_HIP(hipEventRecord(P->ev[3], s));
  P->timed = timed;
  // The spectrum check needs the flag on the host: synchronise on the run's end.
  int flag = 0;
  std::vector<unsigned long long> act(P->n_lat);
  hipError_t e = KPM_HIP(hipMemcpyAsync(&flag, P->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  if (e == hipSuccess)
    e = KPM_HIP(hipMemcpyAsync(act.data(), P->active, act.size() * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s));
  // Wait also after a failure: the copies write this frame's host memory.
  const hipError_t se = ::kpm::after_call(hipStreamSynchronize(s));
  if (e == hipSuccess) e = se;
  if (e != hipSuccess) {
    set_error("reading the run's status flags: %s", hipGetErrorString(e));
    (void)hipGetLastError();
    return ::kpm::hip_status(e);
  }
  P->n_active_total = 0;
  for (auto a : act) P->n_active_total += (int64_t)a;
  if (flag != 0) {
    set_error("moment %d is non-finite or exceeds 1 + 1e-6 in magnitude: the spectrum bounds are too tight",
              flag - 1);
    return KPM_E_SPECTRUM;
  }
  return KPM_OK;
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free entry point: a file-scope device array
// (one copy per GPU, held until the process ends).  In host code its name is
// only a stand-in; its device address comes from hipGetSymbolAddress, once
// per device with that device current, and only that address is passed on.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)KPM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

static int scratch_address(char** out) {
  int dev = 0;
  KPM_TRY_HIP(hipGetDevice(&dev));
  KPM_CHECK_ARG(dev >= 0 && dev < kMaxDevices, "device %d is beyond the %d devices supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    KPM_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    KPM_CHECK_ARG(ptr != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return KPM_OK;
}

}  // namespace kpm

extern "C" {

int kpm_version(void) { return 1; }

int32_t kpm_debug_inject_failure(int32_t nth, int32_t kind) {
  if (nth < 0 || (kind != 0 && kind != 1)) {
    kpm::set_error("kpm_debug_inject_failure: need nth >= 0 and kind 0 or 1");
    return KPM_E_INVALID;
  }
  kpm::g_fault_countdown.store(0, std::memory_order_relaxed);
  const int32_t fired = kpm::g_fault_fired.exchange(0, std::memory_order_relaxed);
  kpm::g_fault_kind.store(kind, std::memory_order_relaxed);
  kpm::g_fault_countdown.store(nth, std::memory_order_relaxed);
  return fired;
}

int64_t kpm_debug_live_allocations(void) { return kpm::g_live_allocs.load(std::memory_order_relaxed); }

const char* kpm_last_error(void) { return kpm::g_err.c_str(); }

int kpm_plan_create(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p, const kpm_tune_t* tune,
                    kpm_plan_t** plan) {
  try {
    kpm::clear_error();
    return kpm::plan_create(lat, n_lat, p, tune, plan);
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_plan_create");
    return KPM_E_DEVICE;
  }
}

int kpm_plan_run(kpm_plan_t* plan, double* mu_per_vector, double* mu_mean, int32_t out_on_device, void* hip_stream) {
  try {
    kpm::clear_error();
    return kpm::plan_run(plan, mu_per_vector, mu_mean, out_on_device, hip_stream);
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_plan_run");
    return KPM_E_DEVICE;
  }
}

int kpm_plan_info(kpm_plan_t* P, kpm_plan_info_t* info) {
  KPM_CHECK_ARG(P != nullptr && info != nullptr, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n_steps = P->n_steps;
  info->n_tiles = P->n_tiles;
  info->grid = P->grid;
  info->block = P->block;
  info->rows = P->Ty;
  info->tile_cells_x = P->Tx;
  info->tile_chunks = P->Ew;
  info->r_padded = P->Rp;
  info->kernel = P->variant;
  info->n_orbitals = P->n_orb;
  info->bytes_per_step = P->bytes_per_step;
  info->n_active_total = P->n_active_total;
  if (P->timed) {
    float ms = 0.f;
    KPM_TRY_SYNC(hipEventSynchronize(P->ev[3]));
    KPM_TRY_HIP(hipEventElapsedTime(&ms, P->ev[1], P->ev[2]));
    info->last_loop_ms = ms;
    KPM_TRY_HIP(hipEventElapsedTime(&ms, P->ev[0], P->ev[3]));
    info->last_run_ms = ms;
  }
  return KPM_OK;
}

int kpm_plan_destroy(kpm_plan_t* plan) {
  if (!plan) return KPM_OK;
  kpm::plan_free(plan);
  delete plan;
  return KPM_OK;
}

int kpm_moments_dos(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p, double* mu_per_vector,
                    double* mu_mean, int32_t out_on_device, void* hip_stream) {
  kpm_plan_t* plan = nullptr;
  kpm_tune_t tune;
  std::memset(&tune, 0, sizeof(tune));
  tune.use_graph = 0;   // a one-shot run gains nothing from capturing the loop
  int st = kpm_plan_create(lat, n_lat, p, &tune, &plan);
  if (st != KPM_OK) return st;
  st = kpm_plan_run(plan, mu_per_vector, mu_mean, out_on_device, hip_stream);
  std::string keep = kpm::g_err;
  kpm_plan_destroy(plan);
  kpm::g_err = keep;
  return st;
}

int kpm_moments_dos_noalloc(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p,
                            double* mu_per_vector, double* mu_mean, int32_t out_on_device, void* hip_stream) {
  try {
    kpm::clear_error();
    kpm_tune_t tune;
    std::memset(&tune, 0, sizeof(tune));
    kpm_plan_t* plan = nullptr;
    int st = kpm::plan_create(lat, n_lat, p, &tune, &plan, kpm::scratch_address, kpm::kNoAllocScratchBytes);
    if (st != KPM_OK) return st;
    st = kpm::plan_run(plan, mu_per_vector, mu_mean, out_on_device, hip_stream);
    const std::string keep = kpm::g_err;
    kpm::plan_free(plan);
    delete plan;
    kpm::g_err = keep;
    return st;
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_moments_dos_noalloc");
    return KPM_E_DEVICE;
  }
}

}  // extern "C"
