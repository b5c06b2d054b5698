// Multi-step sweeps of the conductivity path's Chebyshev chains on gfx950.
//
// Paper passages: eq. Gammanm (the 2D moments Gamma_nm = <r| v T_n v T_m |r>
// from two chains of vectors), eq. generalized velocity (the velocity
// operator h~^a = [r^a, H~]), eq. HQAHE (spinful honeycomb lattice with Rashba
// coupling, exchange field and Peierls phases), Sec. 3(b) and Table 1 (tiles
// of the lattice processed as a unit).
//
// The chains of the Gamma path need every vector of the recursion: the L
// chain stores L_n = T_n(H~) h~^a r, the R chain stores R_m = h~^b T_m(H~) r,
// both into the K-blocked Gamma store.  A sweep forms KS recursion levels
// from one pass over v_n and v_{n-1} (the skewed-level row schedule of the
// DOS sweep kernel in kpm_sweep.hip: level l forms row y0 + j - (2 l - 1) at
// iteration j into a 4-slot LDS ring, one barrier per row) and writes, per
// level, one Gamma block row:
//   mode 0 (L chain): the level's value;
//   mode 1 (R chain): the velocity stencil of the level below it, which reads
//   the same neighbour values as the level itself, so level l also yields
//   h~^b of level l - 1.
// The last two levels go back to HBM for the next sweep.  Per KS steps HBM
// moves two vectors in, two out and KS block rows, against three vectors and
// one block row per step for single steps.
//
// Every thread forms one orbital; on the spinful lattice a ring cell holds
// both spins of a site and each thread reads both spins of its neighbours
// (the 2 x 2 hopping blocks mix them).
//
// A thread column outside a level's range computes values nobody reads (no
// branch on the column); stores and block stores are the only divergent
// branches.

#include "kpm_stencil.h"

#include <type_traits>

namespace kpm {

template <typename T>
struct ChainArgs {
  const LatDev<T>* __restrict__ lats;
  const int4* __restrict__ tiles;   // (lattice, r-group, x0, y0), x0 the first interior column
  int n_tiles;
  const T* __restrict__ v;          // level 0
  const T* __restrict__ w;          // level -1 (read when read_w1)
  T* __restrict__ out_a;            // level nlev - 1 (nlev >= 2)
  T* __restrict__ out_b;            // level nlev
  const T* __restrict__ onsite;     // per-site potential (has_onsite)
  const uint8_t* __restrict__ mask; // vacancy flags (has_mask)
  const T* __restrict__ phase;      // Peierls table [L1][3] complex per lattice (has_phase)
  T* blk;                           // K-blocked Gamma store (split BF16: the hi plane, as __bf16)
  __bf16* blk_lo;                   // split BF16: the lo plane (nullptr: store T values in blk)
  int64_t blk_row0;                 // mode 0: row of level 0 (level l goes to blk_row0 + l); mode 1: row of level 0's velocity
  int64_t blk_rows;                 // rows of the store (padded)
  T a1, b1;                         // level 1 = a1 H~ v - b1 w
  T vel_scale;                      // mode 1: velocity = vel_scale [r^vdir, H] (eV nm)
  int read_w1, nlev, vdir, has_onsite, has_mask, has_phase;
  int Tx, Ty, E, Ew, Rp;
};

// Hopping coefficients of one thread's orbital (per tile): the complex
// coefficient of the value of neighbour k, spin s2, in the result for the
// thread's spin, Peierls phase and hopping folded in.  Spinless: hop *
// exp(i theta_k).  Spinful: exp(i theta_k) times the 2 x 2 Rashba block
// entry, B_k[sp][s2] on sublattice A and conj(B_k[s2][sp]) on sublattice B.
template <typename T, int KIND>
struct Coef {
  static constexpr int NNB = KindTraits<KIND>::NNB, NSPIN = KindTraits<KIND>::NSPIN;
  T re[NNB][NSPIN], im[NNB][NSPIN];
  T vc[NNB];   // velocity weights (mode 1)
};

// One orbital: out = a (H~ v) - b w and, in mode 1, the velocity stencil of
// v, vout = vel_scale sum_k d_k term_k, where term_k is the hop from
// neighbour k (both spins) applied to its values.
template <typename T, int KIND, int MODE>
__device__ inline void chain_site(T a, T b, bool read_w, const Coef<T, KIND>& C, T ons, T vel_scale, bool alive,
                                  const Pack<T>& vo, const Pack<T>& wo,
                                  const Pack<T> (&vn)[KindTraits<KIND>::NNB][KindTraits<KIND>::NSPIN], Pack<T>& out,
                                  Pack<T>& vout) {
  constexpr int NC = Pack<T>::NC;
  constexpr int NSPIN = KindTraits<KIND>::NSPIN;
  constexpr int NNB = KindTraits<KIND>::NNB;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    T hr = ons * vo.v[2 * j], hi = ons * vo.v[2 * j + 1];
    T gr = 0, gi = 0;
    // Complex products as chains of FMAs (the compiler may not reassociate
    // a sum of products into them): four per coefficient and value.  Mode 0
    // adds every term straight into the result; mode 1 keeps each
    // neighbour's term for the velocity sum.
#pragma unroll
    for (int k = 0; k < NNB; ++k) {
      if constexpr (MODE == 1) {
        T tr = C.re[k][0] * vn[k][0].v[2 * j];
        T ti = C.re[k][0] * vn[k][0].v[2 * j + 1];
        tr = fma(-C.im[k][0], vn[k][0].v[2 * j + 1], tr);
        ti = fma(C.im[k][0], vn[k][0].v[2 * j], ti);
#pragma unroll
        for (int s2 = 1; s2 < NSPIN; ++s2) {
          tr = fma(C.re[k][s2], vn[k][s2].v[2 * j], tr);
          tr = fma(-C.im[k][s2], vn[k][s2].v[2 * j + 1], tr);
          ti = fma(C.re[k][s2], vn[k][s2].v[2 * j + 1], ti);
          ti = fma(C.im[k][s2], vn[k][s2].v[2 * j], ti);
        }
        hr += tr;
        hi += ti;
        gr = fma(C.vc[k], tr, gr);
        gi = fma(C.vc[k], ti, gi);
      } else {
#pragma unroll
        for (int s2 = 0; s2 < NSPIN; ++s2) {
          hr = fma(C.re[k][s2], vn[k][s2].v[2 * j], hr);
          hr = fma(-C.im[k][s2], vn[k][s2].v[2 * j + 1], hr);
          hi = fma(C.re[k][s2], vn[k][s2].v[2 * j + 1], hi);
          hi = fma(C.im[k][s2], vn[k][s2].v[2 * j], hi);
        }
      }
    }
    T orr = a * hr, oi = a * hi;
    if (read_w) {
      orr -= b * wo.v[2 * j];
      oi -= b * wo.v[2 * j + 1];
    }
    if (!alive) {
      orr = 0;
      oi = 0;
      gr = 0;
      gi = 0;
    }
    out.v[2 * j] = orr;
    out.v[2 * j + 1] = oi;
    if constexpr (MODE == 1) {
      vout.v[2 * j] = vel_scale * gr;
      vout.v[2 * j + 1] = vel_scale * gi;
    }
  }
}

// Threads: tid = ((column * NSUB + sub) * NSPIN + spin) * Ew + chunk; each
// thread forms one orbital (one spin of one site) and reads both spins of its
// neighbours from the rings.
//
// Memory goes through buffer resources (kpm_stencil.h) so that every wave
// issues the same memory instructions in every row: a row issues the next
// row's v_n loads and then, per level, two 8-byte block stores and one
// vector store (dropped, at offset kOOB, where the thread or the level has
// nothing to store).  The in-order vector-memory counter then lets a row
// wait for its own loads while the previous row's stores are still in flight.
template <typename T, int KIND, int KS, int MODE, bool SPLIT>
__global__ void __launch_bounds__(kMaxStepBlock) chain_sweep_kernel(ChainArgs<T> A) {
  using P = Pack<T>;
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  constexpr int NC = P::NC;
  constexpr int NSUB = KindTraits<KIND>::NSUB;
  constexpr int NSPIN = KindTraits<KIND>::NSPIN;
  constexpr int NNB = KindTraits<KIND>::NNB;
  static_assert(KS >= 2 && KS <= kMaxSweep, "2..kMaxSweep steps per sweep");
  constexpr int NH = 2 * KS - 2;   // site-data history: level l uses the entry 2 l - 3
  // Memory instructions a row issues after the next row's loads: per level two block stores
  // and one vector store.
  constexpr int kWaitVm = 3 * KS;
  static_assert(kWaitVm < 64, "vmcnt range");
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int Ew = A.Ew;
  const int cl = tid % Ew;
  const int grp = tid / Ew;
  const int n_grp = (int)blockDim.x / Ew;
  const int sp_t = (grp / NSUB) % NSPIN;
  const int s = grp % NSUB;
  const int xl = grp / (NSUB * NSPIN);
  const int Rp = A.Rp;
  const int Tx = A.Tx;
  const int nlev = A.nlev;
  constexpr bool split = SPLIT;   // split BF16 store (hi plane in blk, lo plane in blk_lo)
  static_assert(!SPLIT || sizeof(T) == 4, "split BF16 stores FP32 values");
  // Rings: [4 slots][Tx + 2 cells][sub][spin][chunk]; the v_n ring, then one per inner level.
  P* ring0 = reinterpret_cast<P*>(lds);
  const int row0 = (Tx + 2) * NSUB * NSPIN * Ew;
  P* ringl = ring0 + 4 * row0;
  const int xlc = (grp < n_grp) ? xl : Tx;   // surplus threads work on column Tx (cell Tx + 1, never read)
  auto r0 = [&](int slot, int cell, int sub, int sp) -> P& {
    return ring0[slot * row0 + ((cell * NSUB + sub) * NSPIN + sp) * Ew + cl];
  };
  auto rl = [&](int lev, int slot, int cell, int sub, int sp) -> P& {
    return ringl[((lev - 1) * 4 + slot) * row0 + ((cell * NSUB + sub) * NSPIN + sp) * Ew + cl];
  };

  const int xcd = blockIdx.x & 7;
  const int jx = blockIdx.x >> 3;
  const int gx = gridDim.x >> 3;
  const int t_begin = (int)(((int64_t)xcd * A.n_tiles) >> 3);
  const int t_end = (int)(((int64_t)(xcd + 1) * A.n_tiles) >> 3);

  for (int ti = t_begin + jx; ti < t_end; ti += gx) {
    const int4 tl = A.tiles[ti];
    const LatDev<T>& Lg = A.lats[tl.x];
    const int L1 = Lg.L1, L2 = Lg.L2;
    const int64_t site_off = Lg.site_off;
    // On-site energy of this spin: the exchange field +-Delta_ex on the spinful lattice.
    const T ons_spin = (KIND == KPM_HONEYCOMB_SPIN) ? (sp_t == 0 ? Lg.exch : -Lg.exch) : (T)0;
    const T ons_c = Lg.onsite_const + ons_spin;
    const int x0 = tl.z, y0 = tl.w;
    const int n_in = min(Tx - 2 * (KS - 1), L1 - x0);
    const int wcols = n_in + 2 * (KS - 1);
    int xe = (x0 - (KS - 1)) % L1;
    if (xe < 0) xe += L1;
    const int n1 = (xe + xl) % L1;
    // This column's coefficients (the Peierls phases depend on n1 only; the
    // table is indexed by the A site's cell, a B site's bond class 1 goes to
    // the A site of column n1 - 1, and the B side takes the conjugate).
    Coef<T, KIND> C;
    {
      T pre[NNB], pim[NNB];
#pragma unroll
      for (int k = 0; k < NNB; ++k) {
        pre[k] = 1;
        pim[k] = 0;
      }
      if (KIND != KPM_SQUARE && A.has_phase) {
        const int n1m = (n1 == 0) ? L1 - 1 : n1 - 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int na = (s == 0 || k != 1) ? n1 : n1m;
          const T* ph = A.phase + 2 * (Lg.phase_off + (int64_t)na * 3 + k);
          pre[k] = ph[0];
          pim[k] = (s == 0) ? ph[1] : -ph[1];
        }
      }
#pragma unroll
      for (int k = 0; k < NNB; ++k) {
        C.vc[k] = (MODE == 1) ? Lg.vc[A.vdir][s][k] : (T)0;
        if constexpr (KIND == KPM_HONEYCOMB_SPIN) {
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            const T er = (s == 0) ? Lg.blk[k][2 * (sp_t * 2 + s2)] : Lg.blk[k][2 * (s2 * 2 + sp_t)];
            const T ei = (s == 0) ? Lg.blk[k][2 * (sp_t * 2 + s2) + 1] : -Lg.blk[k][2 * (s2 * 2 + sp_t) + 1];
            C.re[k][s2] = pre[k] * er - pim[k] * ei;
            C.im[k][s2] = pre[k] * ei + pim[k] * er;
          }
        } else {
          C.re[k][0] = Lg.hop * pre[k];
          C.im[k][0] = Lg.hop * pim[k];
        }
      }
    }
    const int c = tl.y * Ew + cl;
    const bool lane_ok = (grp < n_grp) && (c < A.E);
    const bool act = lane_ok && (xl < wcols);
    const bool inner = act && (xl >= KS - 1) && (xl <= wcols - KS);
    const int hl = (xe == 0) ? L1 - 1 : xe - 1;
    const int hr = (xe + wcols) % L1;
    const bool load_left = lane_ok && (xl == 0) && (KIND == KPM_SQUARE || s == 0);
    const bool load_right = lane_ok && (xl == wcols - 1) && (KIND == KPM_SQUARE || s == 1);
    const bool load_halo = load_left || load_right;
    const int halo_col = load_left ? hl : hr;
    const int halo_cell = load_left ? 0 : wcols + 1;
    auto wrap = [&](int y) {
      while (y < 0) y += L2;
      while (y >= L2) y -= L2;
      return y;
    };
    auto next_row = [&](int y) { return (y + 1 == L2) ? 0 : y + 1; };
    // Offsets within one lattice row of a vector (a row holds < 2^31 bytes).
    const int64_t row_elems = (int64_t)L1 * NSUB * NSPIN * Rp * 2;
    const int64_t row_sites = (int64_t)L1 * NSUB;
    const uint32_t row_bytes = (uint32_t)(row_elems * (int64_t)sizeof(T));
    const int64_t lane_e = (((int64_t)n1 * NSUB + s) * NSPIN + sp_t) * Rp * 2 + (int64_t)c * NC * 2;
    const uint32_t lane_b = (uint32_t)(lane_e * (int64_t)sizeof(T));
    const uint32_t halo_b =
        (uint32_t)(((((int64_t)halo_col * NSUB + s) * NSPIN + sp_t) * Rp * 2 + (int64_t)c * NC * 2) * (int64_t)sizeof(T));
    const uint32_t lane_site = (uint32_t)(n1 * NSUB + s);
    const uint32_t ons_row_bytes = (uint32_t)(row_sites * (int64_t)sizeof(T));
    const T* vb = A.v + Lg.vec_off;
    const T* wb = A.w + Lg.vec_off;
    T* oa = A.out_a + Lg.vec_off;
    T* ob = A.out_b + Lg.vec_off;
    // The Gamma store: bytes per complex value in a plane (two BF16 or two T),
    // complex values per lattice row, this thread's complex offset within a
    // row, and the bytes from one K block to the next.
    const int esize = split ? 4 : 2 * (int)sizeof(T);
    const uint32_t row_cplx32 = (uint32_t)(row_elems / 2);
    const uint32_t vec_c32 = (uint32_t)(Lg.vec_off / 2);
    const uint32_t lane_c32 = (uint32_t)(lane_e / 2);
    const uint32_t kstride = (uint32_t)(A.blk_rows * kBlkK * esize);
    char* const blk_hi = reinterpret_cast<char*>(A.blk);
    char* const blk_lo = reinterpret_cast<char*>(A.blk_lo);
    // Everything a row needs from HBM (v_n with halos, v_{n-1} and the site
    // data of level 1's row) is loaded one iteration ahead, into one of two
    // register sets.
    P own[2], halo[2], wpre[2];
    T onspre[2];
    bool alivepre[2];
    auto fetch = [&](int k, int yv, int ysd, bool in_range) {
      const __amdgpu_buffer_rsrc_t rv = row_rsrc(row_ptr(vb, yv, row_bytes), row_bytes);
      own[k] = buf_ld_pack<T>(rv, (in_range && act) ? lane_b : kOOB);
      halo[k] = buf_ld_pack<T>(rv, (in_range && load_halo) ? halo_b : kOOB);
      const bool in1 = in_range && act;
      if (A.read_w1)
        wpre[k] = buf_ld_pack<T>(row_rsrc(row_ptr(wb, ysd, row_bytes), row_bytes), in1 ? lane_b : kOOB);
      onspre[k] = ons_c;
      if (A.has_onsite)
        onspre[k] = buf_ld_scalar<T>(row_rsrc(row_ptr(A.onsite + site_off, ysd, ons_row_bytes), ons_row_bytes),
                                     in1 ? lane_site * (uint32_t)sizeof(T) : kOOB) + ons_spin;
      alivepre[k] = true;
      if (A.has_mask)
        alivepre[k] = __builtin_amdgcn_raw_buffer_load_b8(
                          row_rsrc(row_ptr(A.mask + site_off, ysd, (uint32_t)row_sites), (uint32_t)row_sites),
                          in1 ? lane_site : kOOB, 0, 0) != 0;
    };
    // Threads without a cell to fill write to the spare cell after the last
    // ring instead (no branch): valid threads never read it.
    P* const spare = ring0 + 4 * KS * row0 + (s * NSPIN + sp_t) * Ew + cl;
    auto store_row = [&](int k, int slot) {
      *(act ? &r0(slot, xl + 1, s, sp_t) : spare) = own[k];
      *(load_halo ? &r0(slot, halo_cell, s, sp_t) : spare) = halo[k];
    };
    // A level's stores: its Gamma block row (its value in mode 0, the
    // velocity of the level below in mode 1), and the vector when it is one of
    // the sweep's last two levels.  Every level issues the same three store
    // instructions; `own` selects real offsets.
    auto emit = [&](int lev, int yw, bool own, const P& o, const P& g) {
      // Gamma store: row brow of the K blocks that hold lattice row yw.  The
      // row's first complex value ey0 and its K block kb0 are uniform; each
      // thread adds its own complex offset and, where the row does not start
      // on a K-block boundary, the blocks it crosses (32-bit arithmetic: the
      // plan checks the ranges).
      const int brow = (MODE == 0) ? A.blk_row0 + lev : A.blk_row0 + lev - 1;
      const uint32_t ey0 = (uint32_t)yw * row_cplx32 + vec_c32;
      const uint32_t kb0 = ey0 / kBlkK;
      const uint32_t ec = ey0 + lane_c32;
      const uint32_t off = ((ec / kBlkK) - kb0) * kstride + (ec % kBlkK) * (uint32_t)esize;
      const uint64_t base = (uint64_t)kb0 * kstride + (uint32_t)(brow * kBlkK * esize);
      const P& src = (MODE == 0) ? o : g;
      u32x2 h, l;
      if constexpr (split) {
        if constexpr (sizeof(T) == 4) {
          if constexpr (MODE == 0) {
            // Two values per conversion (v_cvt_pk_bf16_f32 rounds a pair;
            // the velocity chain's code is already paired by the compiler).
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const f32x2 x = {src.v[2 * q], src.v[2 * q + 1]};
              const bf16x2 hv = __builtin_convertvector(x, bf16x2);
              const f32x2 r = x - __builtin_convertvector(hv, f32x2);
              const bf16x2 lv = __builtin_convertvector(r, bf16x2);
              h[q] = __builtin_bit_cast(unsigned int, hv);
              l[q] = __builtin_bit_cast(unsigned int, lv);
            }
          } else {
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            bf16x4 hi, lo;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              hi[q] = (__bf16)src.v[q];
              lo[q] = (__bf16)(src.v[q] - (float)hi[q]);
            }
            h = __builtin_bit_cast(u32x2, hi);
            l = __builtin_bit_cast(u32x2, lo);
          }
        }
      } else {
        const u32x4 all = __builtin_bit_cast(u32x4, src);
        h = u32x2{all[0], all[1]};
        l = u32x2{all[2], all[3]};
      }
      // Split: hi plane and lo plane at the same offset; otherwise the two halves of the pack.
      char* p0 = blk_hi + base;
      char* p1 = split ? blk_lo + base : p0 + 8;
      __builtin_amdgcn_raw_buffer_store_b64(h, row_rsrc(p0, 0x7FFFFFFFu), own ? off : kOOB, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b64(l, row_rsrc(p1, 0x7FFFFFFFu), own ? off : kOOB, 0, 0);
      T* dst = (lev == nlev) ? ob : oa;
      const bool to_vec = own && (lev == nlev || lev == nlev - 1);
      buf_st_pack<T>(row_rsrc(row_ptr(dst, yw, row_bytes), row_bytes), to_vec ? lane_b : kOOB, o);
    };
    // The same three instructions, all dropped (a level without work in this row).
    auto emit_none = [&](const P& o) {
      const __amdgpu_buffer_rsrc_t rz = row_rsrc(ob, row_bytes);
      const u32x4 all = __builtin_bit_cast(u32x4, o);
      __builtin_amdgcn_raw_buffer_store_b64(u32x2{all[0], all[1]}, rz, kOOB, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b64(u32x2{all[2], all[3]}, rz, kOOB, 0, 0);
      buf_st_pack<T>(rz, kOOB, o);
    };
    const int ty = min(A.Ty, L2 - y0);
    const int j0 = 2 - KS;
    const int j_last = ty + 2 * KS - 2;
    // Level l (2..KS) works at iterations j with l <= nlev and j - (3 l - 1 - KS)
    // in [0, lev_cnt), and forms row y0 + j - (2 l - 1), one of the tile's
    // rows when j - (2 l - 1) is in [0, ty): one unsigned comparison each.
    uint32_t lev_cnt[KS - 1];
#pragma unroll
    for (int lev = 2; lev <= KS; ++lev) lev_cnt[lev - 2] = (lev <= nlev) ? (uint32_t)(ty + 2 * KS - 2 * lev) : 0u;
    T ons_h[NH];
    bool alive_h[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      ons_h[k] = ons_c;
      alive_h[k] = true;
    }
    // Rows of the next fetch: v_n row yf and its level-1 row ys = yf - 1; the
    // wrapped row yl[l] that level l forms in the current iteration.
    int yf = wrap(y0 + j0 + 1), ys = wrap(y0 + j0);
    int yl[KS + 1];
#pragma unroll
    for (int l = 1; l <= KS; ++l) yl[l] = wrap(y0 + j0 - (2 * l - 1));
    auto row = [&](auto ph, int j) {
      constexpr int p = decltype(ph)::value;
      // This row's v_n has arrived: everything issued before the previous row's stores is complete.
      __builtin_amdgcn_s_waitcnt(0x0F70 | (kWaitVm & 15) | ((kWaitVm >> 4) << 14));
      store_row(p & 1, (p + 2) & 3);
      // Level 1's row: v_{n-1} and the site data arrived with this row's v_n.
      const P w1 = wpre[p & 1];
      const T ons1 = onspre[p & 1];
      const bool alive1 = alivepre[p & 1] || !act;
      __builtin_amdgcn_sched_barrier(0);
      fetch((p + 1) & 1, yf, ys, j + 1 <= ty + KS - 1);
      lds_barrier();
      const int x = xlc + 1;
#pragma unroll
      for (int lev = KS; lev >= 2; --lev) {
        if ((uint32_t)(j - (3 * lev - 1 - KS)) < lev_cnt[lev - 2]) {
          constexpr int sp1 = (p + 3) & 3, s0 = (p + 2) & 3, sm1 = (p + 1) & 3;   // rows y + 1, y, y - 1
          P vn[NNB][NSPIN];
#pragma unroll
          for (int sp = 0; sp < NSPIN; ++sp) {
            if constexpr (KIND == KPM_SQUARE) {
              vn[0][sp] = rl(lev - 1, s0, x + 1, 0, sp);
              vn[1][sp] = rl(lev - 1, s0, x - 1, 0, sp);
              vn[2][sp] = rl(lev - 1, sp1, x, 0, sp);
              vn[3][sp] = rl(lev - 1, sm1, x, 0, sp);
            } else if (s == 0) {
              vn[0][sp] = rl(lev - 1, s0, x, 1, sp);
              vn[1][sp] = rl(lev - 1, sm1, x + 1, 1, sp);
              vn[2][sp] = rl(lev - 1, sm1, x, 1, sp);
            } else {
              vn[0][sp] = rl(lev - 1, s0, x, 0, sp);
              vn[1][sp] = rl(lev - 1, sp1, x - 1, 0, sp);
              vn[2][sp] = rl(lev - 1, sp1, x, 0, sp);
            }
          }
          const P vo = rl(lev - 1, s0, x, s, sp_t);
          const P wo = (lev == 2) ? r0((p + 3) & 3, x, s, sp_t) : rl(lev >= 3 ? lev - 2 : 1, p, x, s, sp_t);
          P o, g;
          chain_site<T, KIND, MODE>((T)2, (T)1, true, C, ons_h[2 * lev - 3], A.vel_scale, alive_h[2 * lev - 3], vo,
                                    wo, vn, o, g);
          if (lev < KS) rl(lev, p, x, s, sp_t) = o;
          emit(lev, yl[lev], inner && (uint32_t)(j - (2 * lev - 1)) < (uint32_t)ty, o, g);
        } else {
          emit_none(own[p & 1]);
        }
      }
      // Level 1 (row y0 + j - 1) from v_n rows y0 + j - 2 .. y0 + j.
      if (j <= ty + KS - 1) {
        constexpr int sp1 = (p + 2) & 3, s0 = (p + 1) & 3, sm1 = p;
        P vn[NNB][NSPIN];
#pragma unroll
        for (int sp = 0; sp < NSPIN; ++sp) {
          if constexpr (KIND == KPM_SQUARE) {
            vn[0][sp] = r0(s0, x + 1, 0, sp);
            vn[1][sp] = r0(s0, x - 1, 0, sp);
            vn[2][sp] = r0(sp1, x, 0, sp);
            vn[3][sp] = r0(sm1, x, 0, sp);
          } else if (s == 0) {
            vn[0][sp] = r0(s0, x, 1, sp);
            vn[1][sp] = r0(sm1, x + 1, 1, sp);
            vn[2][sp] = r0(sm1, x, 1, sp);
          } else {
            vn[0][sp] = r0(s0, x, 0, sp);
            vn[1][sp] = r0(sp1, x - 1, 0, sp);
            vn[2][sp] = r0(sp1, x, 0, sp);
          }
        }
        const P vo = r0(s0, x, s, sp_t);
        P o, g;
        chain_site<T, KIND, MODE>(A.a1, A.b1, A.read_w1 != 0, C, ons1, A.vel_scale, alive1, vo, w1, vn, o, g);
        rl(1, p, x, s, sp_t) = o;
        emit(1, yl[1], inner && (uint32_t)(j - 1) < (uint32_t)ty, o, g);
      } else {
        emit_none(own[p & 1]);
      }
      // Site-data history: after the shift, entry k holds the site data of row y0 + j - k - 1.
#pragma unroll
      for (int k = NH - 1; k > 0; --k) {
        ons_h[k] = ons_h[k - 1];
        alive_h[k] = alive_h[k - 1];
      }
      ons_h[0] = ons1;
      alive_h[0] = alive1;
      yf = next_row(yf);
      ys = next_row(ys);
#pragma unroll
      for (int l = 1; l <= KS; ++l) yl[l] = next_row(yl[l]);
    };
    // Prologue: v_n rows y0 - KS and y0 - KS + 1 into slots 0 and 1, then the first row's loads
    // followed by KS sets of dropped stores, the pattern every later row sees.
    fetch(0, wrap(y0 - KS), wrap(y0 - KS), true);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store_row(0, 0);
    fetch(1, wrap(y0 - KS + 1), wrap(y0 - KS + 1), true);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store_row(1, 1);
    fetch(0, wrap(y0 + j0), wrap(y0 + j0 - 1), true);
#pragma unroll
    for (int k = 0; k < KS; ++k) emit_none(own[1]);
    for (int j = j0; j <= j_last; j += 4) {
      row(std::integral_constant<int, 0>{}, j);
      row(std::integral_constant<int, 1>{}, j + 1);
      row(std::integral_constant<int, 2>{}, j + 2);
      row(std::integral_constant<int, 3>{}, j + 3);
    }
    __syncthreads();   // the next tile reuses the rings
  }
}

template <typename T, int KIND, int KS>
static void* pick_chain_mode(int mode, bool split) {
  if constexpr (sizeof(T) == 4) {
    if (split)
      return mode == 0 ? (void*)chain_sweep_kernel<T, KIND, KS, 0, true> : (void*)chain_sweep_kernel<T, KIND, KS, 1, true>;
  }
  return mode == 0 ? (void*)chain_sweep_kernel<T, KIND, KS, 0, false> : (void*)chain_sweep_kernel<T, KIND, KS, 1, false>;
}

template <typename T, int KIND>
static void* pick_chain_ks(int ks, int mode, bool split) {
  if (ks == 2) return pick_chain_mode<T, KIND, 2>(mode, split);
  if (ks == 3) return pick_chain_mode<T, KIND, 3>(mode, split);
  return pick_chain_mode<T, KIND, 4>(mode, split);
}

void* chain_kernel_fn(int prec, int kind, int ks, int mode, bool split) {
  if (ks < 2 || ks > 4 || (mode != 0 && mode != 1) || (split && prec != KPM_FP32)) return nullptr;
  if (prec == KPM_FP32) {
    if (kind == KPM_HONEYCOMB) return pick_chain_ks<float, KPM_HONEYCOMB>(ks, mode, split);
    if (kind == KPM_HONEYCOMB_SPIN) return pick_chain_ks<float, KPM_HONEYCOMB_SPIN>(ks, mode, split);
    return pick_chain_ks<float, KPM_SQUARE>(ks, mode, split);
  }
  if (kind == KPM_HONEYCOMB) return pick_chain_ks<double, KPM_HONEYCOMB>(ks, mode, false);
  if (kind == KPM_HONEYCOMB_SPIN) return pick_chain_ks<double, KPM_HONEYCOMB_SPIN>(ks, mode, false);
  return pick_chain_ks<double, KPM_SQUARE>(ks, mode, false);
}

}  // namespace kpm

// ---------------------------------------------------------------------------
// Host side: launch shape, tile list, sweep loop.
// ---------------------------------------------------------------------------
#include "kpm_plan.h"

#include <algorithm>
#include <climits>

namespace kpm {

int chain_plan_create(const kpm_plan* P, int ks, int rows, int64_t blk_rows, ChainPlan* C) {
  *C = ChainPlan();
  KPM_CHECK_ARG(ks >= 2 && ks <= 4, "chain sweep: 2..4 steps per sweep");
  KPM_CHECK_ARG(P->n_lat == 1, "chain sweep: one lattice per plan");
  // The spinful FP64 kernel spills registers at four steps per sweep.
  if (P->prec == KPM_FP64 && P->n_spin == 2) ks = std::min(ks, 3);
  int lds_max = 65536;
  {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      lds_max = v;
  }
  const int nsub = P->n_sub, nspin = P->n_spin;
  // A tile covers up to 128 contiguous bytes of each site (8 chunks spinless, 4 chunks per spin).
  const int ew = (int)std::min<int64_t>(P->E, nspin == 2 ? 4 : 8);
  // The largest workgroup whose rings fit the LDS with at least 4 KS thread columns.
  int block = 0, tx = 0;
  size_t lds = 0;
  for (int b = kMaxStepBlock; b >= 64; b -= 64) {
    const int t = b / (nsub * nspin * ew);   // a thread per orbital
    // Rings plus one spare cell: the surplus threads of column Tx read one cell past the last row.
    const size_t r = ((size_t)4 * ks * (t + 2) + 1) * nsub * nspin * ew * 16;
    if (t >= 4 * ks && r <= (size_t)lds_max) {
      block = b;
      tx = t;
      lds = r;
      break;
    }
  }
  if (block == 0) {
    set_error("chain sweep: no tile shape fits %d bytes of LDS", lds_max);
    return KPM_E_UNSUPPORTED;
  }
  const kpm_lattice_t& L = P->lats[0];
  // The kernels address a lattice row of a vector, and the Gamma store rows of
  // one lattice row, with 32-bit byte offsets.
  const double row_cplx = (double)L.L1 * nsub * nspin * P->Rp;
  if (row_cplx * 2 * P->tsize >= 2147483648.0 || (double)P->n_orb * P->Rp >= 4294967296.0 ||
      (row_cplx / kBlkK + 2) * (double)blk_rows * kBlkK * 2 * P->tsize >= 2147483648.0) {
    set_error("chain sweep: lattice rows too long for 32-bit offsets");
    return KPM_E_UNSUPPORTED;
  }
  const int xstep = tx - 2 * (ks - 1);
  const int n_rg = (int)ceil_div(P->E, ew);
  // Rows per tile: the fewest rounds of concurrent workgroups, each round costing the tile's
  // rows plus the 3 (KS - 1) iterations of its skewed start and drain.
  int n_cu = 256;
  {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n_cu = v;
  }
  const int per_cu = std::max(1, std::min(kMaxStepBlock * 4 / block, (int)(lds_max / lds)));
  const int64_t conc = (int64_t)n_cu * per_cu;
  int best_ty = rows;
  double best_cost = 1e300;
  for (int ty : {256, 192, 128, 96, 64, 48, 32, 16, 8}) {
    if (rows > 0) break;   // rows given
    const int64_t nt = (int64_t)n_rg * ceil_div(L.L2, ty) * ceil_div(L.L1, xstep);
    const int64_t rounds = ceil_div(nt, conc);
    const double cost = (double)rounds * (double)(ceil_div(std::min(ty, L.L2) + 3 * (ks - 1), 4) * 4);
    if (cost < best_cost * 0.999) {
      best_cost = cost;
      best_ty = ty;
    }
  }
  std::vector<int4> tiles;
  for (int g = 0; g < n_rg; ++g)
    for (int y0 = 0; y0 < L.L2; y0 += best_ty)
      for (int x0 = 0; x0 < L.L1; x0 += xstep) tiles.push_back(make_int4(0, g, x0, y0));
  C->ks = ks;
  C->block = block;
  C->Tx = tx;
  C->Ty = best_ty;
  C->Ew = ew;
  C->lds_bytes = lds;
  C->n_tiles = (int)tiles.size();
  C->grid = (int)(ceil_div(std::min<int64_t>((int64_t)tiles.size(), conc), 8) * 8);
  for (int m = 0; m < 2; ++m)
    for (int sp = 0; sp < 2; ++sp) C->fn[m][sp] = chain_kernel_fn(P->prec, P->kind, ks, m, sp == 1);
  const size_t vec_bytes = (size_t)P->n_orb * P->Rp * 2 * P->tsize;
  hipError_t e = dev_malloc(&C->tiles, tiles.size() * sizeof(int4));
  if (e == hipSuccess) e = dev_malloc(&C->Z, vec_bytes);
  if (e == hipSuccess) e = dev_malloc(&C->W, vec_bytes);
  if (e == hipSuccess)
    e = KPM_HIP(hipMemcpy(C->tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice));
  if (e != hipSuccess) {
    set_error("chain sweep setup: %s", hipGetErrorString(e));
    (void)hipGetLastError();
    chain_plan_free(C);
    return hip_status(e);
  }
  return KPM_OK;
}

void chain_plan_free(ChainPlan* C) {
  (void)dev_free(C->tiles);
  (void)dev_free(C->Z);
  (void)dev_free(C->W);
  C->tiles = nullptr;
  C->Z = C->W = nullptr;
}

template <typename T>
static hipError_t chain_launch(const kpm_plan* P, const ChainPlan& C, hipStream_t s, int mode, const void* v,
                               const void* w, void* out_a, void* out_b, bool first, int nlev, void* blk, void* blk_lo,
                               int64_t row0, int64_t blk_rows, int vdir, double vel_scale) {
  ChainArgs<T> a;
  a.lats = (const LatDev<T>*)P->latdev;
  a.tiles = C.tiles;
  a.n_tiles = C.n_tiles;
  a.v = (const T*)v;
  a.w = (const T*)w;
  a.out_a = (T*)out_a;
  a.out_b = (T*)out_b;
  a.onsite = (const T*)P->onsite;
  a.mask = P->mask;
  a.phase = (const T*)P->phase;
  a.blk = (T*)blk;
  a.blk_lo = (__bf16*)blk_lo;
  a.blk_row0 = row0;
  a.blk_rows = blk_rows;
  a.a1 = first ? (T)1 : (T)2;
  a.b1 = first ? (T)0 : (T)1;
  a.vel_scale = (T)vel_scale;
  a.read_w1 = first ? 0 : 1;
  a.nlev = nlev;
  a.vdir = vdir;
  a.has_onsite = P->has_onsite ? 1 : 0;
  a.has_mask = P->has_mask ? 1 : 0;
  a.has_phase = P->has_phase ? 1 : 0;
  a.Tx = C.Tx;
  a.Ty = C.Ty;
  a.E = P->E;
  a.Ew = C.Ew;
  a.Rp = P->Rp;
  void* args[] = {&a};
  void* fn = C.fn[mode][blk_lo != nullptr ? 1 : 0];
  if (fn == nullptr) return hipErrorInvalidDeviceFunction;
  return after_call(hipLaunchKernel(fn, dim3(C.grid), dim3(C.block), args, C.lds_bytes, s));
}

hipError_t chain_run(const kpm_plan* P, const ChainPlan& C, hipStream_t s, int mode, void* v0, void* w0,
                     int n_levels, void* blk, void* blk_lo, int64_t blk_rows, int vdir, double vel_scale,
                     double* bytes) {
  if (mode != 0 && mode != 1) return hipErrorInvalidValue;
  const double vec_b = (double)P->n_orb * P->Rp * 2 * P->tsize;
  const double site_b = (P->has_onsite ? (double)P->n_sites * P->tsize : 0.0) + (P->has_mask ? (double)P->n_sites : 0.0);
  void* cur = v0;
  void* prev = w0;
  void* fa = C.Z;
  void* fb = C.W;
  double moved = 0.0;
  for (int k = 0; k < n_levels; k += C.ks) {
    const int nlev = std::min(C.ks, n_levels - k);
    const bool first = k == 0;
    const hipError_t e =
        P->prec == KPM_FP32
            ? chain_launch<float>(P, C, s, mode, cur, prev, fa, fb, first, nlev, blk, blk_lo, k, blk_rows, vdir, vel_scale)
            : chain_launch<double>(P, C, s, mode, cur, prev, fa, fb, first, nlev, blk, blk_lo, k, blk_rows, vdir,
                                   vel_scale);
    if (e != hipSuccess) return e;
    // v_n (and v_{n-1} after the first sweep) in, the last two levels out, a block row per level.
    moved += vec_b * ((first ? 1.0 : 2.0) + (nlev >= 2 ? 2.0 : 1.0) + nlev) + site_b;
    void* oc = cur;
    void* op = prev;
    cur = fb;
    prev = fa;
    fa = oc;
    fb = op;
  }
  if (bytes) *bytes += moved;
  return hipSuccess;
}

}  // namespace kpm
