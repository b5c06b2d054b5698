// Multi-step Chebyshev sweeps (temporal blocking) on gfx950.
//
// Paper passages: eq. e6 (matrix Chebyshev recursion), Sec. 2(c) (stochastic
// trace: moments from random vectors), Sec. 3(a) (matrix-free pattern-rule
// Hamiltonian), Sec. 3(b) and Table 1 (tiles of the lattice processed as a
// unit; the TILE blocking).  The layout of vectors, tiles and moment slots is
// that of the single-step kernels in kpm_dos.hip.

#include "kpm_stencil.h"

#include <type_traits>

namespace kpm {

// ---------------------------------------------------------------------------
// KS Chebyshev steps per sweep (temporal blocking) for the spinless lattices
// (with or without Peierls phases): level l = 1..KS of a sweep is v_{n+l},
//     v_{n+1} = a1 H~ v_n - b1 v_{n-1},   v_{n+l} = 2 H~ v_{n+l-1} - v_{n+l-2},
// with the doubling dot products of every step, from one pass over v_n and
// v_{n-1}.  Only the last two levels go back to HBM (the next sweep starts
// from them), so per KS steps HBM moves two vectors in and two out, instead
// of three per step.
//
// A tile is a band of Tx - 2 (KS - 1) interior cell columns and Ty rows of
// one (lattice, r-group).  The workgroup's Tx thread columns cover the
// interior plus KS - 1 columns on each side: level l is formed on thread
// columns [l - 1, Tx - l] (each level needs one neighbour column more than
// the next), so level KS covers the interior; v_n comes with one more halo
// column per side.  Rows are marched upwards: at iteration j, row y0 + j of
// v_n enters a 4-slot LDS ring and level l forms row y0 + j - (2 l - 1) into
// a 4-slot ring of its own (the last level only to HBM), so that the levels of
// one iteration read only rows formed in earlier iterations: one barrier per
// row.  The outputs go to buffers that no tile reads in the same sweep
// (neighbouring tiles still read v_n and v_{n-1} on halos).  nlev < KS runs the
// first nlev levels only (the last, short sweep of a recursion).
// ---------------------------------------------------------------------------

// out = a (H~ v)_i - b w_i at one site (one spin), and, when acc (a uniform
// condition: the row belongs to the tile), the doubling dot products <v|v>,
// <out|v> added to the FP64 sums pv, pw.  The products are formed in FP64
// from the vectors' values (exact for FP32 vectors).  Threads outside the
// tile's interior add values that may be anything (NaN included); their sums
// are discarded once per tile.  With PHASE the neighbour k enters with the
// complex coefficient (hre[k], him[k]) = hop exp(i theta_k) of the site's
// column, else with hop.
template <typename T, int KIND, bool PHASE>
__device__ inline void sweep_site(T a, T b, bool read_w, T hop, const T* hre, const T* him, T ons, bool alive,
                                  const Pack<T>& vo, const Pack<T>& wo, const Pack<T> (&vn)[KindTraits<KIND>::NNB],
                                  Pack<T>& out, bool acc, double* pv, double* pw) {
  constexpr int NC = Pack<T>::NC;
  constexpr int NNB = KindTraits<KIND>::NNB;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    T hr = ons * vo.v[2 * j], hi = ons * vo.v[2 * j + 1];
#pragma unroll
    for (int k = 0; k < NNB; ++k) {
      if constexpr (PHASE) {
        cmul_acc(hr, hi, hre[k], him[k], vn[k].v[2 * j], vn[k].v[2 * j + 1]);
      } else {
        hr += hop * vn[k].v[2 * j];
        hi += hop * vn[k].v[2 * j + 1];
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
    }
    out.v[2 * j] = orr;
    out.v[2 * j + 1] = oi;
  }
  // One uniform branch for all of the site's products.
  if (acc) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const double xr = vo.v[2 * j], xi = vo.v[2 * j + 1];
      pv[j] = fma(xr, xr, fma(xi, xi, pv[j]));
      pw[j] = fma((double)out.v[2 * j], xr, fma((double)out.v[2 * j + 1], xi, pw[j]));
    }
  }
}

// SHAPE 0: the tile shape (chunks per site Ew, thread columns Tx) comes from
// the arguments.  SHAPE 1: 512 threads, 8 chunks per site (the shape the
// benchmarked workloads run): compile-time constants, so every LDS ring
// offset is an instruction immediate instead of an address register.
template <typename T, int KIND, bool ONSITE, bool MASK, bool PHASE, int KS, int SHAPE = 0>
__global__ void __launch_bounds__(kMaxStepBlock) sweep_kernel(SweepArgs<T> A) {
  using P = Pack<T>;
  constexpr int NC = P::NC;
  constexpr int NSUB = KindTraits<KIND>::NSUB;
  constexpr int NNB = KindTraits<KIND>::NNB;
  static_assert(KindTraits<KIND>::NSPIN == 1, "spinless lattices only");
  static_assert(!PHASE || KIND == KPM_HONEYCOMB, "Peierls phases on the honeycomb lattice only");
  static_assert(KS >= 2 && KS <= kMaxSweep, "2..kMaxSweep steps per sweep");
  constexpr int NH = 2 * KS - 1;   // site-data history: level l uses the entry 2 (l - 1) iterations old
  // Rows of loads in flight, register sets (a divisor of the 4-row unroll),
  // and the vector-memory count a row waits for: after a row's loads come
  // its two stores and then, for each later row in flight, its loads and two
  // stores.  Two rows ahead measured no faster than one (the kernel is not
  // waiting on load latency) and costs 14 registers: one row ahead.
  constexpr int kPrefetch = 1;
  constexpr int kSets = 2;
  constexpr int kLoads = 3 + (ONSITE ? 1 : 0) + (MASK ? 1 : 0);
  constexpr int kWaitVm = 2 + (kPrefetch - 1) * (kLoads + 2);
  static_assert(kPrefetch < kSets && 4 % kSets == 0 && kWaitVm < 16, "register sets and wait count");
  extern __shared__ double lds[];

  const int tid = threadIdx.x;
  constexpr int kShapeEw = 8, kShapeBlock = 512;
  const int Ew = SHAPE ? kShapeEw : A.Ew;
  const int cl = tid % Ew;
  const int grp = tid / Ew;
  const int n_grp = (SHAPE ? kShapeBlock : (int)blockDim.x) / Ew;
  const int s = grp % NSUB;
  const int xl = grp / NSUB;
  const int Rp = A.Rp;
  const int Tx = SHAPE ? kShapeBlock / (NSUB * kShapeEw) : A.Tx;
  const int nlev = A.nlev;
  // v_n ring: [4 slots][Tx + 2 cells][sub][chunk] (cell = thread column + 1,
  // halos in cells 0 and wcols + 1); level l (1..KS-1) ring: the same shape;
  // one spare cell after the last ring.  The moment flush reuses the same LDS
  // between tiles.
  P* ring0 = reinterpret_cast<P*>(lds);
  const int row0 = (Tx + 2) * NSUB * Ew;
  P* ringl = ring0 + 4 * row0;
  const int rowl = row0;
  // Every thread computes every level of every active iteration: no branch
  // on its column.  Results of columns outside a level's range are garbage
  // that no thread of the next level reads.  Threads beyond the last whole
  // thread column (when Ew does not divide the workgroup) work on column Tx:
  // they write only cell Tx + 1, which is never read.
  const int xlc = (grp < n_grp) ? xl : Tx;
  auto r0 = [&](int slot, int cell, int sub) -> P& { return ring0[slot * row0 + (cell * NSUB + sub) * Ew + cl]; };
  auto rl = [&](int lev, int slot, int cell, int sub) -> P& {
    return ringl[((lev - 1) * 4 + slot) * rowl + (cell * NSUB + sub) * Ew + cl];
  };

  const int xcd = blockIdx.x & 7;
  const int jx = blockIdx.x >> 3;
  const int gx = gridDim.x >> 3;
  const int t_begin = (int)(((int64_t)xcd * A.n_tiles) >> 3);
  const int t_end = (int)(((int64_t)(xcd + 1) * A.n_tiles) >> 3);

  // The doubling dot products of each level, summed in FP64 over the thread's
  // sites: tv, tw over the current tile (every thread, garbage outside the
  // interior), vv, wv over the tiles of the current moment slot (interior
  // threads' tile sums only).
  double vv[KS][NC], wv[KS][NC], tv[KS][NC], tw[KS][NC];
#pragma unroll
  for (int l = 0; l < KS; ++l)
#pragma unroll
    for (int j = 0; j < NC; ++j) vv[l][j] = wv[l][j] = tv[l][j] = tw[l][j] = 0.0;
  // The two levels that go to HBM (levels nlev - 1 and nlev), kept from the
  // level loop until the row's two stores.
  P o_a = {}, o_b = {};

  for (int ti = t_begin + jx; ti < t_end; ti += gx) {
    const int4 tl = A.tiles[ti];
    const LatDev<T>& Lg = A.lats[tl.x];
    const int L1 = Lg.L1, L2 = Lg.L2;
    const int64_t site_off = Lg.site_off;
    const T hop = Lg.hop, ons_c = Lg.onsite_const;
    const int x0 = tl.z, y0 = tl.w;
    const int n_in = min(Tx - 2 * (KS - 1), L1 - x0);   // interior columns of this tile
    const int wcols = n_in + 2 * (KS - 1);              // thread columns in use
    int xe = (x0 - (KS - 1)) % L1;                       // column of thread column 0
    if (xe < 0) xe += L1;
    const int n1 = (xe + xl) % L1;
    // Hopping coefficients of this thread's column (Peierls phases depend on n1
    // only; the table is indexed by the A site's cell: a B site's bond class 1
    // goes to the A site of column n1 - 1, and the B side takes the conjugate).
    T hre[3], him[3];
    if constexpr (PHASE) {
      const int n1m = (n1 == 0) ? L1 - 1 : n1 - 1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int na = (s == 0 || k != 1) ? n1 : n1m;
        const T* ph = A.phase + 2 * (Lg.phase_off + (int64_t)na * 3 + k);
        hre[k] = hop * ph[0];
        him[k] = (s == 0) ? hop * ph[1] : -hop * ph[1];
      }
    }
    const int c = tl.y * Ew + cl;
    const bool lane_ok = (grp < n_grp) && (c < A.E);
    const bool act = lane_ok && (xl < wcols);
    const bool inner = act && (xl >= KS - 1) && (xl <= wcols - KS);
    const int64_t coff = (int64_t)c * NC * 2;
    const T* __restrict__ vb = A.v + Lg.vec_off;
    const T* __restrict__ wb = A.w + Lg.vec_off;
    T* __restrict__ oa = A.out_a + Lg.vec_off;
    T* __restrict__ ob = A.out_b + Lg.vec_off;
    // Halo cells of v_n: left of thread column 0, right of thread column wcols - 1.
    const int hl = (xe == 0) ? L1 - 1 : xe - 1;
    const int hr = (xe + wcols) % L1;
    const bool load_left = lane_ok && (xl == 0) && (KIND == KPM_SQUARE || s == 0);
    const bool load_right = lane_ok && (xl == wcols - 1) && (KIND == KPM_SQUARE || s == 1);
    // Row index modulo L2 (used once per tile; rows then advance by one per
    // iteration and wrap with one comparison).
    auto wrap = [&](int y) {
      while (y < 0) y += L2;
      while (y >= L2) y -= L2;
      return y;
    };
    auto next_row = [&](int y) { return (y + 1 == L2) ? 0 : y + 1; };
    // Everything a row needs from HBM (v_n with halos, v_{n-1}, on-site
    // potential and vacancy flag of level 1's row) is loaded into registers
    // kPrefetch iterations ahead, as one group: the levels themselves only
    // touch LDS and store.  The register sets rotate with the row phase
    // (kPrefetch + 1 of them live at a time).  A thread loads at most one
    // halo cell (a sweep tile has at least three thread columns, and on the
    // honeycomb lattice only sublattice 0 needs the left halo and only
    // sublattice 1 the right one).
    struct RowSet {
      P own, halo, w;
      T ons;
      bool alive;
    };
    RowSet set[kSets];
    const bool load_halo = load_left || load_right;
    const int halo_col = load_left ? hl : hr;
    const int halo_cell = load_left ? 0 : wcols + 1;
    // Byte offsets within a lattice row (a row holds < 2^31 bytes), kOOB for
    // threads without data.
    const int64_t row_elems = (int64_t)L1 * NSUB * Rp * 2;
    const int64_t row_sites = (int64_t)L1 * NSUB;
    const uint32_t row_bytes = (uint32_t)(row_elems * (int64_t)sizeof(T));
    const uint32_t lane_b = (uint32_t)((((int64_t)n1 * NSUB + s) * Rp * 2 + coff) * (int64_t)sizeof(T));
    const uint32_t halo_b = (uint32_t)((((int64_t)halo_col * NSUB + s) * Rp * 2 + coff) * (int64_t)sizeof(T));
    const uint32_t lane_site = (uint32_t)(n1 * NSUB + s);
    const uint32_t off_own = act ? lane_b : kOOB;
    const uint32_t off_halo = load_halo ? halo_b : kOOB;
    const uint32_t off_ons = act ? lane_site * (uint32_t)sizeof(T) : kOOB;
    const uint32_t off_mask = act ? lane_site : kOOB;
    // Loads of one row of v_n (when in range) and of the site data and v_{n-1}
    // of the row below it; out of range, the same instructions with kOOB.
    auto fetch = [&](RowSet& S, int yv, int ys, bool in_range) {
      const __amdgpu_buffer_rsrc_t rv = row_rsrc(row_ptr(vb, yv, row_bytes), row_bytes);
      const __amdgpu_buffer_rsrc_t rw = row_rsrc(row_ptr(wb, ys, row_bytes), row_bytes);
      S.own = buf_ld_pack<T>(rv, in_range ? off_own : kOOB);
      S.halo = buf_ld_pack<T>(rv, in_range ? off_halo : kOOB);
      S.w = buf_ld_pack<T>(rw, in_range ? off_own : kOOB);
      const uint32_t ons_row_bytes = (uint32_t)(row_sites * (int64_t)sizeof(T));
      if constexpr (ONSITE) {
        S.ons = buf_ld_scalar<T>(row_rsrc(row_ptr(A.onsite + site_off, ys, ons_row_bytes), ons_row_bytes),
                                 in_range ? off_ons : kOOB);
      } else {
        S.ons = ons_c;
      }
      if constexpr (MASK) {
        S.alive = __builtin_amdgcn_raw_buffer_load_b8(row_rsrc(row_ptr(A.mask + site_off, ys, (uint32_t)row_sites),
                                                                (uint32_t)row_sites),
                                                      in_range ? off_mask : kOOB, 0, 0) != 0;
      } else {
        S.alive = true;
      }
    };
    auto fetch_v = [&](RowSet& S, int yv) {
      const __amdgpu_buffer_rsrc_t rv = row_rsrc(row_ptr(vb, yv, row_bytes), row_bytes);
      S.own = buf_ld_pack<T>(rv, off_own);
      S.halo = buf_ld_pack<T>(rv, off_halo);
    };
    auto store_row = [&](const RowSet& S, int slot) {
      if (act) r0(slot, xl + 1, s) = S.own;
      if (load_halo) r0(slot, halo_cell, s) = S.halo;
    };
    const int ty = min(A.Ty, L2 - y0);
    // Level l forms row y0 + j - (2 l - 1) at iteration j: it reads rows of
    // level l - 1 formed one, two and three iterations earlier, so the levels
    // of one iteration are independent and one barrier per row suffices.
    // Level l is active for j in [3 l - 1 - KS, ty + KS + l - 2].
    const int j0 = 2 - KS;
    const int j_last = ty + 2 * KS - 2;
    // Iterations of level l (2..KS): l <= nlev and j - (3 l - 1 - KS) in
    // [0, lev_cnt), one unsigned comparison per level and row (levels above
    // nlev get a count of 0).  Level l forms row y0 + j - (2 l - 1), which
    // belongs to the tile when j - (2 l - 1) is in [0, ty).
    uint32_t lev_cnt[KS - 1];
#pragma unroll
    for (int lev = 2; lev <= KS; ++lev) lev_cnt[lev - 2] = (lev <= nlev) ? (uint32_t)(ty + 2 * KS - 2 * lev) : 0u;
    // Level nlev - 1 (stored to out_a) exists when nlev >= 2.
    const uint32_t a_cnt = (nlev >= 2) ? (uint32_t)ty : 0u;
    // Site data of the rows the levels form, as a shift register.  The
    // centre value and w of a level come from this thread's own cell of the
    // LDS rings (no other thread writes that cell before the read).
    T ons_h[NH];
    bool alive_h[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      ons_h[k] = ons_c;
      alive_h[k] = true;
    }
    // Wrapped rows of the current iteration j: yf = y0 + j + kPrefetch (the
    // v_n row fetched), ys = yf - 1 (its site data and v_{n-1}), yb = the row
    // level nlev forms (stored to out_b) and ya = yb + 2 (level nlev - 1,
    // stored to out_a).
    int yf = wrap(y0 + j0 + kPrefetch), ys = wrap(y0 + j0 + kPrefetch - 1), yb = wrap(y0 + j0 - (2 * nlev - 1)),
        ya = wrap(y0 + j0 - (2 * nlev - 3));
    // One iteration with phase p = (j - j0) mod 4: set[p % kSets] holds v_n
    // row y0 + j and the site data of row y0 + j - 1.  v_n row y0 + j sits in
    // LDS slot (p + 2) & 3, the rows level l forms at iteration j in slot p.
    auto row = [&](auto ph, auto full, int j) {
      constexpr int p = decltype(ph)::value;
      // A full sweep (nlev == KS, every launch but the recursion's last) has
      // no level selects: a compile-time level count.
      constexpr bool FULL = decltype(full)::value;
      const int nl = FULL ? KS : nlev;
      RowSet& cur = set[p % kSets];
      RowSet& nxt = set[(p + kPrefetch) % kSets];
      // cur has arrived: everything issued before the last kPrefetch rows'
      // stores and the loads between them is complete (expcnt and lgkmcnt
      // left at their maxima).
      __builtin_amdgcn_s_waitcnt(0x0F70 | kWaitVm);
      store_row(cur, (p + 2) & 3);
#pragma unroll
      for (int k = NH - 1; k > 0; --k) {
        ons_h[k] = ons_h[k - 1];
        alive_h[k] = alive_h[k - 1];
      }
      ons_h[0] = cur.ons;
      alive_h[0] = cur.alive;
      __builtin_amdgcn_sched_barrier(0);
      fetch(nxt, yf, ys, j + kPrefetch <= ty + KS - 1);
      lds_barrier();
      // Levels from the deepest down: level l reads w from level l - 2's ring
      // slot of four iterations back, the slot that level l - 2 refills now.
#pragma unroll
      for (int lev = KS; lev >= 2; --lev) {
        if ((uint32_t)(j - (3 * lev - 1 - KS)) < lev_cnt[lev - 2]) {
          constexpr int sp1 = (p + 3) & 3, s0 = (p + 2) & 3, sm1 = (p + 1) & 3;   // rows y + 1, y, y - 1
          const int x = xlc + 1;   // this thread's cell
          P vn[NNB];
          if constexpr (KIND == KPM_SQUARE) {
            vn[0] = rl(lev - 1, s0, x + 1, 0);
            vn[1] = rl(lev - 1, s0, x - 1, 0);
            vn[2] = rl(lev - 1, sp1, x, 0);
            vn[3] = rl(lev - 1, sm1, x, 0);
          } else if (s == 0) {
            vn[0] = rl(lev - 1, s0, x, 1);
            vn[1] = rl(lev - 1, sm1, x + 1, 1);
            vn[2] = rl(lev - 1, sm1, x, 1);
          } else {
            vn[0] = rl(lev - 1, s0, x, 0);
            vn[1] = rl(lev - 1, sp1, x - 1, 0);
            vn[2] = rl(lev - 1, sp1, x, 0);
          }
          const P vo = rl(lev - 1, s0, x, s);   // level lev-1, row y
          // Level lev-2 at row y: v_n row y0 + j - 3 (its slot is refilled by
          // the next iteration's row, from this same thread for its own cell),
          // or level lev-2's output of four iterations back.
          const P wo = (lev == 2) ? r0((p + 3) & 3, x, s) : rl(lev >= 3 ? lev - 2 : 1, p, x, s);
          P o;
          sweep_site<T, KIND, PHASE>((T)2, (T)1, true, hop, hre, him, ons_h[2 * lev - 2], alive_h[2 * lev - 2], vo, wo,
                                     vn, o, (uint32_t)(j - (2 * lev - 1)) < (uint32_t)ty, tv[lev - 1], tw[lev - 1]);
          if (lev < KS) rl(lev, p, x, s) = o;
          // The stored levels: KS and KS - 1 in a full sweep, else nlev and
          // nlev - 1 of the recursion's last, short sweep (element-wise
          // selects: a conditional copy of the whole pack would be kept in
          // scratch memory).
          if (lev == KS) o_b = o;
          if (lev == KS - 1) o_a = o;
          if (!FULL && nl < KS) {
            const bool cb = lev == nl, ca = lev == nl - 1;
#pragma unroll
            for (int q = 0; q < 2 * NC; ++q) {
              o_b.v[q] = cb ? o.v[q] : o_b.v[q];
              o_a.v[q] = ca ? o.v[q] : o_a.v[q];
            }
          }
        }
      }
      // Level 1 (row y0 + j - 1) from v_n rows y0 + j - 2 .. y0 + j.
      {
        if (j <= ty + KS - 1) {
          constexpr int sp1 = (p + 2) & 3, s0 = (p + 1) & 3, sm1 = p;   // v_n rows y + 1, y, y - 1
          const int x = xlc + 1;
          P vn[NNB];
          if constexpr (KIND == KPM_SQUARE) {
            vn[0] = r0(s0, x + 1, 0);
            vn[1] = r0(s0, x - 1, 0);
            vn[2] = r0(sp1, x, 0);
            vn[3] = r0(sm1, x, 0);
          } else if (s == 0) {
            vn[0] = r0(s0, x, 1);
            vn[1] = r0(sm1, x + 1, 1);
            vn[2] = r0(sm1, x, 1);
          } else {
            vn[0] = r0(s0, x, 0);
            vn[1] = r0(sp1, x - 1, 0);
            vn[2] = r0(sp1, x, 0);
          }
          const P vo = r0(s0, x, s);   // v_n row y
          P o;
          sweep_site<T, KIND, PHASE>(A.a1, A.b1, A.read_w1 != 0, hop, hre, him, ons_h[0], alive_h[0], vo, cur.w, vn, o,
                                     (uint32_t)(j - 1) < (uint32_t)ty, tv[0], tw[0]);
          rl(1, p, x, s) = o;
          if constexpr (KS == 2) o_a = o;   // a full two-step sweep stores levels 1 and 2
          if (!FULL && nl <= 2) {
            const bool cb = nl == 1;
#pragma unroll
            for (int q = 0; q < 2 * NC; ++q) {
              o_b.v[q] = cb ? o.v[q] : o_b.v[q];
              o_a.v[q] = cb ? o_a.v[q] : o.v[q];
            }
          }
        }
      }
      // The row's two stores: level nlev at row y0 + j - (2 nlev - 1), level
      // nlev - 1 two rows higher (a thread stores its interior cells of the
      // tile's own rows; every other store is dropped).
      {
        const bool own_b = inner && (uint32_t)(j - (2 * nl - 1)) < (uint32_t)ty;
        const bool own_a = inner && (uint32_t)(j - (2 * nl - 3)) < (FULL ? (uint32_t)ty : a_cnt);
        buf_st_pack<T>(row_rsrc(row_ptr(ob, yb, row_bytes), row_bytes), own_b ? lane_b : kOOB, o_b);
        buf_st_pack<T>(row_rsrc(row_ptr(oa, ya, row_bytes), row_bytes), own_a ? lane_b : kOOB, o_a);
      }
      yf = next_row(yf);
      ys = next_row(ys);
      yb = next_row(yb);
      ya = next_row(ya);
    };
    // Prologue: v_n rows y0 - KS and y0 - KS + 1 into slots 0 and 1, the
    // first iteration's row and site data into registers.
    fetch_v(set[0], wrap(y0 - KS));
    store_row(set[0], 0);
    fetch_v(set[0], wrap(y0 - KS + 1));
    store_row(set[0], 1);
    // The first kPrefetch rows' loads, each followed by two dropped stores:
    // the loop is entered with the same pattern of memory instructions as
    // every later row sees (a row's loads, then that row's two stores), so
    // its waits stay the same.
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
      fetch(set[k], wrap(y0 + j0 + k), wrap(y0 + j0 + k - 1), true);
      const __amdgpu_buffer_rsrc_t rz = row_rsrc(ob, row_bytes);
      buf_st_pack<T>(rz, kOOB, o_b);
      buf_st_pack<T>(rz, kOOB, o_a);
    }
    auto march = [&](auto full) {
      for (int j = j0; j <= j_last; j += 4) {
        row(std::integral_constant<int, 0>{}, full, j);
        row(std::integral_constant<int, 1>{}, full, j + 1);
        row(std::integral_constant<int, 2>{}, full, j + 2);
        row(std::integral_constant<int, 3>{}, full, j + 3);
      }
    };
    // Five-step sweeps keep one copy of the loop: a second would push them
    // further into scratch memory (their rings and levels already use most
    // of the registers).
    if (KS < 5 && nlev == KS)
      march(std::true_type{});
    else
      march(std::false_type{});
    // The tile's sums count for interior threads only (a select: the others' may be NaN).
#pragma unroll
    for (int l = 0; l < KS; ++l)
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        vv[l][q] += inner ? tv[l][q] : 0.0;
        wv[l][q] += inner ? tw[l][q] : 0.0;
        tv[l][q] = tw[l][q] = 0.0;
      }
    __syncthreads();   // the next tile (or the moment flush) reuses the LDS
    const int tn = ti + gx;
    const int slot = A.slot_of[ti];
    if (tn >= t_end || A.slot_of[tn] != slot) {
#pragma unroll
      for (int l = 0; l < KS; ++l)
        if (l < nlev) flush_slot<NC>(lds, A.part[l], slot, tid, Ew, grp, n_grp, vv[l], wv[l]);
    }
  }
}

template <typename T, int KIND, bool PHASE, int KS, int SHAPE = 0>
static void* pick_sweep_ks(bool onsite, bool mask) {
  if (onsite)
    return mask ? (void*)sweep_kernel<T, KIND, true, true, PHASE, KS, SHAPE>
                : (void*)sweep_kernel<T, KIND, true, false, PHASE, KS, SHAPE>;
  return mask ? (void*)sweep_kernel<T, KIND, false, true, PHASE, KS, SHAPE>
              : (void*)sweep_kernel<T, KIND, false, false, PHASE, KS, SHAPE>;
}

template <typename T, int KIND, bool PHASE>
static void* pick_sweep(int ks, bool onsite, bool mask, bool shape1) {
  if (ks == 2) return pick_sweep_ks<T, KIND, PHASE, 2>(onsite, mask);
  if (ks == 3) return pick_sweep_ks<T, KIND, PHASE, 3>(onsite, mask);
  if (ks == 4)
    return shape1 ? pick_sweep_ks<T, KIND, PHASE, 4, 1>(onsite, mask) : pick_sweep_ks<T, KIND, PHASE, 4>(onsite, mask);
  return pick_sweep_ks<T, KIND, PHASE, 5>(onsite, mask);
}

// The square lattice has no Peierls table.
template <typename T>
static void* pick_sweep_kind(int kind, int ks, bool onsite, bool mask, bool phase, bool shape1) {
  if (kind == KPM_SQUARE) return pick_sweep<T, KPM_SQUARE, false>(ks, onsite, mask, shape1);
  return phase ? pick_sweep<T, KPM_HONEYCOMB, true>(ks, onsite, mask, shape1)
               : pick_sweep<T, KPM_HONEYCOMB, false>(ks, onsite, mask, shape1);
}

void* sweep_kernel_fn(int prec, int kind, int ks, bool onsite, bool mask, bool phase, int block, int tx, int ew) {
  const int nsub = kind == KPM_SQUARE ? 1 : 2;
  const bool shape1 = block == 512 && ew == 8 && tx == 512 / (nsub * 8);
  return prec == KPM_FP32 ? pick_sweep_kind<float>(kind, ks, onsite, mask, phase, shape1)
                          : pick_sweep_kind<double>(kind, ks, onsite, mask, phase, shape1);
}

}  // namespace kpm
