// Internal plan of libkpm (DOS/LDOS and conductivity chains).  Not part of the ABI.
#pragma once

#include "kpm_internal.h"

#include <vector>

namespace kpm {
struct ModelLat;
struct PhaseLat;

// One launch of the Chebyshev step kernel over the plan's tile list.
struct StepLaunch {
  const void* v = nullptr;     // v_n
  const void* w = nullptr;     // v_{n-1}
  void* out = nullptr;         // v_{n+1}
  bool velocity = false;       // compute the velocity stencil h~^vdir v_n
  void* vel = nullptr;         // its standard-layout output (nullptr = not stored)
  void* blk = nullptr;         // K-blocked store (Gamma blocks), nullptr = none
  void* blk_lo = nullptr;      // non-null: store split BF16, hi plane in blk, lo plane here (FP32 only)
  int blk_src = 0;             // 0: store v_{n+1}, 1: store the velocity
  int64_t blk_row = 0, blk_rows = 0;
  double a = 2.0, b = 1.0;     // v_{n+1} = a H~ v_n - b v_{n-1}
  double vel_scale = 1.0;
  int read_w = 1, write_out = 1, dots = 1;
  int vdir = 0;                // velocity stencil: 0 x, 1 y ([r^a, H]); 2 xx, 3 xy, 4 yy ([r^a, [r^b, H]])
  double* part = nullptr;      // moment slots for this step (dots)
};

hipError_t plan_launch_step(kpm_plan* P, hipStream_t s, const StepLaunch& L);

// Multi-step sweeps of the conductivity chains (kpm_chain.hip) over a plan's
// lattice, site arrays and vector buffers X, Y: a tile list of their own, two
// more vector buffers, and the launch shape.
struct ChainPlan {
  int ks = 0, block = 0, Tx = 0, Ty = 0, Ew = 0, grid = 0, n_tiles = 0;
  size_t lds_bytes = 0;
  int4* tiles = nullptr;
  void* Z = nullptr;
  void* W = nullptr;
  void* fn[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [mode 0 levels / 1 velocities][split BF16]
};
// ks = steps per sweep (2..4), rows = rows per tile (0: chosen here),
// blk_rows = rows of the Gamma store.  KPM_E_UNSUPPORTED when no tile shape
// fits the LDS or a lattice row is too long for 32-bit offsets (the caller
// then runs single steps).
int chain_plan_create(const kpm_plan* P, int ks, int rows, int64_t blk_rows, ChainPlan* C);
void chain_plan_free(ChainPlan* C);
// n_levels recursion levels from level 0 in v0 (level 1 = H~ v0, then 2 H~ v - w),
// with one Gamma block row per level: mode 0 stores levels 1..n_levels into rows
// 1..n_levels; mode 1 stores the velocity vel_scale [r^vdir, H] of levels
// 0..n_levels-1 into rows 0..n_levels-1.  w0 is a free vector buffer (X or Y).
// *bytes receives the algorithmic HBM bytes moved.
hipError_t chain_run(const kpm_plan* P, const ChainPlan& C, hipStream_t s, int mode, void* v0, void* w0,
                     int n_levels, void* blk, void* blk_lo, int64_t blk_rows, int vdir, double vel_scale,
                     double* bytes);
hipError_t plan_launch_prep(kpm_plan* P, hipStream_t s);
int plan_set_vector_base(kpm_plan* P, int64_t r0);
// arena_get != nullptr: after the arguments are validated, arena_get supplies a device arena of
// arena_cap bytes; every device buffer is carved from it instead of hipMalloc, and no stream, event
// or graph is created (the allocation-free entry point).
int plan_create(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p, const kpm_tune_t* tune,
                kpm_plan** out, int (*arena_get)(char**) = nullptr, size_t arena_cap = 0);
void plan_free(kpm_plan* P);
bool tune_cache_lookup(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p, kpm_tune_t* t);
double cell_area_nm2(int kind);
}  // namespace kpm

struct kpm_plan {
  std::vector<kpm_lattice_t> lats;
  kpm_dos_params_t p;
  std::vector<int64_t> sites;
  int n_lat = 0, kind = 0, prec = 0, n_sub = 0, n_spin = 0;
  int M = 0, R = 0, Rp = 0, NC = 0, E = 0, Ew = 0, n_rg = 0, Tx = 0, Ty = 0, block = 0, grid = 0;
  int n_steps = 0, n_tiles = 0, n_slots = 0, steps_per_chunk = 0;
  bool has_onsite = false, has_mask = false, has_phase = false, use_graph = true;
  int64_t n_orb = 0, n_sites = 0, n_phase = 0;
  std::vector<int64_t> site_off, vec_off, phase_off;
  size_t tsize = 0;
  // device memory
  void* X = nullptr;
  void* Y = nullptr;
  void* Z = nullptr;           // two more vectors for the multi-step sweep kernels (variants 3-6)
  void* W = nullptr;
  void* onsite = nullptr;
  uint8_t* mask = nullptr;
  void* phase = nullptr;
  void* latdev = nullptr;
  int4* tiles = nullptr;
  int* slot_of = nullptr;
  int2* ranges = nullptr;
  double* part = nullptr;
  double* dots = nullptr;
  uint64_t* keys = nullptr;
  int64_t* d_sites = nullptr;
  unsigned long long* active = nullptr;
  kpm::ModelLat* mlat = nullptr;
  kpm::PhaseLat* plat = nullptr;
  int* flag = nullptr;
  double* mu_dev = nullptr;
  double* mean_dev = nullptr;
  void* step_fn = nullptr;
  void* step_fn_vel = nullptr;
  void* sweep_fn = nullptr;    // multi-step sweep kernel (variants 3-6)
  int variant = 2;             // 1 = direct-load step kernel, 2 = LDS row ring, 3..6 = 2..5 steps per sweep
  int sweep = 1;               // Chebyshev steps per launch (variant - 1 for the sweep kernels, else 1)
  size_t lds_bytes = 0;
  int64_t r_base = 0;          // global index of the plan's first random vector
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_loop = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
  double bytes_per_step = 0.0;
  int64_t n_active_total = 0;
  // Caller-provided device memory that the buffers above are carved from (nullptr: hipMalloc).
  bool use_arena = false;
  char* arena_base = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  size_t dev_bytes = 0;   // device bytes of the plan's buffers
};


