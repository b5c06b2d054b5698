// Launch-shape autotuner for the Chebyshev step kernel.
//
// The paper leaves the TILE size of its CPU blocking to the user, who must
// tune it per machine (Sec. 3(b); Sec. 5, Table 1).  Here the analogous
// choices are the kernel variant (one step or 2..5 steps per sweep),
// workgroup size, rows per tile, the site chunks a tile covers and the
// persistent grid; kpm_autotune measures each candidate on the real workload
// (a short recursion of probe_steps steps, timed with hipEvents on the
// caller's stream) and records the fastest in a plain-text cache keyed by
// (lattice kind, precision, padded vectors per orbital, floor(log2 orbitals)).
// kpm_plan_create consults the cache named by the KPM_TUNE_CACHE environment
// variable when the caller passes no launch shape.

#include "kpm_internal.h"
#include "kpm_plan.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace kpm {

struct TuneKey {
  int kind, prec, rp, log2n;
};

static TuneKey make_key(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p) {
  const int n_sub = lat[0].kind == KPM_SQUARE ? 1 : 2;
  const int n_spin = lat[0].kind == KPM_HONEYCOMB_SPIN ? 2 : 1;
  int64_t n_orb = 0;
  for (int l = 0; l < n_lat; ++l) n_orb += (int64_t)lat[l].L1 * lat[l].L2 * n_sub * n_spin;
  const int R = p->start == KPM_START_SITES ? p->num_sites : p->num_random;
  const int nc = p->precision == KPM_FP32 ? 2 : 1;
  TuneKey k;
  k.kind = lat[0].kind;
  k.prec = p->precision;
  k.rp = (R + nc - 1) / nc * nc;
  k.log2n = n_orb > 0 ? (int)std::floor(std::log2((double)n_orb)) : 0;
  return k;
}

static std::mutex g_cache_mu;

// Returns true and fills *t when the cache file has an entry for the key.
bool tune_cache_lookup(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p, kpm_tune_t* t) {
  const char* path = std::getenv("KPM_TUNE_CACHE");
  if (!path || !*path) return false;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  std::ifstream f(path);
  if (!f) return false;
  const TuneKey k = make_key(lat, n_lat, p);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    int kind, prec, rp, lg, kern, block, rows, grid, chunks;
    double gbs;
    if (!(is >> kind >> prec >> rp >> lg >> kern >> block >> rows >> grid >> chunks >> gbs)) continue;
    if (kind == k.kind && prec == k.prec && rp == k.rp && lg == k.log2n) {
      t->kernel = kern;
      t->block = block;
      t->rows = rows;
      t->grid = grid;
      t->chunks = chunks;
      found = true;   // the last matching line wins
    }
  }
  return found;
}

static int tune_cache_store(const char* path, const TuneKey& k, const kpm_tune_t& t, double gbs) {
  if (!path || !*path) return KPM_OK;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  std::ofstream f(path, std::ios::app);
  if (!f) {
    set_error("cannot append to tune cache %s", path);
    return KPM_E_INVALID;
  }
  f << k.kind << ' ' << k.prec << ' ' << k.rp << ' ' << k.log2n << ' ' << t.kernel << ' ' << t.block << ' ' << t.rows
    << ' ' << t.grid << ' ' << t.chunks << ' ' << gbs << '\n';
  return KPM_OK;
}

// Recursion steps per millisecond of one plan run (the candidates run the same
// workload; GB/s would not compare variants that move different bytes per
// step), and the algorithmic GB/s of that run.
static int timed_run(kpm_plan* P, void* stream, double* steps_per_ms, double* gbs) {
  int st = kpm_plan_run(P, nullptr, nullptr, 1, stream);
  if (st != KPM_OK && st != KPM_E_SPECTRUM) return st;
  kpm_plan_info_t info;
  st = kpm_plan_info(P, &info);
  if (st != KPM_OK) return st;
  *steps_per_ms = info.n_steps / info.last_loop_ms;
  if (gbs) *gbs = info.bytes_per_step * info.n_steps / (info.last_loop_ms * 1e-3) / 1e9;
  return KPM_OK;
}

// Two phases: every candidate runs probe_steps steps (after one untimed run
// that also instantiates its graph); the three fastest then run 4 probe_steps
// steps in three rounds (each round times every finalist once), and the best
// median wins.  The second
// phase keeps a short first probe from deciding between shapes a few percent
// apart.
static int autotune(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p, int32_t probe_steps,
                    const char* cache_path, kpm_tune_t* best, double* best_gbs, void* stream) {
  KPM_CHECK_ARG(lat && p && best && n_lat >= 1, "NULL argument");
  KPM_CHECK_ARG(probe_steps >= 2 && probe_steps <= 4096, "probe_steps must be in [2, 4096]");
  kpm_dos_params_t q = *p;
  q.num_moments = 2 * probe_steps;
  // Candidates: the single-step kernels over workgroup size, rows per tile
  // and persistent grid; the sweep kernels over workgroup size, rows per
  // tile and the site chunks a tile covers (the library's choice, 4 and 16:
  // wider and narrower tiles; 448 threads is the largest workgroup whose
  // five-step rings fit in LDS at the library's chunks).  256-row bands
  // (library chunks only) re-read half the halo rows of 128-row ones; they run
  // on a 1024-workgroup grid so that each workgroup still takes several tiles.  Duplicates of an
  // already screened shape and shapes that fell back to fewer steps are
  // skipped.
  struct Cand { int kernel, block, rows, grid, chunks; };
  std::vector<Cand> cands;
  for (int kv : {1, 2})
    for (int b : {256, 512})
      for (int r : {32, 128})
        for (int g : {1024, 2048}) cands.push_back({kv, b, r, g, 0});
  for (int kv : {3, 4, 5, 6})
    for (int b : {256, 448, 512}) {
      if (b == 448 && kv != 6) continue;
      for (int r : {32, 128, 256})
        for (int c : {0, 4, 16})
          if (r < 256 || c == 0) cands.push_back({kv, b, r, r >= 256 ? 1024 : 2048, c});
    }
  std::vector<std::pair<double, kpm_tune_t>> screened;
  std::vector<std::array<int, 5>> seen;   // (variant, block, rows, grid, chunks in use)
  for (const Cand& cd : cands) {
    kpm_tune_t t;
    std::memset(&t, 0, sizeof(t));
    t.kernel = cd.kernel;
    t.block = cd.block;
    t.rows = cd.rows;
    t.grid = cd.grid;
    t.chunks = cd.chunks;
    t.use_graph = 1;
    kpm_plan* P = nullptr;
    int st = plan_create(lat, n_lat, &q, &t, &P);
    if (st != KPM_OK) return st;
    const std::array<int, 5> shape = {P->variant, P->block, P->Ty, P->grid, P->Ew};
    // Fell back (LDS, lattice kind) or same shape as an earlier candidate: skip.
    if (P->variant != cd.kernel || std::find(seen.begin(), seen.end(), shape) != seen.end()) {
      plan_free(P);
      delete P;
      continue;
    }
    seen.push_back(shape);
    double rate = 0.0;
    st = kpm_plan_run(P, nullptr, nullptr, 1, stream);
    if (st == KPM_OK || st == KPM_E_SPECTRUM) st = timed_run(P, stream, &rate, nullptr);
    plan_free(P);
    delete P;
    if (st != KPM_OK && st != KPM_E_SPECTRUM) return st;
    screened.push_back({rate, t});
  }
  if (screened.empty()) {
    set_error("autotune: no candidate launch shape");
    return KPM_E_INVALID;
  }
  std::sort(screened.begin(), screened.end(),
            [](const std::pair<double, kpm_tune_t>& x, const std::pair<double, kpm_tune_t>& y) { return x.first > y.first; });
  const int n_fin = (int)std::min<size_t>(3, screened.size());
  kpm_dos_params_t q2 = *p;
  q2.num_moments = 8 * probe_steps;
  // One plan alive at a time (the finalists may each need much of the HBM).
  std::vector<std::vector<std::pair<double, double>>> rates(n_fin);   // (steps/ms, GB/s)
  for (int rep = 0; rep < 3; ++rep)
    for (int i = 0; i < n_fin; ++i) {
      kpm_plan* P = nullptr;
      int st = plan_create(lat, n_lat, &q2, &screened[i].second, &P);
      if (st != KPM_OK) return st;
      double r = 0.0, g = 0.0;
      st = kpm_plan_run(P, nullptr, nullptr, 1, stream);
      if (st == KPM_OK || st == KPM_E_SPECTRUM) st = timed_run(P, stream, &r, &g);
      plan_free(P);
      delete P;
      if (st != KPM_OK && st != KPM_E_SPECTRUM) return st;
      rates[i].push_back({r, g});
    }
  int bi = 0;
  double bmed = -1.0, bgbs = 0.0;
  for (int i = 0; i < n_fin; ++i) {
    std::sort(rates[i].begin(), rates[i].end());
    const auto med = rates[i][rates[i].size() / 2];
    if (med.first > bmed) {
      bmed = med.first;
      bgbs = med.second;
      bi = i;
    }
  }
  *best = screened[bi].second;
  if (best_gbs) *best_gbs = bgbs;
  return tune_cache_store(cache_path, make_key(lat, n_lat, p), *best, bgbs);
}

}  // namespace kpm

extern "C" int kpm_autotune(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p, int32_t probe_steps,
                            const char* cache_path, kpm_tune_t* best, double* best_gbs, void* hip_stream) {
  try {
    kpm::clear_error();
    return kpm::autotune(lat, n_lat, p, probe_steps, cache_path, best, best_gbs, hip_stream);
  } catch (...) {
    kpm::set_error("internal error (exception) in kpm_autotune");
    return KPM_E_DEVICE;
  }
}
