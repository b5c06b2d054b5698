/*
 * kpm.h -- C ABI of libkpm: the data-parallel hot path of the kernel
 * polynomial (Chebyshev) spectral method of KITE (arXiv:1910.05194) on
 * AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status: KPM_OK (0) or a negative KPM_E_*
 *   code.  On failure kpm_last_error() returns a thread-local message.  No
 *   C++ exception crosses the ABI and the library never aborts the process.
 * - Arguments are validated before any device work is enqueued.
 * - The caller owns every input and output buffer.  "Host" pointers are
 *   ordinary CPU memory; "device" pointers are HIP device allocations (for
 *   example torch tensors' data_ptr()).  The library owns its workspace,
 *   which lives inside a plan (kpm_plan_*) or, for the one-shot calls, is
 *   released before the call returns.
 * - hip_stream is a hipStream_t (NULL = the default stream).  Device work is
 *   enqueued on it.  Host outputs are complete when the call returns; device
 *   outputs are complete once the stream has been synchronised.
 * - Energies are in eV, lengths in nm.  Moments are always FP64.
 *
 * Model (paper Sec. 3(a) pattern rules, Sec. 3(d) lattice listing, eq. HQAHE,
 * Sec. 4 magnetic field):
 * - KPM_HONEYCOMB: 2 orbitals per cell (sublattices A, B), a1 = (a, 0),
 *   a2 = (a/2, a sqrt(3)/2), a = 0.24595 nm, A at (0, -a_cc/2), B at
 *   (0, +a_cc/2), a_cc = 0.142 nm; bonds A(n) - B(n + d), d in {(0,0),
 *   (1,-1), (0,-1)} with matrix element t.
 * - KPM_HONEYCOMB_SPIN: the same with two spins per site (4 orbitals per
 *   cell) and the Rashba term (2i/3) lambda_R (s x d_ij)_z, d_ij the unit
 *   bond vector from site j to site i.
 * - KPM_SQUARE: 1 orbital per cell, bonds to the four nearest cells.
 * - Periodic boundaries in both directions.  Peierls phases for a uniform
 *   flux (flux per cell in units of h/e, flux * L1 an integer) use the Landau
 *   gauge A = flux * (0, s1) in fractional coordinates: a hop from site j to
 *   site i gets exp(2 pi i flux (s1_i + s1_j)/2 (s2_i - s2_j)), evaluated with
 *   the unwrapped image of the neighbour.
 * - Anderson disorder V_site = W (u - 1/2), identical for both spins; a site
 *   is vacant iff u' < vacancy_p (its orbitals and bonds are removed).
 * - Orbital index o = ((n2*L1 + n1)*n_sub + s)*n_spin + sigma.
 * - Random numbers: counter-based SplitMix64 (Steele, Lea & Flood 2014),
 *   key(purpose, seed, a, b) = mix(mix(mix(seed + purpose*G) + a*G) + b*G),
 *   x_i = mix(key + (i+1)*G), u_i = (x_i >> 11) 2^-53, G = 0x9E3779B97F4A7C15.
 *   Purposes: 1 = random phase (a = lattice index in the batch, b = vector r,
 *   counter = orbital), 2 = Anderson (counter = site), 3 = vacancy.
 */
#ifndef KPM_H
#define KPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KPM_OK 0
#define KPM_E_INVALID (-1)      /* bad argument, detected before any launch */
#define KPM_E_NOMEM (-2)        /* device allocation failed */
#define KPM_E_DEVICE (-3)       /* HIP runtime error */
#define KPM_E_SPECTRUM (-4)     /* |mu_n| > 1 + 1e-6 or non-finite: the bounds do not enclose the spectrum */
#define KPM_E_UNSUPPORTED (-5)  /* valid request outside what the library implements */

#define KPM_HONEYCOMB 0
#define KPM_HONEYCOMB_SPIN 1
#define KPM_SQUARE 2

#define KPM_FP32 0
#define KPM_FP64 1

#define KPM_START_RANDOM_PHASE 0
#define KPM_START_SITES 1

#define KPM_GAMMA_FP64 0
#define KPM_GAMMA_FP32 1
#define KPM_GAMMA_SPLIT_BF16 2

/* One lattice (a KITE configuration + disorder + modification). */
typedef struct kpm_lattice_t {
  int32_t kind;            /* KPM_HONEYCOMB | KPM_HONEYCOMB_SPIN | KPM_SQUARE */
  int32_t L1, L2;          /* unit cells along a1, a2; each >= 2 */
  double t;                /* nearest-neighbour hopping matrix element, eV */
  double rashba;           /* lambda_R, eV (KPM_HONEYCOMB_SPIN only, else 0) */
  double flux;             /* flux per cell in h/e; flux*L1 integer; not for KPM_SQUARE */
  double anderson_w;       /* W >= 0, eV */
  double vacancy_p;        /* 0 <= p < 1 */
  uint64_t disorder_seed;
  double e_min, e_max;     /* spectrum bounds used for the rescaling, eV, e_min < e_max; rejected
                              (KPM_E_INVALID) when they cut into the Gershgorin interval [-G, G],
                              G = W/2 + |exchange| + Z|t| + 2|rashba| (Z = 3 honeycomb, 4 square),
                              by more than (e_max - e_min)/8; tighter bounds give KPM_E_SPECTRUM */
  double exchange;         /* Delta_ex, eV: + Delta_ex on spin up, - on spin down (eq. HQAHE; KPM_HONEYCOMB_SPIN
                              only, else 0) */
} kpm_lattice_t;

/* DOS / LDOS moment request (KITE Calculation.dos / ldos). */
typedef struct kpm_dos_params_t {
  int32_t num_moments;     /* M >= 2 */
  int32_t num_random;      /* R >= 1 random vectors per lattice (ignored for KPM_START_SITES) */
  uint64_t vector_seed;
  int32_t precision;       /* KPM_FP32 | KPM_FP64: vector storage and recursion arithmetic */
  int32_t start;           /* KPM_START_RANDOM_PHASE | KPM_START_SITES */
  const int64_t* sites;    /* host array of orbital indices (KPM_START_SITES); R := num_sites */
  int32_t num_sites;
} kpm_dos_params_t;

/* Optional launch shape of the Chebyshev step kernel (0 = library choice / autotune cache). */
typedef struct kpm_tune_t {
  int32_t block;           /* threads per workgroup (64..512, multiple of 64); 0 = 512 for the sweep kernels
                              (less where their row rings would not fit in LDS), 256 otherwise */
  int32_t rows;            /* lattice rows (along a2) per tile; 0 = the largest power of two <= 128 (sweep
                              kernels) or <= 64 (single-step) that leaves >= 2048 tiles */
  int32_t grid;            /* persistent workgroups (multiple of 8); 0 = one per tile */
  int32_t use_graph;       /* 1 = replay the step loop as a captured hipGraph (default), 0 = eager */
  int32_t kernel;          /* 0 = default (5 where eligible, else 2), 1 = direct neighbour loads, 2 = LDS row
                              ring, 3/4/5/6 = 2/3/4/5 steps per sweep (spinless lattices, Peierls phases
                              included, with room for four vectors; a sweep whose row rings do not fit in LDS
                              takes one step fewer, down to 2) */
  int32_t chunks;          /* 16-byte vector chunks per site that one tile covers (1..E, E = the site's R_padded
                              complex values in 16-byte chunks); a tile then spans block / (sublattices * chunks)
                              cell columns; 0 = library choice */
} kpm_tune_t;

typedef struct kpm_plan_info_t {
  int32_t n_steps;               /* recursion steps per run (ceil(M/2)); variants 3..6 launch once per 2..5 */
  int32_t n_tiles;               /* tiles in the work list */
  int32_t grid, block, rows, tile_cells_x;
  int32_t r_padded;              /* vectors per orbital as stored (R rounded up) */
  int32_t kernel;                /* step kernel variant in use (1 direct, 2 LDS ring, 3..6 = 2..5 steps per
                                    sweep) */
  int64_t n_orbitals;            /* orbitals in the batch, vacancies included */
  double bytes_per_step;         /* algorithmic HBM bytes per recursion step (variants 3..6: two vectors
                                    and the site arrays in, two vectors out, per sweep of 2..5 steps) */
  double last_loop_ms;           /* step loop of the last run (hipEvents on the run's stream) */
  double last_run_ms;            /* whole last run (hipEvents) */
  int64_t n_active_total;        /* active orbitals summed over lattices (after the last run) */
  int32_t tile_chunks;           /* 16-byte vector chunks per site a tile covers */
} kpm_plan_info_t;

typedef struct kpm_plan kpm_plan_t;

int kpm_version(void);
const char* kpm_last_error(void);

/*
 * DOS / LDOS Chebyshev moments (paper eqs. e6, e8; Sec. 2(c) stochastic trace;
 * eq. PcomplexityFactor: R vectors, S = n_lat realisations per call).
 *
 * For every lattice l and start vector r:
 *   mu^(l,r)_n = <r|T_n(H~_l)|r> / norm_l,   n = 0..M-1,
 *   H~ = (H - de+)/de-, de+- = (e_max +- e_min)/2 (eqs. rescalingH/E),
 * with |r> = sum_o exp(2 pi i u_{r,o}) |o> over active orbitals and norm_l =
 * number of active orbitals (random phase), or |r> = |sites[r]> and norm = 1
 * (LDOS, Sec. 4 LDOS example).  All lattices of a batch share M, R, precision
 * and start kind and run in one persistent kernel per Chebyshev step.
 *
 * Outputs (either may be NULL):
 *   mu_per_vector  [n_lat][R][M] FP64
 *   mu_mean        [n_lat][M]    FP64, the mean over r
 * out_on_device: 0 = host pointers, 1 = device pointers.
 * Errors: KPM_E_INVALID (L < 2, M < 2, R < 1, e_min >= e_max, flux*L1 not an
 * integer, flux on a square lattice, Rashba on a spinless lattice, lattices of
 * different kinds in one batch, an LDOS site out of range or vacant);
 * KPM_E_SPECTRUM if a moment is non-finite or exceeds 1 + 1e-6 in magnitude,
 * i.e. the bounds do not enclose the spectrum (the paper warns that estimated
 * bounds need checking; outputs are still written); KPM_E_NOMEM, KPM_E_DEVICE.
 */
int kpm_moments_dos(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p,
                    double* mu_per_vector, double* mu_mean, int32_t out_on_device, void* hip_stream);

/*
 * Allocation-free form of kpm_moments_dos, for callers that cannot allocate
 * device memory: code running under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, outputs, launch shape,
 * results (bit for bit) and errors as kpm_moments_dos, except that:
 * - the device workspace (vectors, disorder arrays, tile list, moment
 *   partials) is carved from a static device array of
 *   KPM_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on
 *   holds until the process ends; the call makes no hipMalloc or hipFree and
 *   creates no stream, event or graph (the loop runs eagerly on hip_stream);
 * - it runs on the current HIP device (hip_stream must belong to it);
 * - a workload whose workspace exceeds the array (roughly n_orbitals x
 *   R_padded complex values x 4 vectors, or x 2 when four do not fit in three
 *   quarters of it) is rejected with KPM_E_INVALID before any launch, and
 *   kpm_last_error() states the bytes it needs.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (the kernels write everything they later read; counters and flags
 * are cleared by kernels on hip_stream).  The call synchronises hip_stream
 * before it returns, so calls made one after another are safe; calls that
 * overlap on one GPU (two host threads, or a second call before the first has
 * returned) race on the array and give wrong results.
 */
#define KPM_NOALLOC_SCRATCH_BYTES (64ull << 20)
int kpm_moments_dos_noalloc(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p,
                            double* mu_per_vector, double* mu_mean, int32_t out_on_device, void* hip_stream);

/*
 * Launch-shape autotuner (the analogue of the paper's user-tuned TILE size,
 * Sec. 3(b) and Table 1).  Runs the recursion for probe_steps steps with each
 * candidate (kernel variant 1..6 x block x rows x grid x chunks) on the given
 * workload, timed with hipEvents on hip_stream, re-times the three fastest on
 * 4 probe_steps steps (median of three rounds), and returns the one with the
 * shortest time per step in *best (and its algorithmic GB/s in *best_gbs, may
 * be NULL; the sweep variants move fewer bytes per step, so GB/s does not rank
 * variants).  If cache_path is non-NULL the
 * result is appended to that text file; kpm_plan_create reads the file named
 * by the environment variable KPM_TUNE_CACHE whenever it is called without a
 * launch shape (tune NULL or all of block, rows, grid, kernel zero).  Allocates
 * one full-size plan at a time.
 */
int kpm_autotune(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p, int32_t probe_steps,
                 const char* cache_path, kpm_tune_t* best, double* best_gbs, void* hip_stream);

/* Reusable form of kpm_moments_dos: create allocates the device workspace
 * (two vector buffers of n_orbitals * R_padded complex values, per-site disorder
 * arrays, the tile work list, moment partials); run builds the disorder, the
 * start vectors and runs the whole recursion (replayed as a hipGraph after the
 * first run when tune->use_graph != 0); destroy frees everything.  A plan may
 * be run on different streams but not concurrently with itself.  With the
 * environment variable KPM_LOG set (and not "0"), plan creation (also inside
 * kpm_moments_dos and kpm_moments_dos_noalloc) writes a one-line summary of the
 * chosen plan to stderr: workload, kernel variant, tile shape, grid, LDS and
 * device bytes, algorithmic bytes per step. */
int kpm_plan_create(const kpm_lattice_t* lat, int32_t n_lat, const kpm_dos_params_t* p,
                    const kpm_tune_t* tune, kpm_plan_t** plan);
int kpm_plan_run(kpm_plan_t* plan, double* mu_per_vector, double* mu_mean, int32_t out_on_device,
                 void* hip_stream);
int kpm_plan_info(kpm_plan_t* plan, kpm_plan_info_t* info);
int kpm_plan_destroy(kpm_plan_t* plan);

/*
 * Jackson-damped DOS reconstruction (eqs. e7, delta_function_cheb_expansion;
 * Jackson kernel of Weisse et al., Rev. Mod. Phys. 78, 275 (2006), which the
 * paper cites):
 *   rho(E_k) = [g_0 mu_0 + 2 sum_{n=1}^{M-1} g_n mu_n T_n(eps_k)] / (pi sqrt(1-eps_k^2) de-),
 *   g_n = [(M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))]/(M+1),
 * eps_k = (E_k - de+)/de-; energies outside (e_min, e_max) give 0.  The
 * printed factor of eqs. sss/e8 is read as 2/(1+delta_n0) (see eqs. e4, e7).
 * mu [M], energies_ev [K], rho [K] (per eV per orbital), all FP64; host
 * pointers (on_device = 0) or device pointers (on_device = 1).  M may be any
 * prefix length of a longer moment table (post-processing with fewer moments).
 */
int kpm_reconstruct_jackson(const double* mu, int32_t M, const double* energies_ev, int32_t K,
                            double e_min, double e_max, double* rho, int32_t on_device,
                            void* hip_stream);

/*
 * The damping factors of the KPM reconstructions (Sec. 2(a)): g[i] = g_{n0 + i}
 * of an M-moment expansion, i < count, for kernel 0 = Jackson (Weisse et al.
 * 2006, as in kpm_reconstruct_jackson) or 1 = Lorentz with lambda (as in
 * kpm_reconstruct_lorentz).  g [count] FP64, host (on_device = 0) or device.
 * KPM_E_INVALID unless 0 <= n0 < n0 + count <= M and (Lorentz) lambda > 0.
 */
int kpm_kernel_factors(int32_t kernel, int32_t M, double lambda, int32_t n0, int32_t count, double* g,
                       int32_t on_device, void* hip_stream);

/*
 * The same KPM reconstruction with the Lorentz kernel the paper prints for
 * damping Gibbs oscillations (Sec. 2(a)): g_n = sinh(lambda (1 - n/M)) /
 * sinh(lambda), n = 0..M-1; a delta peak becomes a Lorentzian of half width
 * ~ lambda/M in rescaled units.  Arguments as kpm_reconstruct_jackson;
 * lambda > 0 (KPM_E_INVALID otherwise).
 */
int kpm_reconstruct_lorentz(const double* mu, int32_t M, const double* energies_ev, int32_t K,
                            double e_min, double e_max, double lambda, double* rho, int32_t on_device,
                            void* hip_stream);

/*
 * CPGF reconstruction (eqs. green_function_cheb_expansion and
 * green_function_cheb_expansionb, retarded sector): the traced resolvent
 *   G(E) = (1/N) Tr 1/(E - H + i eta) = (1/de-) sum_{n<M} g_n(z) mu_n / (1 + delta_n0),
 *   g_n(z) = -2 i exp(-i n arccos z) / sqrt(1 - z^2),  z = (E - de+)/de- + i eta/de-,
 * and rho(E) = -Im G(E) / pi (the DOS broadened by a Lorentzian of half width
 * eta, per eV per orbital).  Defined for every E, inside or outside the
 * spectrum bounds; the truncation error decays like exp(-M Im(-arccos z)),
 * i.e. M ~ several de-/eta terms converge.  mu [M], energies_ev [K] (eV),
 * rho [K], green [K][2] (re, im; may be NULL), all FP64, host or device
 * pointers as on_device says.  eta_ev > 0 (KPM_E_INVALID otherwise).
 */
int kpm_reconstruct_cpgf(const double* mu, int32_t M, const double* energies_ev, int32_t K, double e_min,
                         double e_max, double eta_ev, double* rho, double* green, int32_t on_device,
                         void* hip_stream);

/* Conductivity moment request (KITE Calculation.conductivity_dc/optical, direction = alpha beta). */
typedef struct kpm_cond_params_t {
  int32_t num_moments;     /* M >= 2: Gamma is M x M */
  int32_t num_random;      /* R >= 1 random-phase vectors */
  uint64_t vector_seed;
  int32_t alpha, beta;     /* 0 = x, 1 = y */
  int32_t gamma_mode;      /* KPM_GAMMA_SPLIT_BF16 (MFMA, FP32 blocks) | KPM_GAMMA_FP64 (FP64 dot products) */
  int32_t precision;       /* KPM_FP32 | KPM_FP64: Chebyshev vectors and stored blocks */
  int32_t max_batch;       /* most vectors per batch (0 = as many as fit in device memory) */
} kpm_cond_params_t;

/*
 * Rank-2 Gamma tensor (paper eq. Gammanm with the stochastic trace of Sec. 2(c)):
 *   Gamma_nm = 1/(R N) sum_r <r| h~^a T_n(H~) h~^b T_m(H~) |r> / ((1+d_n0)(1+d_m0)),
 * h~^a = [r^a, H] in eV nm (the paper's h~ = (i hbar) h, anti-Hermitian), from
 * the physical H (bond vectors d_ij = r_i - r_j, so the operator is defined on
 * the torus), N = number of active orbitals, |r> random phases as for the DOS
 * (lattice index 0, vector r).  Computed as <L_n|R_m> with L_n = T_n(H~)(-h~^a r)
 * and R_m = h~^b T_m(H~) r: both chains are stored as [M][orbitals x vectors]
 * blocks (vectors batched to fit memory) and contracted by a GEMM
 * (split-BF16 x 3 on MFMA with FP32 accumulation per K chunk and FP64 across
 * chunks, or FP64).
 * Output gamma [M][M][2] (re, im) FP64, host (out_on_device = 0) or device.
 * Errors: as kpm_moments_dos; KPM_E_INVALID also for bad alpha/beta/mode or
 * split-BF16 with FP64 blocks; KPM_E_NOMEM when one vector's blocks
 * (2 M N complex values) do not fit.
 */
int kpm_moments_cond(const kpm_lattice_t* lat, const kpm_cond_params_t* p, double* gamma, int32_t out_on_device,
                     void* hip_stream);

/*
 * Rank-1 tensor (the Gamma_n^{ab} of the paper's Gamma family, eq. Gammanm and
 * the examples after it) with the stochastic trace of Sec. 2(c):
 *   Gamma_n^{ab} = 1/(R N) sum_r <T_n(H~) r | h~^{ab} r> / (1 + d_n0),
 * h~^{ab} = [r^a, [r^b, H]] in eV nm^2 (Hermitian; bond vectors as for h~^a),
 * |r> the random phases of kpm_moments_cond (same seed, same vectors).  Uses
 * p->num_moments (>= 1), num_random, vector_seed, alpha, beta, precision;
 * gamma_mode and max_batch are ignored (all vectors in one pass: three
 * vectors of n_orbitals x R_padded complex values).  Output gamma1 [M][2]
 * (re, im) FP64, host (out_on_device = 0) or device.  Errors: as
 * kpm_moments_cond.
 */
int kpm_moments_gamma1(const kpm_lattice_t* lat, const kpm_cond_params_t* p, double* gamma1, int32_t out_on_device,
                       void* hip_stream);

/*
 * Single-shot Fermi-surface DC conductivity (the paper's 'single-shot'
 * algorithm, Sec. 3(b): no double recursion), T = 0, in units of e^2/h:
 *   sigma_ab(E) = -2 pi^2 (1/Omega) Tr[h~^a d_eta(E-H) h~^b d_eta(E-H)],
 *   d_eta(E - H) = -(1/pi) Im G^R(E + i eta) = sum_n c_n(E) T_n(H~),
 *   c_n = -Im g_n(z~) / (pi de- (1 + d_n0))  (eq. green_function_cheb_expansionb),
 * Omega = L1 L2 * cell area, with the stochastic trace over the random phases
 * of kpm_moments_cond (same seed, same vectors): -(1/R) sum_r <a|b>,
 * a = d_eta h~^a r, b = h~^b d_eta r.  Two Chebyshev recursions per vector of
 * p->num_moments steps serve all K energies: each writes its vectors into a
 * history of B (3..64) vectors, flushed every B steps into 2 K accumulator
 * vectors (B and the energies per batch fitted to the free device memory;
 * workspace B + 2 kb + 2 vectors of n_orbitals x R_padded complex values).
 * Uses num_moments (>= 2), num_random, vector_seed, alpha, beta, precision.
 * energies_ev [K] (1 <= K <= 4096), sigma [K]: both host (on_device = 0) or
 * both device.  Errors: as kpm_moments_cond; KPM_E_INVALID also for eta <= 0;
 * KPM_E_NOMEM when not even a 3-vector history and one energy's accumulators
 * fit.
 */
int kpm_sigma_singleshot(const kpm_lattice_t* lat, const kpm_cond_params_t* p, const double* energies_ev, int32_t K,
                         double eta_ev, double* sigma, int32_t out_on_device, void* hip_stream);

/* Timing and work of the last kpm_moments_cond call on the calling thread
 * (hipEvents on the call's stream). */
typedef struct kpm_cond_stats_t {
  int32_t n_batches, vectors_per_batch;
  double chain_ms;            /* both Chebyshev chains, all batches */
  double gemm_ms;             /* Gamma GEMM + its chunk reduction, all batches */
  double total_ms;            /* the whole call */
  double chain_bytes;         /* algorithmic HBM bytes of the chain launches */
  double gemm_useful_flops;   /* 4 M^2 (2 N R) real flops = 8 M^2 N R */
  double gemm_mfma_flops;     /* flops issued to the matrix cores (x3 for split-BF16) */
  double gemm_operand_bytes;  /* both stored blocks read once */
} kpm_cond_stats_t;
int kpm_cond_last_stats(kpm_cond_stats_t* stats);

/*
 * T = 0 longitudinal conductivity from Gamma (alpha = beta), in units of e^2/h:
 *   sigma(E) = -2 pi^2 (N/Omega) / de-^2 sum_nm g_n g_m D_n(eps) D_m(eps) Re Gamma_nm,
 *   D_n(eps) = 2 T_n(eps)/(pi sqrt(1 - eps^2))  (eq. delta_function_cheb_expansion),
 * g_n the Jackson kernel, N/Omega = orbitals_per_nm2.  This is the Fermi-surface
 * (Kubo-Greenwood) limit of the first-order conductivity (eq. cond 1st order) at
 * T = 0, omega -> 0; the paper's KITE-tools use the full Kubo-Bastin form.
 * gamma [M][M][2], energies_ev [K], sigma [K]; host or device pointers.
 */
int kpm_reconstruct_sigma(const double* gamma, int32_t M, const double* energies_ev, int32_t K, double e_min,
                          double e_max, double orbitals_per_nm2, double* sigma, int32_t on_device, void* hip_stream);

/*
 * Kubo-Bastin conductivity from Gamma^{ab} (any a, b; a = x, b = y is the
 * Hall conductivity) at chemical potential mu and temperature T, in units of
 * e^2/h: the static limit of the first-order formula (eq. cond 1st order,
 * with its Fermi function f) with the delta function of eq.
 * delta_function_cheb_expansion and the CPGF resolvents of eqs.
 * green_function_cheb_expansion(b) at broadening eta, contracted with Gamma as
 * in eq. conductivity_1st_order (the Lambda_nm of a static field):
 *   sigma_ab(mu) = Re{ -2 pi i (N/Omega)/de-^2 int_{-1}^{1} d eps f(eps)
 *                  sum_nm Gamma_nm [Delta_n(eps) g'^R_m(eps) - g'^A_n(eps) Delta_m(eps)] },
 * g' = d g / d eps, f = 1/(1 + exp((E - mu)/kT)), N/Omega = orbitals_per_nm2.
 * The integral runs in theta (eps = cos theta) over n_theta equal cells of
 * [0, pi] (n_theta = 0: 4 M): the integrand apart from f at each cell's
 * midpoint times int_cell f(cos theta) d theta, which at kT_ev = 0 is the
 * length of the cell inside [theta_mu, pi] (mu~ = (mu - de+)/de- = cos
 * theta_mu) and at kT_ev > 0 a midpoint sum over 32 sub-cells (the cells
 * should then be narrower than a few kT).
 * gamma [M][M][2] (re, im) as kpm_moments_cond writes it, energies_ev [K]
 * Fermi energies, sigma [K]; all host (on_device = 0) or all device pointers.
 * Allocates a device workspace of ~16 (Mp^2 + 2 (n_theta + 64) Mp) bytes,
 * Mp = M rounded up to 64, and frees it before returning; synchronises
 * hip_stream.  Errors: KPM_E_INVALID (NULL, M outside [1, 16384], K < 1,
 * e_min >= e_max, eta <= 0, kT < 0, orbitals_per_nm2 <= 0, n_theta outside
 * [0, 2^20]); KPM_E_DEVICE.
 */
int kpm_reconstruct_sigma_bastin(const double* gamma, int32_t M, const double* energies_ev, int32_t K, double e_min,
                                 double e_max, double eta_ev, double kT_ev, double orbitals_per_nm2, int32_t n_theta,
                                 double* sigma, int32_t on_device, void* hip_stream);

/*
 * Optical conductivity sigma_ab(omega) in units of e^2/h at chemical potential
 * mu and temperature T (kT_ev, 0 allowed), from the rank-1 Gamma_n^{ab}
 * (kpm_moments_gamma1) and the rank-2 Gamma_nm^{a,b} (kpm_moments_cond) of
 * the same lattice and directions (eq. conductivity_1st_order with the
 * Lambda_n and Lambda_nm(omega) of the paper and the Fermi function f):
 *   sigma(w) = (-2 pi i (N/Omega)/E_w) [ sum_n Gamma_n L_n + (1/de-) sum_nm Gamma_nm L_nm(w) ],
 *   L_n = int d eps f(eps) Delta_n(eps),
 *   L_nm(w) = int d eps f(eps) [g^R_n(eps + w~) Delta_m(eps) + Delta_n(eps) g^A_m(eps - w~)],
 * E_w = hbar omega > 0 in eV (w~ = E_w/de-), g^{R,A} the CPGF coefficients at
 * broadening eta; energy integrals and occupation weights as in
 * kpm_reconstruct_sigma_bastin.
 * gamma_nm [M][M][2], gamma_n [M][2], omegas_ev [K], sigma [K][2] (re, im);
 * all host (on_device = 0) or all device pointers (the frequencies are copied
 * to the host either way).  Work per frequency: two coefficient tables and
 * one M x M x n_theta contraction.  Allocates and frees a device workspace;
 * synchronises hip_stream.  Errors: KPM_E_INVALID (NULL, M outside
 * [1, 16384], K outside [1, 65536], a frequency <= 0, e_min >= e_max,
 * eta <= 0, kT < 0, orbitals_per_nm2 <= 0, n_theta outside [0, 2^20]);
 * KPM_E_DEVICE.
 */
int kpm_reconstruct_sigma_optical(const double* gamma_nm, const double* gamma_n, int32_t M, const double* omegas_ev,
                                  int32_t K, double mu_ev, double e_min, double e_max, double eta_ev, double kT_ev,
                                  double orbitals_per_nm2, int32_t n_theta, double* sigma, int32_t on_device,
                                  void* hip_stream);

/*
 * Wave-packet time evolution (the paper's spintronics example, Sec. 4).
 * psi(t + dt) = U(dt) psi(t) with the Chebyshev expansion of the time-evolution
 * operator of the rescaled Hamiltonian (Tal-Ezer and Kosloff):
 *   U(dt) = exp(-i de+ dt/hbar) sum_{n < M} (2 - d_n0) (-i)^n J_n(de- dt/hbar) T_n(H~),
 * read with (-i)^n where the paper prints (-1)^n (Jacobi-Anger; only this is
 * unitary).  M = num_moments terms per time step must exceed |de- dt/hbar| by a
 * margin (J_n decays faster than exponentially beyond n ~ |de- dt/hbar|).
 */
typedef struct kpm_evolve_params_t {
  int32_t num_moments;     /* Chebyshev terms per time step, >= 2 */
  int32_t num_points;      /* time points t_k = k dt, k = 0 .. num_points - 1 (>= 1) */
  int32_t num_packets;     /* R states evolved together (1 .. 4096) */
  int32_t precision;       /* KPM_FP32 | KPM_FP64: vectors of the recursion (sums in FP64) */
  double dt_fs;            /* time step in fs (nonzero; negative runs backwards) */
} kpm_evolve_params_t;

/*
 * Gaussian wave packet psi(0, r) = exp(-|r - r_c|^2 / (2 width^2)) sum_j exp(i k_j.r) spinor_j
 * (Sec. 4; the printed exponent is garbled: width is read as the envelope's
 * standard deviation), r the site position n1 a1 + n2 a2 + tau_s (nm), r_c =
 * c1 a1 + c2 a2 for center_cells = (c1, c2), zero on vacant sites, normalised
 * to 1.  k_vectors [n_k][2] (1/nm), spinors [n_k][orbitals per cell][2] (re, im;
 * per cell sublattice-major, then spin up, down), psi [n_orbitals][2] FP64 in
 * the library's orbital order ((n2 L1 + n1) sublattices + s) spins + spin.
 * k_vectors, spinors and center_cells are host arrays; psi is host (on_device
 * = 0) or device.  Synchronises hip_stream.  Errors: KPM_E_INVALID (NULL,
 * n_k outside [1, 4096], width <= 0, a zero-norm packet, invalid lattice);
 * KPM_E_NOMEM; KPM_E_DEVICE.
 */
int kpm_wavepacket_gaussian(const kpm_lattice_t* lat, int32_t n_k, const double* k_vectors, const double* spinors,
                            double width_nm, const double* center_cells, double* psi, int32_t on_device,
                            void* hip_stream);

/*
 * Evolves p->num_packets states of one lattice by p->num_points - 1 time steps
 * of p->dt_fs and records at each t_k = k dt (k = 0 included) the observables
 * of Sec. 4 per packet: [norm, <x>, <y>, <x^2>, <y^2>, <sigma_x>, <sigma_y>,
 * <sigma_z>] (nm, nm^2, hbar/2; all but the norm divided by it; spin zero on
 * spinless lattices; positions as in kpm_wavepacket_gaussian, meaningful while
 * the packet stays away from the periodic seam).  psi [R][n_orbitals][2] FP64:
 * on entry the states at t = 0 (entries on vacant orbitals are ignored: the
 * model has no such states), on return at t = (num_points - 1) dt;
 * observables [num_points][R][8] FP64; both host (on_device = 0) or both
 * device.  Workspace: the plan's two vectors and a history of up to 32 vectors
 * of n_orbitals x R_padded complex values (fewer if memory is short).
 * Synchronises hip_stream.  Errors: KPM_E_INVALID (NULL, parameters outside
 * their ranges, invalid lattice); KPM_E_NOMEM (not even a 3-vector history
 * fits); KPM_E_DEVICE.
 */
int kpm_time_evolve(const kpm_lattice_t* lat, const kpm_evolve_params_t* p, double* psi, double* observables,
                    int32_t on_device, void* hip_stream);

/* Timing and work of the last kpm_time_evolve call on the calling thread. */
typedef struct kpm_evolve_stats_t {
  int32_t history;            /* vectors in the history (flush every this many Chebyshev terms) */
  int32_t time_steps;         /* num_points - 1 */
  double loop_ms;             /* the time-step loop with its observables (hipEvents on the call's stream;
                                 excludes workspace allocation, model build and the copies in and out) */
  double bytes;               /* algorithmic HBM bytes of the loop: per recursion step v_n, v_(n-1),
                                 v_(n+1) and the per-site arrays; per flush the history vectors read
                                 and psi(t + dt) written (and read after the first flush) */
} kpm_evolve_stats_t;
int kpm_evolve_last_stats(kpm_evolve_stats_t* stats);

/*
 * Moment-extrapolation MLP (the paper has no learned component: this is the
 * learned part of this implementation, specified by its shape alone).
 * Network n_in -> n_hidden -> n_hidden -> n_out, exact GELU x Phi(x) after the
 * first two layers, FP32 parameters in device memory owned by the handle.
 * Parameters are exchanged in packed order W1 [n_in][n_hidden], b1, W2
 * [n_hidden][n_hidden], b2, W3 [n_hidden][n_out], b3 (row-major: y = x W + b).
 * Initialisation: W ~ U(-sqrt(3/fan_in), +sqrt(3/fan_in)) from the SplitMix64
 * stream (purpose 5, seed, layer), b = 0.
 * Loss: L = 1/(B n_out) sum_{b,j} (w_j (Y_bj - T_bj))^2 with caller-supplied
 * weights w (the Jackson factors of the predicted orders).
 * x [B][n_in], target [B][n_out], weights [n_out], y [B][n_out]: FP32 device
 * pointers.  forward: use_bf16 = 1 runs the GEMMs with BF16 operands and FP32
 * accumulation (MFMA), 0 in FP32 (MFMA).  train_step: forward, loss, backward
 * and one Adam step (beta1 0.9, beta2 0.999, eps 1e-8), loss written to the
 * device double loss_dev_out (may be NULL).  gradients: forward + backward
 * only; gradients copied to grads_host in packed order (FP32), loss to *loss.
 * Work is enqueued on hip_stream; get/set_params synchronise the device.
 */
typedef struct kpm_mlp kpm_mlp_t;
int kpm_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, uint64_t seed, kpm_mlp_t** mlp);
int kpm_mlp_destroy(kpm_mlp_t* mlp);
int kpm_mlp_num_params(const kpm_mlp_t* mlp, int64_t* n);
int kpm_mlp_get_params(kpm_mlp_t* mlp, float* params_host);
int kpm_mlp_set_params(kpm_mlp_t* mlp, const float* params_host);
int kpm_mlp_forward(kpm_mlp_t* mlp, const float* x, int32_t batch, float* y, int32_t use_bf16, void* hip_stream);
int kpm_mlp_train_step(kpm_mlp_t* mlp, const float* x, const float* target, const float* weights, int32_t batch,
                       float lr, double* loss_dev_out, void* hip_stream);
int kpm_mlp_gradients(kpm_mlp_t* mlp, const float* x, const float* target, const float* weights, int32_t batch,
                      float* grads_host, double* loss, void* hip_stream);
/* Optional per-column standardisation: x [n_rows][n_in] and target [n_rows][n_out]
 * (device) give column means and standard deviations; from then on forward
 * maps x -> (x - mean)/sd before the network and y' -> mean + sd y' after it,
 * and training uses the standardised targets with weights w * sd_out (the same
 * loss in original units).  Gradients then refer to the standardised network. */
int kpm_mlp_fit_scaling(kpm_mlp_t* mlp, const float* x, const float* target, int64_t n_rows, void* hip_stream);
/* Acceptance measure of predicted moment tables: the network's output y for
 * x [batch][n_in] (original units, use_bf16 as in forward) against reference
 * moments ref [batch][n_cmp] (FP64) on its first n_cmp orders, weighted by
 * weights [n_cmp] (FP32):
 *   err[b] = ||w (y_b - ref_b)|| / ||w ref_b||   (FP64, [batch]).
 * Validation loss: the training loss L of the network's output (original
 * units) against target with weights, no update, into the device double
 * loss_dev_out.  All pointers device; work enqueued on hip_stream. */
int kpm_mlp_rel_error(kpm_mlp_t* mlp, const float* x, const double* ref, const float* weights, int32_t batch,
                      int32_t n_cmp, int32_t use_bf16, double* err, void* hip_stream);
/* Acceptance measure against the statistical error of the reference moments
 * (Sec. 2(c), the stochastic trace: its error falls as 1/sqrt(R N)).  For
 * random-phase vectors the variance of one vector's estimate of
 * Tr T_n(H~)/N is sum_{i != j} |T_n,ij|^2 / N^2 <= Tr T_n(H~)^2 / N^2 <= 1/N,
 * so the mean over R vectors has a standard error of at most 1/sqrt(N R);
 * noise [batch] (FP64, device, each > 0; not checked on the host, a zero
 * gives an overflowing z) holds that scale per row.  With the same x,
 * ref, weights and use_bf16 as kpm_mlp_rel_error:
 *   z[b] = ||w (y_b - ref_b)|| / (noise_b ||w||)   (FP64, [batch]),
 * the weighted RMS deviation of the prediction in units of the reference's
 * standard error (about 1 when the prediction is within the reference's
 * noise).  All pointers device; work enqueued on hip_stream. */
int kpm_mlp_noise_z(kpm_mlp_t* mlp, const float* x, const double* ref, const double* noise, const float* weights,
                    int32_t batch, int32_t n_cmp, int32_t use_bf16, double* z, void* hip_stream);
int kpm_mlp_eval_loss(kpm_mlp_t* mlp, const float* x, const float* target, const float* weights, int32_t batch,
                      int32_t use_bf16, double* loss_dev_out, void* hip_stream);

/*
 * HBM bandwidth probe (measurement support for the roofline; not part of the
 * method).  Streams float4 arrays of bytes_per_array bytes with a grid-stride
 * kernel of the given shape: pattern 0 = copy (dst = src), 1 = read-only
 * reduction, 2 = in-place w = 2 v - w (two reads and one write per element,
 * the memory pattern of a Chebyshev step), 3 = copy with four elements per
 * thread and iteration, loads before stores.  nontemporal != 0 uses streaming
 * loads/stores.  Allocates and frees its own arrays; synchronises the stream.
 * Outputs: average milliseconds per launch over iters launches (after one
 * warm-up launch) and the bytes moved per launch.
 */
int kpm_bandwidth_probe(int32_t pattern, int64_t bytes_per_array, int32_t iters, int32_t grid, int32_t block,
                        int32_t nontemporal, void* hip_stream, double* ms_per_iter, double* bytes_moved_per_iter);

/*
 * Error-path testing (test support; not part of the method).
 *
 * kpm_debug_inject_failure arms a countdown over the library's checked HIP
 * operations in this process: device allocations, host/device copies, stream
 * and event calls, and the status checks after kernel launches.  The nth of
 * them from now on fails with the injected error and the countdown disarms:
 * kind 0 = out of memory (the call returns KPM_E_NOMEM), kind 1 = launch
 * failure (KPM_E_DEVICE).  An allocation or an enqueue so failed is not
 * performed; a synchronising call or a kernel launch is performed and only
 * its status is replaced.  nth = 0 disarms.  Returns how many failures were
 * injected since the previous call (0 or 1), or KPM_E_INVALID for nth < 0 or
 * an unknown kind.  Calls from every thread take part in the countdown.
 *
 * kpm_debug_live_allocations returns the number of device buffers the
 * library holds at the moment (plans, networks, per-call workspaces), so a
 * test can check that a failed call released everything it allocated.
 */
int32_t kpm_debug_inject_failure(int32_t nth, int32_t kind);
int64_t kpm_debug_live_allocations(void);

#ifdef __cplusplus
}
#endif
#endif /* KPM_H */
