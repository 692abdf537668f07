/*
 * miloc.h -- C ABI of the MI355X ALI line radiative-transfer library (libmiloc.so).
 *
 * The library solves the non-LTE level populations of one molecular species
 * in a 1D spherical cloud (nested shells), a 3D regular Cartesian grid or a
 * 3D octree (a regular root grid with nested refinement) by
 * alternating a deterministic ray march (radiative transfer) with per-cell
 * statistical-equilibrium solves, as in Juvela (2020), "LOC program for line
 * radiative transfer":
 *   - problem statement: a model, a molecule and a fixed ray set; radiation
 *     field and level populations iterated until converged; the final
 *     populations kept and spectra made by a last line-of-sight integration
 *     (Sect. 2);
 *   - per-step radiative update and absorbed-photon counting (Sect. 2,
 *     Eqs. (2)-(3)); the diagonal accelerated lambda iteration, A_ul scaled by
 *     the escape probability (Sect. 2);
 *   - 1D impact-parameter rays through shells (Sect. 2.1), 3D HEALPix ray
 *     directions with one ray per upstream surface element and side
 *     re-entry, and in octrees rays split at refinement boundaries
 *     (Sect. 2.2).
 *
 * Conventions (all calls):
 *   - Units are CGS and Kelvin.  Host arrays are row-major.
 *   - Every call returns miloc_status: MILOC_OK (0) or a negative error code.
 *     On error nothing is written to caller buffers and miloc_last_error()
 *     describes the failure.  No C++ exception crosses this boundary.
 *   - Inputs are copied before the call returns; the caller keeps ownership
 *     of every buffer it passes.  Outputs go to caller-allocated host buffers
 *     sized from miloc_get_sizes().  The library owns all device memory.
 *   - A context is not thread-safe; use one context per host thread.  All
 *     device work of a context is issued on one HIP stream (its own, or one
 *     the caller lends at creation and keeps alive until miloc_destroy).
 *   - Calls in the wrong order (run before a model, molecule and spectral
 *     grid are loaded; spectra before populations exist) return MILOC_ESTATE.
 *
 * Tuning (environment, read when a context prepares its first run):
 *   - MILOC_LANES: lanes per ray of the march (1D and regular 3D: 8, 16, 32
 *     or 64; octree: 8 or 16).  Default: by the widest channel window
 *     (regular 3D), 16 (1D), 8 (octree).  Results do not depend on it beyond
 *     FP32 summation order.
 *   - MILOC_STEP_BUFFER_GB: device memory (GB) for the 3D per-step partial
 *     sums of one march launch (default 16 for regular grids, 160 for
 *     octrees); the transitions of an iteration that do not fit are marched
 *     in further launches.
 *   - MILOC_WIDE_OFFSETS (set, any value; read at every march launch): the
 *     FP32 regular-grid march addresses its cell tables with 64-bit offsets
 *     also where 32-bit ones suffice (grids below 2^24 cells whose tables
 *     stay below 4 GB).  The results are identical; for testing.
 *   - MILOC_FULL_CHANNEL_VECTORS (set, any value; read when a context first
 *     marches a regular grid after its windows were built): the FP32
 *     regular-grid march keeps every ray's whole channel vector in LDS rather
 *     than only the span of channels the ray's windows reach (which allows
 *     more workgroups per compute unit).  The results are identical; for
 *     testing.
 */
#ifndef MILOC_H
#define MILOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MILOC_OK = 0,
    MILOC_EINVAL = -1,   /* bad argument: NULL, size, NaN, negative physical value, band too narrow */
    MILOC_ENOMEM = -2,   /* device or host allocation failed                                        */
    MILOC_EDEVICE = -3,  /* HIP runtime error, or no usable gfx950 device                            */
    MILOC_ESTATE = -4,   /* call out of order                                                        */
    MILOC_ENOTCONV = -5, /* miloc_run reached max_iter without meeting tol (results still valid)     */
    MILOC_ENUMERIC = -6, /* non-finite or negative populations, or a maser: a step whose line-centre */
                         /* optical depth is below -40 (population inversion; see miloc_run)         */
    MILOC_EBUSY = -7     /* resource exhausted (serving: no slot / budget)                           */
} miloc_status;

typedef struct miloc_ctx miloc_ctx;

/* Library version string, e.g. "miloc 0.1 gfx950". Static storage. */
const char* miloc_version(void);

/* Create a context on HIP device `hip_device`.  `hip_stream` (a hipStream_t)
 * may be NULL: the context then creates and owns a stream of default
 * priority.  *out receives the context.  Fails with MILOC_EDEVICE when the
 * device does not exist or is not gfx950. */
miloc_status miloc_create(int hip_device, void* hip_stream, miloc_ctx** out);

/* Release every device and host resource of the context.  NULL is allowed. */
void miloc_destroy(miloc_ctx* ctx);

/* Text of the last error on this context (static "" when none); valid until
 * the next call on the same context. */
const char* miloc_last_error(const miloc_ctx* ctx);

/* ---------------------------------------------------------------- molecule */
/* Level and transition tables of the species (Sect. 2: Einstein A, B and
 * collision coefficients; one collision partner, H2).
 *   n_levels        number of energy levels (2..32)
 *   E_K[n_levels]   level energy / k_B [K]
 *   g[n_levels]     statistical weights (> 0)
 *   n_trans         number of radiative transitions (1..n_levels*(n_levels-1)/2)
 *   up, lo[n_trans] level indices, up > lo, distinct pairs
 *   A[n_trans]      Einstein A_ul [s^-1] (> 0)
 *   nu_Hz[n_trans]  rest frequency [Hz] (> 0)
 *   gamma_down[n_levels*n_levels] downward collision rate coefficient
 *                   [cm^3 s^-1], entry [u*n_levels + l] for u > l (other
 *                   entries ignored); temperature independent.  Upward rates
 *                   follow from detailed balance at the local T_kin.
 *   mass_amu        molecular mass for the thermal line width.
 * Loading a molecule discards populations computed with a previous one. */
typedef struct {
    int n_levels;
    const double* E_K;
    const double* g;
    int n_trans;
    const int* up;
    const int* lo;
    const double* A;
    const double* nu_Hz;
    const double* gamma_down;
    double mass_amu;
} miloc_molecule;

miloc_status miloc_load_molecule(miloc_ctx* ctx, const miloc_molecule* mol);

/* ------------------------------------------------------------------ models */
/* 1D spherical model (Sect. 2.1): shell k spans (r_out[k-1], r_out[k]]
 * (r_out[-1] = 0), with values constant inside it.
 *   n_shells (1..65536); r_out strictly increasing, > 0 [cm];
 *   n_H2 [cm^-3] >= 0, T_kin [K] > 0, b_turb [cm/s] >= 0 (microturbulent
 *   Doppler parameter, added in quadrature to the thermal one),
 *   v_r [cm/s] radial velocity (positive outwards), abundance >= 0;
 *   n_rays (1..65536) impact-parameter rays; impact_cm NULL => equidistant
 *   b_j = (j + 1/2) R/n_rays, else n_rays strictly increasing values in (0, R).
 * Each ray's weight is the annulus between the mid-points of neighbouring
 * impact parameters. */
typedef struct {
    int n_shells;
    const double* r_out_cm;
    const double* n_H2;
    const double* T_kin;
    const double* b_turb_cms;
    const double* v_r_cms;
    const double* abundance;
    int n_rays;
    const double* impact_cm;
} miloc_model1d;

/* 3D model on an N^3 root grid of cubic cells of side root_cell_cm
 * (Sect. 2.2).  Root cell (x, y, z) has index (z*N + y)*N + x.
 *   n_oct_levels = 0: regular grid, 2 <= N <= 1024; n_cells_per_level and
 *     first_child are ignored and the fields hold N^3 values.
 *   n_oct_levels >= 1: octree with levels 0..n_oct_levels-1 (at most 12),
 *     1 <= N <= 1024.  n_cells_per_level[l] cells per level (level 0: N^3);
 *     cells are numbered level by level (global index = cells of the levels
 *     before + index in the level), at most 2^28 - 1 in all.  first_child[l][i]
 *     (l < n_oct_levels - 1) is the level-(l+1) index of the first of the 8
 *     children of cell i of level l, children ordered cx + 2 cy + 4 cz by
 *     their position in the parent, or -1 for a leaf; child blocks are
 *     multiples of 8, each claimed by exactly one parent, and the last level
 *     has no children.  The fields hold one value per cell of every level;
 *     values of refined cells are read but have no effect (their populations
 *     are left as set).  Rays follow the refinement (new rays where it
 *     increases, ending where it decreases); 48 directions give every leaf the
 *     same path length per unit size for each direction.
 * Per-cell float fields as in miloc_model1d plus the velocity vector
 * (vx, vy, vz) [cm/s].  The library copies everything it needs. */
typedef struct {
    int n0[3];
    int n_oct_levels;
    double root_cell_cm;
    const int64_t* n_cells_per_level;
    const int32_t* const* first_child;
    const float* n_H2;
    const float* T_kin;
    const float* b_turb_cms;
    const float* vx;
    const float* vy;
    const float* vz;
    const float* abundance;
} miloc_model3d;

/* Loading a model replaces the previous one (1D or 3D) and its populations. */
miloc_status miloc_load_model_1d(miloc_ctx* ctx, const miloc_model1d* model);
miloc_status miloc_load_model_3d(miloc_ctx* ctx, const miloc_model3d* model);

/* Ray schedule of an octree model for the given directions (Sect. 2.2), as
 * the octree march replays it; host computation only (needs no device or
 * context), for inspection and tests.  With steps_out and trees_out NULL only
 * the sizes are returned; otherwise steps_out receives 2 * n_steps words
 * (word 0: cell index in bits 0..27, bit 28 "save the incoming intensity",
 * bits 29..30 how the intensity starts: 0 continue, 1 background, 2 copy of
 * the last saved vector, 3 copy of it and drop it; word 1: the step length in
 * root-cell units as an IEEE float) and trees_out 4 * n_trees values (first
 * step, step count, direction, root element j*N + i), largest trees first.
 * plain = 1 traces the root lines alone (no new rays, no ending; lines of
 * sight), plain = 2 the brute-force lattice (every line of the finest level,
 * 4^Lmax per root element, traced straight; see miloc_set_octree_rays),
 * plain = 0 the octree scheme.  MILOC_EINVAL for an invalid model,
 * directions or plain. */
miloc_status miloc_octree_schedule(const miloc_model3d* model, int n_dir, const double* dirs, int plain,
                                   int64_t* n_steps, int64_t* n_trees, int* max_depth, uint32_t* steps_out,
                                   int64_t* trees_out);

/* Device memory a context holds for a model, host computation only (no
 * device or context needed): exactly one of m1 (1D) and m3 (3D) is given,
 * with the species' level and transition counts, the channel count, the 3D
 * ray directions (dirs[3*n_dir], or NULL for the 48 HEALPix ones) and the
 * march precision (MILOC_MARCH_FP32 / _FP64).  Octrees need the step count
 * of their ray schedule (oct_steps, from miloc_octree_schedule with the same
 * directions); it is ignored otherwise.  *fixed_bytes: populations,
 * opacities, sums and per-cell data, the channel-window table and the ray
 * tables (for octrees including 2 GiB for the saved-intensity stacks, their
 * cap); *sums_bytes: the 3D per-step partial sums of a march launch of one
 * transition (0 in 1D).  A context refuses, with MILOC_ENOMEM and before
 * allocating them, a 3D model whose fixed bytes plus one launch's sums
 * exceed the free device memory (or MILOC_DEVICE_BUDGET_GB, an environment
 * cap in GB for tests); with room, the launches take as many transitions as
 * fit (see MILOC_STEP_BUFFER_GB).  MILOC_EINVAL for invalid arguments. */
miloc_status miloc_model_footprint(const miloc_model1d* m1, const miloc_model3d* m3, int n_levels, int n_trans,
                                   int n_channels, int n_dir, const double* dirs, int precision, int64_t oct_steps,
                                   size_t* fixed_bytes, size_t* sums_bytes);

/* Velocity channels (Sect. 2: a regular velocity grid per ray):
 * centres v_c = v_min + (c + 1/2) dv, c = 0..n_channels-1 (8..4096).  The
 * band must contain every cell's line out to 5 Doppler widths at any
 * projected velocity (checked at miloc_run: MILOC_EINVAL). */
miloc_status miloc_set_spectral(miloc_ctx* ctx, int n_channels, double v_min_cms, double dv_cms);

/* Isotropic background B_nu(T_bg) entering at every ray start (Sect. 2,
 * Eq. (1)).  Default 2.73 K.  T_bg >= 0 (0 => no background). */
miloc_status miloc_set_background(miloc_ctx* ctx, double T_bg_K);

/* Hyperfine structure of transition `trans` with LTE between its components
 * (Sect. 1; the NH3(1,1) and HCN(1-0) examples of Sect. 3): the line profile
 * becomes sum_k w_k phi(v - dv_k), phi the cell's Gaussian, component k
 * centred at channel velocity dv_cms[k] - (u . d).  strength[k] > 0 are
 * relative strengths (normalised to sum 1 here); n_comp in
 * 0..MILOC_MAX_HF_COMPONENTS, 0 restores the single Gaussian.  The arrays
 * are copied.  The statistical equilibrium treats the multiplet as one
 * transition.  Needs the molecule; reset by miloc_load_molecule.  Every
 * transition's channel window then spans the lowest to the highest offset
 * of all multiplets plus the profile cut, and the band check of
 * miloc_set_spectral includes the offsets.  The 1D request loop
 * (miloc_server_*) serves single-Gaussian lines only.  Errors: MILOC_ESTATE
 * without a molecule, MILOC_EINVAL for a bad index, count, offset or
 * strength (state unchanged). */
#define MILOC_MAX_HF_COMPONENTS 32
miloc_status miloc_set_hyperfine(miloc_ctx* ctx, int trans, int n_comp, const double* dv_cms,
                                 const double* strength);

/* Rays of the octree march (Sect. 2.2).  MILOC_OCT_RAYS_SCHEME (default):
 * rays created on entering refined cells and through side faces, ended in
 * coarser cells, each of the level of the cells it crosses.
 * MILOC_OCT_RAYS_LATTICE: the brute-force alternative the paper weighs
 * against it, a regular lattice of 4^Lmax straight lines per root surface
 * element (Lmax = the deepest level), each of weight h_Lmax^2 |d_m|, no rays
 * created or ended (cost grows as 4^Lmax: for shallow trees).  Applies to
 * octree models (ignored otherwise); the ray schedule is rebuilt at the next
 * miloc_run, which returns MILOC_EINVAL when the lattice could exceed 4e9
 * steps ((N 2^Lmax)^2 lines per direction of at most 3 N 2^Lmax steps).
 * MILOC_EINVAL for another value of rays. */
#define MILOC_OCT_RAYS_SCHEME 0
#define MILOC_OCT_RAYS_LATTICE 1
miloc_status miloc_set_octree_rays(miloc_ctx* ctx, int rays);

/* 3D ray directions: the 12*nside^2 HEALPix pixel centres (Sect. 2.2; 48 for
 * nside = 2, the default).  nside 1..8. */
miloc_status miloc_set_directions_healpix(miloc_ctx* ctx, int nside);

/* 3D ray directions given explicitly: n_dir (1..1024) vectors, dirs[3*n_dir],
 * normalised by the library (zero vectors: MILOC_EINVAL).  Each direction
 * stands for a solid angle 4 pi / n_dir. */
miloc_status miloc_set_directions(miloc_ctx* ctx, int n_dir, const double* dirs);

/* How a 1D model's iterations march the transitions (Sect. 4 of the paper
 * proposes processing all transitions at the same time instead of repeating
 * the ray tracing per transition): on = 0 (default) one launch covers every
 * (ray, transition) pair independently; on = 1 one wavefront marches one ray
 * for four transitions at once, sharing the ray's steps, the shells' data and
 * the line profile of each step (the same in velocity units for every
 * transition), with the absorbed counts summed by FP64 device atomics.  The
 * results are the same to FP32 (FP64) rounding.  Lines of sight, core
 * sub-iterations and hyperfine multiplets march per transition.  Ignored
 * for 3D models.  MILOC_EINVAL unless on is 0 or 1. */
miloc_status miloc_set_transition_batching(miloc_ctx* ctx, int on);

/* Arithmetic of the ray march: MILOC_MARCH_FP32 (default; FP32 intensities,
 * FP64 accumulation) or MILOC_MARCH_FP64 (everything in FP64). */
typedef enum { MILOC_MARCH_FP32 = 0, MILOC_MARCH_FP64 = 1 } miloc_march_precision;
miloc_status miloc_set_march_precision(miloc_ctx* ctx, int precision);

/* Sub-iterations in the optically thick core of a 1D model (the paper's
 * Sect. 4 proposes updating the populations more often where the lines are
 * thick).  After every iteration's global solve, the core -- shells 0..K,
 * K the outermost shell whose radial line-centre optical depth to the
 * model's surface (static gas, the new populations, any transition) reaches
 * tau_min -- is iterated n_sub more times on its own: the rays that reach
 * it march their inward envelope steps once (the intensity they enter the
 * core with, from the envelope's new populations, which stay fixed), then
 * n_sub times the core pieces of those rays are marched from those entry
 * intensities and the core shells are solved (ALI form, weights W of the
 * full ray set).  The convergence measure stays that of the global solve.
 * The fixed point is that of plain ALI; thick cores need fewer iterations.
 * n_sub = 0 (default) turns it off.  miloc_run returns MILOC_EINVAL when
 * n_sub > 0 with a 3D model, use_ali = 0 or a hyperfine multiplet.  Errors
 * here: MILOC_EINVAL for n_sub outside 0..1000 or a non-finite tau_min. */
miloc_status miloc_set_subiterations(miloc_ctx* ctx, int n_sub, double tau_min);

/* ------------------------------------------------------------- iteration */
/* Populations = Boltzmann distribution at T_kin in every cell (LTE start,
 * Sect. 3.3.2).  Needs a model and a molecule. */
miloc_status miloc_init_lte(miloc_ctx* ctx);

/* Populations from the caller: x[n_cells*n_levels], cell-major; each row is
 * renormalised to sum 1; negative or non-finite entries => MILOC_EINVAL.
 * Together with miloc_get_populations this is the checkpoint/resume pair. */
miloc_status miloc_set_populations(miloc_ctx* ctx, const double* x);

/* Run up to max_iter (>= 1) iterations.  One iteration = for every
 * transition, march all rays with the current populations and accumulate
 * the absorbed counts and the diagonal operator per cell; then solve the
 * statistical equilibrium of every cell (FP64); then the convergence test
 * delta = max |x_new - x_old| / x_new over x_new >= 1e-10 (FP64, on the
 * device).  use_ali != 0 selects the ALI form (Sect. 2), 0 the plain lambda
 * iteration.  Stops early when delta < tol (tol <= 0: never).  Populations
 * are initialised to LTE if none are set.  iters_done / last_delta may be
 * NULL.  Returns MILOC_ENOTCONV when tol > 0 was not met (state is valid).
 * Inverted populations (negative opacity, a maser) are marched as written as
 * long as no single step's line-centre optical depth falls below -40; such a
 * step stops the run with MILOC_ENUMERIC and the populations of the failed
 * iteration are not kept (miloc_get_spectra refuses it the same way). */
miloc_status miloc_run(miloc_ctx* ctx, int max_iter, double tol, int use_ali,
                       int* iters_done, double* last_delta);

/* Sizes of the loaded problem (any pointer may be NULL). */
miloc_status miloc_get_sizes(const miloc_ctx* ctx, int64_t* n_cells, int* n_levels,
                             int* n_trans, int* n_channels);

/* Current populations x[n_cells*n_levels] (cell-major). */
miloc_status miloc_get_populations(miloc_ctx* ctx, double* x_out);

/* Radiation terms of the last iteration, each [n_trans*n_cells]
 * (transition-major): J = mean intensity of the external field weighted by
 * the line profile [erg s^-1 cm^-2 Hz^-1 sr^-1] (with the plain lambda
 * iteration: the full field), lambda = diagonal operator (1 - escape
 * probability).  Either pointer may be NULL. */
miloc_status miloc_get_radiation(miloc_ctx* ctx, double* J_out, double* lambda_out);

/* Spectra of transition `trans` from the current populations by a final
 * line-of-sight march (Sect. 2), dI = I - I_bg per channel
 * [erg s^-1 cm^-2 Hz^-1 sr^-1], dI_out[n_los*n_channels].
 *   1D: n_los rays at impact parameters impact_cm[n_los] (in [0, R)), or the
 *       model's own ray set when impact_cm is NULL (n_los must then equal
 *       n_rays).
 *   3D: a map towards +z, one line of sight per (x, y) cell column through
 *       the cell centres; n_los must be N*N, index y*N + x; impact_cm NULL. */
miloc_status miloc_get_spectra(miloc_ctx* ctx, int trans, int n_los, const double* impact_cm,
                               double* dI_out);

/* Counters since the last reset (miloc_reset_counters). */
typedef struct {
    int64_t iterations;          /* ALI/LI iterations run                                    */
    int64_t march_launches;      /* launches of the ray-march kernel                          */
    double march_ms;             /* summed device time of those launches (HIP events)        */
    double accumulate_ms;        /* per-cell gather of the march's per-step sums (3D grids)  */
    double prepare_ms;           /* populations -> opacity/emissivity kernels                */
    double solve_ms;             /* statistical equilibrium + convergence kernels            */
    double ray_steps;            /* ray-cell steps per transition, summed over launches      */
    double channel_updates;      /* ray_steps x n_channels (nominal, window not subtracted)  */
    int32_t march_lanes;         /* lanes per ray of the march kernel (set by the first run) */
    int32_t reserved;
} miloc_counters;

miloc_status miloc_get_counters(const miloc_ctx* ctx, miloc_counters* out);
miloc_status miloc_reset_counters(miloc_ctx* ctx);

/* ----------------------------------------------------------------- serving */
/* A request loop for 1D models (continuous batching).  Requests are queued by
 * miloc_server_submit (inputs copied before return) and admitted by an
 * admission thread of the server when one of max_slots slots is free and the
 * request's device footprint fits in the remaining part of hbm_budget_bytes
 * (first fit in arrival order); admission (host image, upload, device set-up
 * on a stream of its own) runs while the worker thread's ticks run, and the
 * model joins at the next tick after it.  Each tick advances every resident
 * model by one ALI
 * iteration (Sect. 2: march all transitions, FP32 with FP64 accumulation; FP64
 * equilibrium solves; FP64 convergence test per model) through one captured
 * HIP graph; models join and leave between ticks.  A model finishes when its
 * maximum relative change drops below tol (MILOC_OK), after max_iter
 * iterations (MILOC_ENOTCONV if tol > 0), or on a numerical failure
 * (MILOC_ENUMERIC); a failing request does not disturb the others.  On
 * completion the server computes the spectra of every transition towards the
 * model centre (impact parameter 0).  All server calls are thread-safe.
 * Limits per request: 2..20 levels, at most 19 transitions x 8192 rays,
 * 1..2048 shells, 8..512 channels. */
typedef struct miloc_server miloc_server;

typedef struct {
    int iterations;       /* ALI iterations run                                   */
    double last_delta;    /* maximum relative change of the last iteration        */
    double latency_s;     /* submit -> result ready (host clock)                  */
    double queue_s;       /* submit -> admitted                                   */
    int status;           /* miloc_status of the request                          */
} miloc_result_info;

typedef struct {
    int64_t submitted, admitted, completed, failed, cancelled;
    int64_t queued, active, peak_active;   /* current / largest number resident   */
    int64_t ticks;                         /* graph replays                        */
    double busy_s;                         /* host time spent in ticks             */
    int64_t arena_used;                    /* device bytes held by resident models */
} miloc_server_stats;

/* hbm_budget_bytes (>= 1 MiB) is allocated up front as the arena of resident
 * models; max_slots in 1..4096.  The worker and admission threads start
 * immediately. */
miloc_status miloc_server_create(int hip_device, size_t hbm_budget_bytes, int max_slots, miloc_server** out);

/* Stops the admission and worker threads (after the current admission round
 * and tick); queued requests are dropped. */
void miloc_server_destroy(miloc_server* server);

const char* miloc_server_last_error(const miloc_server* server);

/* Queue one request.  n_channels, v_min_cms, dv_cms as miloc_set_spectral;
 * T_bg_K as miloc_set_background; tol > 0 is the convergence threshold of
 * the maximum relative population change.  *ticket identifies the request.
 * MILOC_EINVAL for invalid inputs (nothing queued), MILOC_EBUSY if the
 * request can never fit the budget. */
miloc_status miloc_server_submit(miloc_server* server, const miloc_molecule* mol, const miloc_model1d* model,
                                 int n_channels, double v_min_cms, double dv_cms, double T_bg_K, double tol,
                                 int max_iter, uint64_t* ticket);

/* Device bytes the request would hold in the server's arena while resident
 * (validates the inputs exactly as miloc_server_submit does; queues nothing).
 * Lets a caller size hbm_budget_bytes. */
miloc_status miloc_server_footprint(miloc_server* server, const miloc_molecule* mol, const miloc_model1d* model,
                                    int n_channels, double v_min_cms, double dv_cms, double T_bg_K,
                                    size_t* bytes);

/* *done = 1 when the request has finished (any status). */
miloc_status miloc_server_poll(miloc_server* server, uint64_t ticket, int* done);

/* Block until the request finishes or timeout_s elapses; *done as poll. */
miloc_status miloc_server_wait(miloc_server* server, uint64_t ticket, double timeout_s, int* done);

/* Sizes of a request's results. */
miloc_status miloc_server_result_sizes(miloc_server* server, uint64_t ticket, int* n_shells, int* n_levels,
                                       int* n_trans, int* n_channels);

/* Results of a finished request, which is then forgotten: populations
 * x_out[n_shells*n_levels], centre spectra dI[n_trans*n_channels]
 * (erg s^-1 cm^-2 Hz^-1 sr^-1), info.  Any output pointer may be NULL.
 * Returns the request's status (MILOC_ESTATE if not finished yet or
 * cancelled). */
miloc_status miloc_server_take(miloc_server* server, uint64_t ticket, double* x_out, double* spectra_out,
                               miloc_result_info* info);

/* Cancel a queued or resident request (a resident one leaves after the
 * current tick). */
miloc_status miloc_server_cancel(miloc_server* server, uint64_t ticket);

miloc_status miloc_server_get_stats(miloc_server* server, miloc_server_stats* out);

/* ------------------------------------------------- allocation-free 1D solve */
/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc or hipFree: tight request loops, harnesses that forbid device
 * allocation).  Solves one 1D model exactly as
 *   miloc_create(hip_device, hip_stream) + miloc_load_molecule(mol) +
 *   miloc_load_model_1d(model) + miloc_set_spectral(n_channels, v_min_cms,
 *   dv_cms) + miloc_set_background(T_bg_K) + miloc_run(max_iter, tol, ALI)
 *   + miloc_get_populations(x_out) + miloc_destroy
 * would (FP32 march, FP64 solves; the same kernels), but every device buffer
 * lives in a static device array of MILOC_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends; the call
 * allocates no device memory, creates no stream or event and keeps no
 * counters.  Inputs are host buffers, copied in; x_out[n_shells*n_levels]
 * (host, caller-allocated) receives the populations, iters_done and
 * last_delta (either may be NULL) the iteration count and the last maximum
 * relative change.  Work runs on hip_stream (NULL: the null stream) and is
 * complete when the call returns.
 * Errors: as the calls above (MILOC_ENOTCONV still writes the results);
 * MILOC_ENOMEM when the model needs more device memory than the scratch
 * holds (roughly: 8 bytes per ray step, with n_rays*n_shells steps at most,
 * plus 40 bytes per shell and level or transition; about 2500 shells with as
 * many rays).  Calls that overlap on one GPU (from several threads) share
 * the one array and race: serialise them. */
#define MILOC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
miloc_status miloc_solve_1d_noalloc(int hip_device, void* hip_stream, const miloc_molecule* mol,
                                    const miloc_model1d* model, int n_channels, double v_min_cms, double dv_cms,
                                    double T_bg_K, int max_iter, double tol, int* iters_done, double* last_delta,
                                    double* x_out);

#ifdef __cplusplus
}
#endif
#endif /* MILOC_H */
