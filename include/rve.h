/*
 * rve.h - C ABI of the MI355X (gfx950) Galerkin-FFT homogenization solver for lattice materials
 * with empty (zero-stiffness) phases.
 *
 * Method (paper: "Adaptation and validation of FFT methods for homogenization of lattice based
 * materials", section "Galerkin-FFT with discrete differences and mixed loading control"):
 * find the periodic, compatible, zero-mean strain fluctuation eps on a regular voxel grid such that
 *     F^{-1}{ Ghat(xi') : F{ C(x) : eps } } = - F^{-1}{ Ghat(xi') : F{ C(x) : Ebar } }     (eq. gallin)
 * with C(x) = phi(x) C_solid + (1 - phi(x)) C_void (Voigt rule, section "Voigt approaches"), the
 * projection Ghat of eq. (galop) under pure strain control, the rotated forward-difference modified
 * frequencies xi' of eq. (freqrot), and MINRES as the Krylov solver; convergence is tested on the
 * relative residual of eq. (galres).
 *
 * Conventions used by every entry point
 *   - grid: n[0] x n[1] x n[2] voxels, axis 2 contiguous; voxel sizes h_p = L[p] / n[p].
 *   - tensors are Mandel 6-vectors (11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12); the Euclidean dot
 *     product of two Mandel vectors is the Frobenius product of the tensors.
 *   - fields are component-major: field[case][component][i0][i1][i2].
 *   - "device" pointers are HIP device memory on the current device; "host" pointers are host memory.
 *   - the caller owns every buffer.  The library keeps no pointer after a call returns and never
 *     allocates device memory: all scratch comes from the caller's workspace.
 *   - calls run on the given HIP stream (NULL = default stream); host outputs are written and the
 *     stream is synchronised before the call returns.  solve_rve captures each chunk of check_every
 *     MINRES iterations (rounded up to a multiple of 6) into a HIP graph that it replays until
 *     convergence and keeps cached for the next call with the same buffers (capture needs a non-NULL
 *     stream; with the NULL stream, or RVE_DISABLE_GRAPHS=1 in the environment, it launches directly).
 *     The captured graphs, the second stream of solve_rve and their events are cached per (device,
 *     solve stream), process-wide and mutex-guarded, and freed by rve_release_caches(); solves on
 *     different threads and streams may run concurrently.
 *   - argument validation happens on the host before any HIP call; a rejected call touches no
 *     device state.
 */
#ifndef RVE_H
#define RVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RVE_OK = 0,
  RVE_NOT_CONVERGED = 1,     /* max_iter reached; outputs hold the last iterate */
  RVE_BREAKDOWN = 2,         /* MINRES rotation with zero norm (inconsistent singular system) */
  RVE_EINVAL = -1,           /* bad argument (null pointer, non-finite or out-of-range value) */
  RVE_EUNSUPPORTED_SIZE = -2,/* a grid length the FFT kernels do not provide */
  RVE_ENONFINITE = -3,       /* non-finite input or a non-finite Krylov scalar during the solve */
  RVE_ENOMEM = -4,           /* workspace smaller than rve_workspace_bytes() */
  RVE_EDEVICE = -5           /* a HIP runtime error */
} rve_status;

enum { RVE_FP32_MIXED = 0, RVE_FP64 = 1 };
enum { RVE_SCHEME_ROTATED = 0, RVE_SCHEME_CONTINUOUS = 1 };
enum { RVE_NYQ_NATURAL = 0, RVE_NYQ_ZERO_ALL = 1 };
enum { RVE_APPLY_OPERATOR = 0, RVE_APPLY_PROJECTION = 1, RVE_APPLY_STIFFNESS_ROUNDTRIP = 2 };

typedef struct {
  int32_t n[3]; /* voxels per axis, each a length rve_supported_length() accepts */
  double L[3];  /* cell edge lengths (> 0) */
} rve_grid;

typedef struct {
  double tol;           /* relative residual target ||A eps - b|| / ||b||  (eq. galres), > 0 */
  int32_t max_iter;     /* MINRES iterations cap per load case (summed over refinement sweeps) */
  int32_t precision;    /* RVE_FP32_MIXED: FP32 fields and transforms, FP64 scalars, inner products,
                           true residual and refinement;  RVE_FP64: everything FP64 */
  int32_t max_refine;   /* FP32_MIXED: maximum FP64 residual-refinement sweeps (>= 1) */
  int32_t nyquist;      /* RVE_NYQ_NATURAL (default): the projection vanishes only where the
                           modified frequency vanishes; RVE_NYQ_ZERO_ALL: also at every Nyquist index */
  int32_t scheme;       /* RVE_SCHEME_ROTATED (eq. freqrot, default) or RVE_SCHEME_CONTINUOUS (eq. freq) */
  int32_t check_every;  /* iterations between host checks of the convergence flags (>= 1) */
  double inner_floor;   /* FP32_MIXED: an inner FP32 sweep stops no later than at this fraction of its
                           own starting residual (default 3e-2; in (0, 1)).  FP32 Lanczos on these
                           near-singular operators stalls when asked for much deeper reductions; the
                           FP64 refinement restarts from the true residual instead */
  double inner_safety;  /* FP32_MIXED: an inner sweep aims at inner_safety * tol * ||b|| (default 0.9; the
                           FP64 residual decides, so a sweep that ends just above tol is followed by
                           another one) */
  int32_t stress_mask;  /* mixed macroscopic control (eq. galop, eq. gallin; section "Galerkin-FFT with
                           discrete differences and mixed loading control"): bit a set = Mandel component
                           a (0..5 = 11, 22, 33, 23, 13, 12) is stress-controlled, the others
                           strain-controlled.  0 (default): pure strain control.  The projection at
                           xi = 0 is then the identity on the stress-controlled components, and the
                           fluctuation's mean over them is the macroscopic strain they take */
  const double* macro_stress; /* host [n_cases][6] Mandel macroscopic stress; only the stress-controlled
                           components are read (NULL: zero, e.g. uniaxial stress).  The macroscopic
                           strain's stress-controlled components are ignored.  Read during the call only */
} rve_options;

/* Fills *opt with the defaults: tol 1e-6, max_iter 5000, FP32_MIXED, max_refine 24, natural Nyquist,
 * rotated scheme, check_every 24, inner_floor 3e-2, inner_safety 0.9, stress_mask 0 (strain control),
 * macro_stress NULL. */
void rve_default_options(rve_options* opt);

/* 1 if the FFT kernels provide axis length n, else 0: every n in [2, 256] without a prime factor
 * above 5 (n = NA*NB, each stage a register DFT composed of radix 2, 3, 4 and 5 steps). */
int32_t rve_supported_length(int32_t n);

/* Host-side validation of a solve_rve call's scalar arguments (no HIP call, no pointer dereference
 * of device buffers).  Returns RVE_OK or the error solve_rve would return. */
rve_status rve_validate(const rve_grid* grid, const double* phase_stiffness, const double* macro_strain,
                        int32_t n_cases, const rve_options* opt);

/* Workspace bytes solve_rve needs for this grid, number of load cases and options (0 on bad input). */
size_t rve_workspace_bytes(const rve_grid* grid, int32_t n_cases, const rve_options* opt);

/* Galerkin-FFT homogenization of one RVE under n_cases macroscopic loads (eq. gallin): macro strains, or
 * with opt->stress_mask mixed strain/stress control.
 *   voxel_fraction_field  device float [N]: solid fraction phi in [0,1] of each voxel (Voigt rule)
 *   phase_stiffness       host double [2][36]: Mandel 6x6 stiffness of the empty phase ([0], usually
 *                         all zero) and of the solid ([1]); each must be symmetric and finite
 *   macro_strain          host double [n_cases][6]: Mandel macro strains Ebar
 *   eps0                  device [n_cases][6][N] warm start (float for FP32_MIXED, double for FP64) or
 *                         NULL for the zero start; it is projected onto compatible fields first,
 *                         and a case whose projected start has ||b - A x0|| >= ||b|| starts from
 *                         zero instead (see rve_last_solve_info)
 *   strain_out            device [n_cases][6][N] (float / double): the fluctuation eps (total = Ebar+eps,
 *                         Ebar without its stress-controlled components; see rve_last_mean_strain)
 *   stress_out            device [n_cases][6][N] (float / double) or NULL: sigma = C(x)(Ebar + eps)
 *   eff_stress            host double [n_cases][6]: volume average <sigma> (FP64); for unit Mandel
 *                         macro strains e_J this is column J of the effective stiffness
 *   iterations            host int32 [n_cases]: MINRES iterations (operator applications in the loop)
 *   rel_residual          host double [n_cases]: ||b - A eps|| / ||b|| recomputed in FP64 at exit
 * Work is queued on hip_stream and on a second stream the library creates once per (device, solve
 * stream) and keeps cached (default priority), joined back into hip_stream before every host check;
 * the call returns after hip_stream has finished.  Returns the worst status over the load cases.
 * A right-hand side that counts as zero (homogeneous or all-empty cell, zero macro strain; ||b|| at the
 * rounding level of the transforms of a constant field) returns eps = 0 exactly and 0 iterations,
 * also when a warm start eps0 is given. */
rve_status solve_rve(const rve_grid* grid, const float* voxel_fraction_field, const double* phase_stiffness,
                     const double* macro_strain, int32_t n_cases, const rve_options* opt, const void* eps0,
                     void* strain_out, void* stress_out, double* eff_stress, int32_t* iterations,
                     double* rel_residual, void* workspace, size_t workspace_bytes, void* hip_stream);

/* One RVE of a heterogeneous batch: the arguments of a solve_rve call (see there), plus its status. */
typedef struct {
  rve_grid grid;
  const float* voxel_fraction_field; /* device [N] */
  const double* phase_stiffness;     /* host [2][36] */
  const double* macro_strain;        /* host [n_cases][6] */
  int32_t n_cases;
  const void* eps0;                  /* device [n_cases][6][N] or NULL */
  void* strain_out;                  /* device [n_cases][6][N] */
  void* stress_out;                  /* device [n_cases][6][N] or NULL */
  double* eff_stress;                /* host [n_cases][6] */
  int32_t* iterations;               /* host [n_cases] */
  double* rel_residual;              /* host [n_cases] */
  const double* macro_stress;        /* host [n_cases][6] or NULL: this RVE's macroscopic stress under
                                        mixed control (replaces opt->macro_stress for this item) */
  double* mean_strain;               /* host [n_cases][6] or NULL: total macroscopic strain per case
                                        (as rve_last_mean_strain) */
  int32_t status;                    /* out: this RVE's status (as solve_rve's) */
} rve_batch_item;

/* Workspace for solve_rve_batch: per group of RVEs with the same grid and phase stiffness, the
 * workspace of one solve over all their load cases plus a copy of each case's phase map (and, where an
 * item has a warm start, of the warm starts).  0 on a bad item. */
size_t rve_batch_workspace_bytes(const rve_batch_item* items, int32_t n_items, const rve_options* opt);

/* Many RVEs of uneven size (each with its own grid, phase map and load cases) in one solve (the batched
 * form of eq. gallin): RVEs with equal grid and phase stiffness are grouped, and each group is one
 * multi-case solve whose cases carry their own phase map; all groups run their FP32 sweeps and FP64
 * refinements in lockstep, and the MINRES iterations of all groups are one captured HIP graph whose
 * parallel branches are the groups (replayed chunk by chunk until every case of every RVE has
 * finished; a finished case's kernels return at once).  Results equal those of solve_rve on each item
 * (same per-case arithmetic).  All items are validated before any work starts.  Runs on hip_stream
 * (the library's branch streams fork from it and join back); returns the worst status, per-item
 * statuses are in items[i].status.  Differs from solve_rve in one respect: rve_last_solve_info and
 * rve_last_mean_strain are not updated (use items[i].mean_strain). */
rve_status solve_rve_batch(rve_batch_item* items, int32_t n_items, const rve_options* opt, void* workspace,
                           size_t workspace_bytes, void* hip_stream);

/* Workspace bytes rve_apply needs. */
size_t rve_apply_workspace_bytes(const rve_grid* grid, int32_t n_cases, int32_t precision);

/* One application of the Galerkin operator pieces to n_cases fields (eq. linearOp):
 *   mode RVE_APPLY_OPERATOR:            y = F^{-1}{ Ghat : F{ C(x) : x } }
 *   mode RVE_APPLY_PROJECTION:          y = F^{-1}{ Ghat : F{ x } }       (C = identity)
 *   mode RVE_APPLY_STIFFNESS_ROUNDTRIP: y = F^{-1}{ F{ C(x) : x } }       (Ghat = identity)
 * x, y: device [n_cases][6][N] float (precision RVE_FP32_MIXED) or double (RVE_FP64); phase_stiffness
 * as in solve_rve (ignored for PROJECTION); stress_mask as in rve_options (Ghat at xi = 0). */
rve_status rve_apply(const rve_grid* grid, const float* voxel_fraction_field, const double* phase_stiffness,
                     int32_t n_cases, int32_t precision, int32_t scheme, int32_t nyquist, int32_t stress_mask,
                     int32_t mode, const void* x, void* y, void* workspace, size_t workspace_bytes,
                     void* hip_stream);

/* Optional per-kernel timing (instrumentation for benchmarks, not on by default).  When enabled,
 * every kernel launched inside the MINRES iteration loop of solve_rve is bracketed by HIP events
 * recorded on the solve stream; elapsed times are accumulated per kernel kind at the host's
 * convergence checks.  Kinds, in order: P1 stiffness + FFT axis 2 (+ Lanczos alpha), P2 FFT axis 1,
 * P3 FFT axis 0 + projection + inverse, P4 inverse FFT axis 1, P5 inverse FFT axis 2 + Lanczos
 * update, S1 Lanczos alpha (now computed by extra blocks of P2, so this kind records no launches
 * and P2's time includes it), S2 Givens step, U2 direction + solution update; kinds 0-7 count these
 * passes on FP32 fields, kinds 8-15 (names ending in _f64) the same passes on FP64 fields.
 * rve_profile_read fills total milliseconds and launch counts for up to max_kinds kinds and
 * returns the number of kinds (16).  Profiled solves launch their kernels directly (no graph
 * replay) and one at a time, so each launch can be bracketed and is timed alone; an unprofiled
 * solve runs U2 on a second stream beside the next iteration's P3 (solve_rve).
 * Launch counts include the iterations of the last launched chunk after convergence, whose kernels
 * return at once (a few microseconds each); divide by the iteration count for the time of a
 * working launch. */
void rve_profile_enable(int32_t on);
void rve_profile_reset(void);
int32_t rve_profile_read(double* total_ms, int64_t* launches, int32_t max_kinds);
const char* rve_profile_kind_name(int32_t kind);

/* Autotuner.  Times the operator apply for each registered factorisation N = NA * NB of every axis
 * length (e.g. 64 = 8*8 or 16*4, 96 = 12*8 or 16*6), the P3 component split (whole / halves, and
 * for FP64 also thirds) and every
 * admissible tile width of each pass kind (P3 pencils per block, P2/P4 rows per block, P1/P5 rows
 * per block; coordinate descent, HIP events on
 * hip_stream, 10 repetitions each) for this grid and precision, using the caller's workspace (at least
 * rve_workspace_bytes(grid, n_cases, default options of that precision)).  The fastest tiles are kept
 * in a process-wide table used by every later solve_rve / rve_apply on the same grid and precision,
 * and, if cache_path is non-NULL, the whole table is written there (one JSON object per line).
 * best_ms (host, may be NULL) receives the tuned apply time in milliseconds. */
rve_status rve_autotune(const rve_grid* grid, int32_t n_cases, int32_t precision, void* workspace,
                        size_t workspace_bytes, void* hip_stream, const char* cache_path, double* best_ms);

/* Loads a table written by rve_autotune (also read once from $RVE_TUNE_FILE when the library first
 * plans a grid).  Returns the number of entries loaded, -1 if the file cannot be read. */
int32_t rve_load_tuning(const char* path);

/* Tiles the next call on this grid and precision will use: tiles7 = {P1/P5 rows, P3 pencils,
 * P2/P4 rows, P3 component split in effect (1: six components per thread, 2: three per thread over
 * two block halves, each whole 64-lane waves; 3: two per thread over three one-wave groups, which
 * needs NB of axis 0 to divide 64), then for axes 0, 1, 2 the
 * first-stage radix NA of the factorisation N = NA * NB in use}.  Returns 1 if they come from the
 * tuner, 0 if they are the built-in heuristic. */
int32_t rve_tuned_tiles(const rve_grid* grid, int32_t precision, int32_t* tiles7);

/* Text of the last HIP runtime failure behind an RVE_EDEVICE in this thread ("" if none). */
const char* rve_last_error(void);

/* Start of the last solve_rve that returned on this thread, per load case (first max_cases):
 * initial_rel_residual[c] = ||b - A x0|| / ||b|| of the start x0 (0 for a zero right-hand side; 1 for
 * a zero start), warm_rejected[c] = 1 if a warm start eps0 was dropped because that ratio was not
 * below 1 (the solve then started from zero).  Either pointer may be NULL.  Returns the number of
 * cases of that solve (0 if none). */
int32_t rve_last_solve_info(double* initial_rel_residual, int32_t* warm_rejected, int32_t max_cases);

/* For callers that cannot allocate (code that may not call hipMalloc, tight serving loops, harnesses
 * that forbid allocation): solve_rve without a workspace argument.  Same arguments, outputs, statuses
 * and arithmetic as solve_rve; the caller still passes inputs and outputs.  Its scratch is a static
 * device array of rve_noalloc_scratch_bytes() bytes (128 MiB) compiled into the library, one copy per
 * GPU, held until the process ends; its address is looked up once per device on the first call there.
 * A solve whose rve_workspace_bytes() exceeds that size returns RVE_ENOMEM (rve_last_error() says by
 * how much) before any device work.  The call allocates no device memory and creates no HIP runtime
 * objects (no streams, events or graphs): the direction update runs on hip_stream and every kernel is
 * launched directly.  Every call on one GPU shares that GPU's scratch, which keeps the last call's
 * contents (each call initialises what it reads): calls that overlap on one GPU, from several host
 * threads or streams, race and must be serialised by the caller. */
rve_status solve_rve_noalloc(const rve_grid* grid, const float* voxel_fraction_field,
                             const double* phase_stiffness, const double* macro_strain, int32_t n_cases,
                             const rve_options* opt, const void* eps0, void* strain_out, void* stress_out,
                             double* eff_stress, int32_t* iterations, double* rel_residual, void* hip_stream);

/* Size in bytes of the static scratch solve_rve_noalloc works in (per GPU). */
size_t rve_noalloc_scratch_bytes(void);

/* Frees every cached runtime object the solvers keep between calls: the captured iteration graphs,
 * the second (U2) streams and their events, per (device, solve stream).  Sets in use by a solve that
 * is running on another thread at that moment are kept.  The next solve recreates what it needs.
 * Returns the number of cache sets freed.  (Ownership paragraph of the boundary: the library keeps no
 * device memory of its own; this releases the remaining runtime handles.) */
int32_t rve_release_caches(void);

/* Counts of the cached runtime objects (for leak checks): counts4 = {cache sets, side streams, events,
 * instantiated graphs}; counts4 may be NULL.  Returns the number of cache sets. */
int32_t rve_cache_counts(int64_t* counts4);

/* Total macroscopic strain of the last solve_rve that returned on this thread, per load case (first
 * max_cases): mean_strain [max_cases][6] = Ebar (strain-controlled components) + <eps>, in FP64; under
 * mixed control its stress-controlled components are the strains the prescribed stress produces (e.g.
 * E = <sigma_11> / mean_strain_11 and nu = -mean_strain_22 / mean_strain_11 under uniaxial stress).
 * Returns the number of cases of that solve. */
int32_t rve_last_mean_strain(double* mean_strain, int32_t max_cases);

/* Human-readable name of a status code (static string). */
const char* rve_status_string(rve_status s);

#ifdef __cplusplus
}
#endif

#endif /* RVE_H */
