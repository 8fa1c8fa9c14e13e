/*
 * rwpt.h -- C ABI of the MI355X (gfx950) library for the particle-to-particle
 * mass-transfer step of interacting random-walk particle tracking
 * (Engdahl, Schmidt & Benson, arXiv:1811.05474).
 *
 * One call of rwpt_step advances every realisation of an ensemble by n steps.
 * A step is, in this order (Sec. 1.1 and Sec. 7 of the paper):
 *   1. the random-walk move of Eq. (1)/(2), x <- x + sqrt(2 D_rw dt) dW (plus,
 *      with a velocity, the drift v dt and the hydrodynamic dispersion), with
 *      reflection at the zero-flux box walls (Sec. 3); D_rw = rw_ratio * D (the
 *      "mixed" diffusion split of Sec. 2.2 and Sec. 3, where each operation
 *      applies half of the total);
 *   2. the neighbour search: every pair with separation within the cutoff
 *      s_max = kappa * sigma, sigma = sqrt(8 D dt) (Sec. 2.1, Sec. 2.2);
 *   3. the co-location weights w_ij = exp(-s_ij^2 / (8 D dt)) of Eq. (3), their
 *      normalisation (Sec. 1.1, after Eq. 3) and the explicit exchange of
 *      Eqs. (4) and (6) for every species, from beginning-of-step masses and
 *      positions (the "matrix explicit" scheme of Sec. 1.1);
 *   4. the irreversible reaction A + B -> 0 evaluated per particle after the
 *      transfer (Sec. 3, Sec. 7), and an FP64 audit of the species totals and
 *      of sum(A - B), which the transfer and the reaction both conserve.
 *
 * Conventions
 *   - Every call returns an rwpt_status; nothing aborts or exits.  On error the
 *     context is left as it was and rwpt_last_error() describes the failure.
 *   - Host arrays are read (init) or written (query) in the caller's particle
 *     order: particle i of realisation r has global index off_r + i where off_r
 *     is the sum of the sizes of realisations 0..r-1.
 *   - Positions are N x dim row-major doubles (pos[i*dim + k]); masses are
 *     species-major doubles (mass[s*N + i]).  In the FP32 form they are rounded
 *     to binary32 on entry and widened exactly on exit.
 *   - The context owns all device memory.  A context is used by one host thread
 *     at a time; several contexts may share a device.
 *   - Work is queued on the configured HIP stream; rwpt_step returns before the
 *     GPU finishes.  Query and audit calls synchronise that stream.
 */
#ifndef RWPT_H
#define RWPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RWPT_OK = 0,
  RWPT_EINVAL = -1,      /* invalid argument or configuration */
  RWPT_ENOMEM = -2,      /* host or device allocation failed */
  RWPT_EDEVICE = -3,     /* HIP runtime error, or no usable gfx950 device */
  RWPT_ESTATE = -4,      /* call not valid in the current state (e.g. step before init) */
  RWPT_EUNSUPPORTED = -5 /* valid but not supported combination */
} rwpt_status;

enum { RWPT_FP32 = 0, RWPT_FP64 = 1 };

/* Normalisation of the co-location weights (Sec. 1.1, after Eq. 3).
 * SYM: P_ij = (w_ij / r_i + w_ij / r_j) / 2 with r_i = sum_j w_ij -- the
 *      symmetric part of the paper's row-normalised P; every pair exchange is
 *      antisymmetric, so species mass is conserved (the conservation
 *      requirement of Sec. 6).  Default.
 * ROW: P_ij = w_ij / r_i exactly as printed; not conservative when
 *      neighbourhoods differ. */
enum { RWPT_NORM_SYM = 0, RWPT_NORM_ROW = 1 };

/* Evaluation path.  SPARSE: cell-list neighbour search + per-pair kernels
 * (any kappa, either precision).  DENSE: every pair of the realisation (the
 * full-matrix "brute force" of Sec. 1.1) as a contraction on matrix cores:
 * weight tiles generated from the positions, split into three bf16 parts and
 * multiplied with the bf16-split mass columns with fp32 accumulation; needs
 * kappa = INFINITY (checked at create), RWPT_FP32 (create), and one
 * realisation of at most 131072 particles (init, else RWPT_EUNSUPPORTED).
 * Pairs whose weight is below 2^-40 are skipped tile-wise.
 * AUTO: DENSE when those conditions hold, else SPARSE. */
enum { RWPT_PATH_AUTO = 0, RWPT_PATH_SPARSE = 1, RWPT_PATH_DENSE = 2 };

typedef struct rwpt_config {
  int32_t dim;            /* 1, 2 or 3 */
  int32_t n_species;      /* S, 1..8 */
  int32_t react_a;        /* species index of A in A + B -> 0, or -1 (no reaction) */
  int32_t react_b;        /* species index of B, or -1 */
  double box_lo[3];       /* reflecting walls; entries beyond dim ignored */
  double box_hi[3];
  double kappa;           /* cutoff in units of sigma; > 0; INFINITY = every pair */
  double rw_ratio;        /* D_rw = rw_ratio * D; 0 = positions never move */
  int32_t precision;      /* RWPT_FP32 or RWPT_FP64 */
  int32_t norm;           /* RWPT_NORM_SYM or RWPT_NORM_ROW */
  int32_t path;           /* RWPT_PATH_* */
  int32_t tile_lanes;     /* lanes sharing one particle in the pair kernels, which then
                             share one candidate list per tile: 1, 4, 8 or 16;
                             -1 = one lane per particle with its own candidate rows
                             (sparse neighbourhoods); -2 = half stencil (binary32):
                             every unordered pair evaluated once and its share
                             delivered to both ends (Sec. 6.1: about half as many
                             operations), deterministic; 0 = choose from dim and N */
  double cell_refine[3];  /* cells per cutoff length along each axis (> 0); 0 = choose */
  int32_t device;         /* HIP device ordinal */
  int32_t use_graph;      /* 1 = replay each rwpt_step as one captured HIP graph */
  uint64_t seed;          /* key of the counter-based random walk */
  void *stream;           /* hipStream_t to queue work on; NULL = a stream the context owns */
  /* Advection and hydrodynamic dispersion of the walk (Eq. 1, Eq. 2): a
   * constant velocity v (entries beyond dim ignored) adds v dt per step, and
   * dispersivities alpha_l >= alpha_t >= 0 add the dispersion tensor
   * alpha_t |v| I + (alpha_l - alpha_t) v v^T / |v| to the isotropic walk
   * share D_rw.  Zero velocity (default) gives the pure-diffusion walk. */
  double velocity[3];
  double alpha_l;
  double alpha_t;
} rwpt_config;

typedef struct rwpt_ctx rwpt_ctx;

/* Fill *cfg with defaults: dim 2, S 2, reaction (0, 1), unit box, kappa 3,
 * rw_ratio 1, FP32, SYM, AUTO path, automatic tiling, device 0, graphs on,
 * seed 0, NULL stream, zero velocity and dispersivities. */
void rwpt_config_default(rwpt_config *cfg);

/* Validate *cfg and create a context.  No device memory is touched until
 * rwpt_init_ensemble.  *out receives NULL on failure except for RWPT_EINVAL
 * where a context holding the error message may be returned (free it with
 * rwpt_destroy); pass out == NULL-safe pointers only. */
rwpt_status rwpt_create(const rwpt_config *cfg, rwpt_ctx **out);

/* Load an ensemble of n_real independent realisations.
 *   n_per_real[r] >= 0 particles each (host array, n_real entries; n_real >= 1);
 *   pos:  host, N x dim row-major, N = sum n_per_real; every coordinate finite
 *         and inside the closed box;
 *   mass: host, S x N species-major, finite;
 *   d_scale: host, n_real multipliers of the D given to rwpt_step (D_r = D *
 *         d_scale[r]), each >= 0 and finite; NULL = all 1.
 * Replaces any previous ensemble and resets the step counter to 0. */
rwpt_status rwpt_init_ensemble(rwpt_ctx *ctx, int32_t n_real, const int64_t *n_per_real,
                               const double *pos, const double *mass, const double *d_scale);

/* As rwpt_init_ensemble, with pos and mass given as device pointers (binary64,
 * the same layouts) on the configured device, e.g. torch tensors; n_per_real
 * and d_scale stay host arrays.  The inputs are copied to the host, validated
 * and loaded exactly as by rwpt_init_ensemble (one PCIe round trip at init; the
 * stepping path never leaves the device).  The caller keeps ownership of its
 * buffers, which are only read.  Errors as rwpt_init_ensemble, plus
 * RWPT_EDEVICE if the copy fails (e.g. a pointer that is not device memory). */
rwpt_status rwpt_init_ensemble_device(rwpt_ctx *ctx, int32_t n_real, const int64_t *n_per_real,
                                      const double *pos_dev, const double *mass_dev,
                                      const double *d_scale);

/* Advance every realisation by n_steps >= 0 explicit steps of length dt > 0
 * with mass-transfer diffusion D >= 0 (D_m of Eq. 3).  D * d_scale[r] = 0
 * leaves realisation r's masses to the reaction only.  Asynchronous. */
rwpt_status rwpt_step(rwpt_ctx *ctx, double dt, double D, int32_t n_steps);

/* Wait for all queued work of the context. */
rwpt_status rwpt_sync(rwpt_ctx *ctx);

/* Copy the current masses (S x N species-major, caller's order) to host memory. */
rwpt_status rwpt_query_masses(rwpt_ctx *ctx, double *mass_out);

/* Copy the current positions (N x dim row-major, caller's order) to host memory. */
rwpt_status rwpt_query_positions(rwpt_ctx *ctx, double *pos_out);

/* FP64 audit of the current state, n_real x (S + 1) doubles:
 * out[r*(S+1) + s] = sum_i M_s of realisation r, out[r*(S+1) + S] =
 * sum_i (M_a - M_b) (0 without a reaction).  After init it reports the loaded
 * values; after a step, the values the device computed at the end of it. */
rwpt_status rwpt_audit(rwpt_ctx *ctx, double *out);

/* Number of steps taken since init. */
rwpt_status rwpt_steps_taken(rwpt_ctx *ctx, int64_t *out);

/* Count, for the current positions and the cutoff of (dt, D), the ordered
 * neighbour pairs j != i within the cutoff (pairs_out, summed over
 * realisations) and the candidate evaluations the sparse kernels perform
 * (evals_out, may be NULL).  With the half-stencil tiling (tile_lanes = -2)
 * both counts come from the one-lane tiles of 64 particles (the same pairs;
 * evals_out is then that enumeration's count, not the half stencil's own,
 * which evaluates each unordered pair once).  Synchronous; does not change
 * the state. */
rwpt_status rwpt_count_pairs(rwpt_ctx *ctx, double dt, double D, int64_t *pairs_out,
                             int64_t *evals_out);

/* Debug export of the neighbour lists for the cutoff of (dt, D) and the
 * current positions, as CSR over the caller's particle order with ascending
 * global column indices, j = i included.  The candidates are enumerated as
 * the step's pair kernels enumerate them for the tiling in use (the chunked
 * candidate rows of the binary32 four-lane tiles, whole or split; each
 * particle's own cutoff box for one lane per particle; the stencil rows of
 * the other tilings), each decided by the same cutoff predicate.  Call with cols == NULL to get the
 * number of entries in *nnz_out; then with rowptr (N + 1 int64) and cols
 * (*nnz_out int32) allocated.  Synchronous; does not change the state. */
rwpt_status rwpt_neighbors(rwpt_ctx *ctx, double dt, double D, int64_t *rowptr, int32_t *cols,
                           int64_t *nnz_out);

/* Debug: the row sums r_i = sum_j w_ij of the normalisation (Sec. 1.1, after
 * Eq. 3) for the current positions and the cutoff of (dt, D), computed by the
 * row-sum kernel of the sparse path in the launch shape a step uses (same
 * tiling, candidate enumeration and cutoff predicate), returned in the
 * caller's particle order (r_out: N doubles, host).  unit_weights = 1 replaces
 * every weight by exp(0) = 1, so r_out[i] is exactly the number of particles
 * j (j = i included) that the step's own kernel takes as neighbours of i.
 * Synchronous; masses, positions and the step counter are unchanged.
 * Errors: RWPT_EINVAL (bad dt, D, unit_weights or NULL r_out), RWPT_ESTATE
 * (before init), RWPT_EUNSUPPORTED (full-matrix path), RWPT_EDEVICE. */
rwpt_status rwpt_debug_rowsums(rwpt_ctx *ctx, double dt, double D, int32_t unit_weights, double *r_out);

/* Per-phase timing.  While enabled, rwpt_step launches eagerly (no graph) and
 * brackets each kernel phase with HIP events on the context's stream.
 * rwpt_profile_read returns, per phase p < n_phases (at most 16), the summed
 * milliseconds ms[p] and launch counts cnt[p] since the last reset, and the
 * phase names through rwpt_profile_phase_name. */
rwpt_status rwpt_profile_enable(rwpt_ctx *ctx, int32_t on);
rwpt_status rwpt_profile_reset(rwpt_ctx *ctx);
rwpt_status rwpt_profile_read(rwpt_ctx *ctx, double *ms, int64_t *cnt, int32_t *n_phases);
const char *rwpt_profile_phase_name(int32_t phase);

/* Summary of the context's state (synchronous).  The pair counts are those
 * of rwpt_count_pairs at the current positions for the (dt, D) of the last
 * rwpt_step; before the first step they are -1 and n_cells is 0.  The phase
 * timings are the rwpt_profile_read totals. */
typedef struct rwpt_stats_t {
  int64_t n_particles;        /* N, all realisations */
  int32_t n_real;
  int32_t tile_lanes;         /* tiling in use (see rwpt_config.tile_lanes); 0 before a step */
  double cell_refine[3];      /* cells per cutoff length in use */
  int64_t n_cells;            /* cells of the grid, all realisations */
  int64_t steps_taken;
  int64_t ordered_pairs;      /* pairs j != i within the cutoff */
  int64_t candidate_evals;    /* candidate evaluations of the sparse kernels */
  int32_t n_phases;           /* entries of phase_ms / phase_launches in use (<= 16) */
  int32_t graph_captures;     /* step graphs captured since rwpt_create (use_graph = 1) */
  double phase_ms[16];        /* per-phase milliseconds since the last profile reset */
  int64_t phase_launches[16];
} rwpt_stats_t;
rwpt_status rwpt_stats(rwpt_ctx *ctx, rwpt_stats_t *out);

/* Attainable instruction rates of this device for the pair kernels (not a
 * step of the method: a measurement).  Runs a register-only kernel at full
 * occupancy (8 waves per SIMD) on the context's device and stream and returns
 * the rate in *per_s (synchronous; the state is not changed):
 *   RWPT_PROBE_FMA       independent binary32 FMAs, lane operations per second;
 *   RWPT_PROBE_EXP       binary32 exp2 (v_exp_f32), lane operations per second;
 *   RWPT_PROBE_ROWSUM    candidate evaluations per second of the row-sum inner
 *                        loop of the row-broadcast tiling (tile_lanes = 4):
 *                        distance, cutoff predicate, weight exp(-s^2/sigma^2)
 *                        of Eq. (3) and the row sum r_i, for the context's dim;
 *   RWPT_PROBE_EXCHANGE  the same for the symmetric exchange inner loop (weight,
 *                        P_ij of the symmetric normalisation and the products
 *                        of Eq. (4) for the context's species count).
 * The row-sum and exchange probes execute the kernels' own per-candidate code
 * on operands held in registers (no loads, no neighbour search), so a kernel's
 * measured evaluation rate over this figure is the fraction of its attainable
 * inner-loop rate.  Errors: RWPT_EINVAL (NULL ctx or per_s, unknown kind),
 * RWPT_EDEVICE / RWPT_ENOMEM from the runtime. */
enum { RWPT_PROBE_FMA = 0, RWPT_PROBE_EXP = 1, RWPT_PROBE_ROWSUM = 2, RWPT_PROBE_EXCHANGE = 3 };
rwpt_status rwpt_probe_rate(rwpt_ctx *ctx, int32_t kind, double *per_s);

/* Current tiling: tile_lanes and the per-axis cell refinement in use. */
rwpt_status rwpt_get_tiling(rwpt_ctx *ctx, int32_t *tile_lanes, double *cell_refine3);

/* Autotune the sparse kernels for (dt, D): time every candidate tiling for
 * trial_steps steps on a snapshot of the current state, keep the fastest and
 * restore the state (masses, positions, step counter).  Results are cached in
 * the file named by the environment variable RWPT_TUNE_CACHE if it is set. */
rwpt_status rwpt_autotune(rwpt_ctx *ctx, double dt, double D, int32_t trial_steps);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * allocation-free form of one rwpt_step on a single realisation: one explicit
 * transfer step (Sec. 1.1, Eqs. 3-6) with the reaction, without the walk, on
 * n particles held in the caller's device arrays, computed by the same
 * kernels as rwpt_step (cell sort, row sums, exchange) with cfg->path taken
 * as SPARSE; cfg->rw_ratio, velocity and dispersivities are ignored.
 *   pos:      device, n x dim row-major, binary32 (RWPT_FP32) or binary64
 *             (RWPT_FP64) as cfg->precision says; positions inside the box
 *             (not checked: the data stay on the device);
 *   mass_in:  device, S x n species-major, same type;
 *   mass_out: device, S x n species-major, same type; may not alias mass_in.
 * Every intermediate lives in a fixed 64 MiB scratch area of the library on
 * the current device (held until the process ends), so the call makes no
 * device allocation and no host-device copy; it queues its kernels on
 * cfg->stream (NULL = the device's default stream) and returns without
 * waiting.  A call whose intermediates exceed the area (about 110 bytes per
 * particle in 2-D binary32 with two species, about 340 in 3-D binary64 with
 * eight species, cell counters included: some 6 * 10^5 and 2 * 10^5
 * particles) or whose cutoff
 * spans more than 64 stencil rows returns RWPT_EUNSUPPORTED before queuing
 * anything.  Every call on one device shares that device's area and leaves
 * its contents behind: calls that overlap on one device (other streams or
 * host threads) race and must be serialised by the caller.  The first call on
 * a device looks up the area's address; make it outside graph capture.
 * Errors (message in rwpt_last_error(NULL)): RWPT_EINVAL (bad configuration,
 * n, dt, D or pointers), RWPT_EUNSUPPORTED (dense path, size or stencil
 * beyond the limits), RWPT_EDEVICE (no device, a launch failed). */
rwpt_status rwpt_transfer_noalloc(const rwpt_config *cfg, int32_t n, const void *pos, const void *mass_in,
                                  void *mass_out, double dt, double D);

/* Message of the last failed call on this context ("" if none).  Valid until
 * the next call on the context. */
const char *rwpt_last_error(const rwpt_ctx *ctx);

/* Library version string. */
const char *rwpt_version(void);

/* Release all resources.  NULL is allowed. */
void rwpt_destroy(rwpt_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* RWPT_H */
