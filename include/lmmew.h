/*
 * lmmew: list-mode multi-energy-window OSEM SPECT on one MI355X (gfx950).
 *
 * Method: Rahman, Li, Yu, Laforest, Thorek, Jha, "A list-mode multi-energy
 * window low-count SPECT reconstruction method for isotopes with multiple
 * emission peaks", arXiv 2305.17111.
 *
 * The library evaluates, for every detected photon (detector bin, angle,
 * measured energy), the path mixture of Eq. (3): the unscattered path from
 * each object pixel plus every once-scattered path through a grid of scatter
 * points, each weighted by attenuation (Eq. (6)), the depth-dependent
 * collimator-detector response, the planar Klein-Nishina density and the
 * Gaussian energy resolution evaluated at the photon's true energy.  Those
 * per-event densities a_jq drive the list-mode forward projection
 * p_j = sum_q a_jq lambda_q, the backprojection, the ordered-subsets EM
 * update of Eq. (18)-(20) and the sensitivity image (denominator of
 * Eq. (18), Eq. (7) per pixel).
 *
 * Conventions shared by every entry point
 *   - Image arrays are float32 over the full n x n grid, row-major,
 *     q = iy*n + ix, pixel centre ((ix+1/2)pix - R, (iy+1/2)pix - R),
 *     R = n*pix/2.  Pixels outside the support (centre outside the circular
 *     field of view of radius R, or cleared in the caller's mask) hold 0 in
 *     every output and are never updated.
 *   - Angle a points the detector normal along (cos t, sin t), t = 2 pi a /
 *     n_angles (exact at multiples of 90 degrees); bin b covers the lateral
 *     coordinate u = -x sin t + y cos t in [-R + b*db, -R + (b+1)*db),
 *     db = 2R / n_bins; the detector plane is x.n = R.
 *   - The 3-D model (nz > 0 in lmmew_system): the grid stacks nz slices of
 *     n x n voxels of side pixel_mm; voxel (ix, iy, iz) has flat index
 *     q = (iz*n + iy)*n + ix and centre z = (iz+1/2)pix - Zh, Zh = nz*pix/2;
 *     every "n*n" below then reads n*n*nz.  The camera rotates about z: bin
 *     b is as above and axial bin bz covers z in [-Zh + bz*dbz,
 *     -Zh + (bz+1)*dbz), dbz = 2 Zh / n_bins_z.  The support is the
 *     cylinder of radius R (and the caller's mask).
 *   - Subset s of an n_subsets partition holds the angles a with
 *     a mod n_subsets == s; subsets are visited in order 0..n_subsets-1.
 *   - Every pointer argument documented as "device" is memory the caller
 *     allocated on the current HIP device and keeps ownership of.  The
 *     library owns only what it allocates behind a context or plan handle.
 *   - Work is enqueued on the caller's stream.  Calls that synchronise that
 *     stream say so.  A context (and its plans) must be used by one host
 *     thread at a time.
 *   - Every function returns an lmmew status code; on failure the context's
 *     last error text says why (lmmew_last_error).  No exception, abort or
 *     exit crosses this interface.
 */
#ifndef LMMEW_H
#define LMMEW_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LMMEW_OK         0
#define LMMEW_EINVAL    -1   /* NULL pointer, bad size, event out of range, non-finite input */
#define LMMEW_ENOMEM    -2   /* device or host allocation failed */
#define LMMEW_EDEVICE   -3   /* a HIP runtime call failed */
#define LMMEW_ENUMERIC  -4   /* a non-finite value appeared in a result */

#define LMMEW_MAX_LINES   8
#define LMMEW_MAX_WINDOWS 8

/* System parameters (the sysParam and T inputs of Algorithm 1). */
typedef struct lmmew_system {
    int32_t n;                 /* pixels per side of the square grid */
    int32_t ns;                /* scatter points per side; n/ns must be an even integer */
    int32_t n_bins;            /* detector bins across the field of view */
    int32_t n_angles;          /* angles evenly spaced over 360 degrees */
    int32_t n_lines;           /* emission lines, 1..LMMEW_MAX_LINES */
    int32_t n_windows;         /* energy windows, 1..LMMEW_MAX_WINDOWS */
    double pixel_mm;           /* pixel size */
    double psf_fwhm0_mm;       /* collimator-detector FWHM at depth 0 */
    double psf_fwhm_slope;     /* FWHM growth per mm of depth below the detector plane */
    double coll_dtheta;        /* collimator angular acceptance, radians */
    double line_keV[LMMEW_MAX_LINES];    /* emission energies E_w */
    double line_yield[LMMEW_MAX_LINES];  /* photons per decay alpha_w (Sec. 2.1) */
    double win_lo_keV[LMMEW_MAX_WINDOWS];
    double win_hi_keV[LMMEW_MAX_WINDOWS];
    double eres_frac;          /* energy FWHM as a fraction of eres_ref_keV at that energy */
    double eres_ref_keV;       /* absolute FWHM scales as sqrt(E) (Sec. 3.1.2) */
    double mu_ref_keV;         /* energy at which the attenuation map is given */
    double mu_power;           /* mu(E) = mu(mu_ref) * (E / mu_ref)^(-mu_power) */
    double T;                  /* acquisition time (Eq. (2)) */
    double electron_keV;       /* electron rest energy used by Klein-Nishina */
    /* 3-D single-scatter model (the extension the paper names as its next
     * step, Sec. 5 and the appendix on 3-D computational requirements): Eq.
     * (5) with emission into the solid angle coll_solid_angle / (4 pi), the
     * scattered photon's direction drawn from the Klein-Nishina density per
     * steradian, scatter points on an ns x ns x ns_z grid, and a
     * depth-dependent Gaussian response separable in u and z.  nz = 0 keeps
     * the planar model of the paper's evaluation (coll_dtheta), and then the
     * three fields below are ignored. */
    int32_t nz;                /* slices; 0: planar model */
    int32_t ns_z;              /* scatter points along z; nz/ns_z must be an even integer */
    int32_t n_bins_z;          /* axial detector bins, 1..32767 */
    double coll_solid_angle;   /* collimator acceptance solid angle, sr */
} lmmew_system;

/* List-mode data (lmData of Algorithm 1): one entry per detected photon.
 * All arrays are device arrays of n entries.  The position attribute of
 * Eq. (3) is either a detector bin (position_mm == NULL: the collimator
 * response is the probability of the bin) or, when position_mm is not NULL,
 * a continuous lateral position on the detector in mm (bin is then ignored
 * and may be NULL; the collimator response is the Gaussian density per mm at
 * that position, 0 beyond 7 standard deviations).  The sensitivity is the
 * same for both, since the density integrates over the detector to the same
 * probability.  An event is valid when 0 <= angle < n_angles, energy_keV is
 * finite and lies in some window [lo, hi], and 0 <= bin < n_bins, or
 * -R <= position_mm < R with R = n * pixel_mm / 2. */
typedef struct lmmew_events {
    int64_t n;
    const int16_t *bin;
    const int16_t *angle;
    const float *energy_keV;
    const float *position_mm;
    const int16_t *bin_z;      /* 3-D model: axial bins (required, 0 <= bin_z < n_bins_z;
                                  continuous positions are not supported there); planar:
                                  ignored */
} lmmew_events;

/* Optional statistics of an OSEM call (host memory owned by the caller). */
typedef struct lmmew_stats {
    int64_t skipped_total;   /* out: events with p_j = 0 over all sub-iterations */
    int64_t *skipped;        /* in: NULL or host [n_iters*n_subsets]; out: per sub-iteration */
    double *subset_loglik;   /* in: NULL or host [n_iters*n_subsets]; out: sum over the
                                subset's events of log p_j minus sum_q sens_s[q] lambda_q,
                                before the update, summed over cases; with one subset
                                this is Eq. (8) up to a constant */
} lmmew_stats;

typedef struct lmmew_ctx lmmew_ctx;
typedef struct lmmew_plan lmmew_plan;
typedef struct lmmew_mlp lmmew_mlp;

/* Text for a status code. */
const char *lmmew_status_string(int status);

/* Text of the last failure on this context ("" if none). */
const char *lmmew_last_error(const lmmew_ctx *ctx);

/* Builds a context for one attenuation map: the attenuation line integrals
 * of Eq. (6) from every support pixel to every scatter point and to the
 * detector plane at every angle, and from every scatter point to the
 * detector plane (the precomputation of Algorithm 1).
 *   sys      host; copied.
 *   mu85     device [n*n] float, attenuation at mu_ref_keV in 1/mm, >= 0.
 *   support  device [n*n] uint8 or NULL: pixels allowed to carry activity
 *            (intersected with the circular field of view).
 *   stream   the tables are built on this stream; the call synchronises it
 *            once to read mu85 and support.
 *   out      receives the context; NULL on failure.
 * Errors: EINVAL (bad parameters, NULL pointers, negative or non-finite
 * mu85), ENOMEM, EDEVICE. */
int lmmew_create(const lmmew_system *sys, const float *mu85, const uint8_t *support,
                 hipStream_t stream, lmmew_ctx **out);

/* Releases the context and everything it owns.  Takes no stream: it waits
 * for all work on the device (as freeing device memory does) before
 * releasing anything. */
int lmmew_destroy(lmmew_ctx *ctx);

/* Number of support pixels (the pixels rows and labels cover), -1 for NULL. */
int64_t lmmew_support_size(const lmmew_ctx *ctx);

/* Path-parameter table (optional): the event-independent part of every
 * once-scattered path of Eq. (3) -- for each (angle, scatter point, line,
 * support pixel): the log2 path weight (attenuation along both legs,
 * Klein-Nishina, geometry, energy-Gaussian normalisation) and
 * s_w = sqrt(log2(e) / (2 k E')) of the scattered energy E' (sigma'^2 = k E'),
 * from which the kernel forms the energy factor exp2(-(s_w E - F_w)^2) with
 * F_w = s_w E' = log2(e) / (2 k s_w) --
 * evaluated once into device memory owned by the context: n_angles x scatter
 * points x lines x padded support pixels x 8 bytes (lmmew_path_table_bytes;
 * 4.8 GB for the 64x64 workload's 508 scatter points and 3 lines).  With it the per-event kernel reads these values
 * instead of recomputing them for every tile of events; the rows are still
 * evaluated per event in every sub-iteration, and agree with the rows without
 * the table to rounding.  enable == 0 frees it.  Plans over several maps use
 * the tables only when every case's context has one.  Synchronises.
 * Errors: EINVAL, ENOMEM (also when the table would leave less than 1 GiB of
 * device memory free), EDEVICE. */
int lmmew_path_table(lmmew_ctx *ctx, int enable, hipStream_t stream);
int64_t lmmew_path_table_bytes(const lmmew_ctx *ctx);

/* Unscattered bin-probability table (planar systems): the probability that
 * the unscattered path from every support pixel lands in every detector bin
 * at every angle (the position factor of Eq. (3) for n = 0), n_angles x
 * n_bins x padded support pixels x 4 bytes, owned by the context.  It is
 * built automatically on the context's first plan when it fits in 2 GiB and
 * the allocation succeeds; otherwise, and after enable == 0, the per-event
 * kernel forms each probability from two complementary error functions.
 * Rows agree to rounding either way.  Synchronises the stream.  Returns 1
 * when the table is in use after the call, 0 when not, or an error status
 * (EINVAL, EDEVICE). */
int lmmew_psf_table(lmmew_ctx *ctx, int enable, hipStream_t stream);

/* Sensitivity image per subset: sens[s][q] = T * sum over the subset's
 * angles of the probability that a decay in pixel q is recorded (on the
 * detector and inside a window), unscattered or once scattered: the
 * denominator of Eq. (18) with the window acceptance of every path.
 *   sens     device [n_subsets][n*n] float, written.
 * Errors: EINVAL (n_subsets < 1 or > n_angles, NULL), EDEVICE. */
int lmmew_sensitivity(lmmew_ctx *ctx, int n_subsets, float *sens, hipStream_t stream);

/* List-mode forward projection: p[j] = sum_q a_jq lambda[q] (the
 * denominator of Eq. (19)) for arbitrary events in any order.
 *   ev       events (device arrays); validated.
 *   lambda   device [n*n] float.
 *   p        device [ev->n] float, written in input order.
 * Synchronises the stream once to validate and sort the events.
 * Errors: EINVAL (invalid event: the message names its index), ENOMEM,
 * EDEVICE. */
int lmmew_forward(lmmew_ctx *ctx, const lmmew_events *ev, const float *lambda, float *p,
                  hipStream_t stream);

/* Adjoint of lmmew_forward: out[q] = sum_j a_jq w[j] (events with w[j] = 0
 * contribute nothing).  With w[j] = 1 / p_j over a subset's events,
 * lambda[q] * out[q] is Algorithm 1's sumZbar[q]: the sum over the events of
 * the expected path counts z-bar of Eq. (19), the numerator of Eq. (18).
 *   w        device [ev->n] float, input order.
 *   out      device [n*n] float, written.
 * Synchronises the stream once.  Errors as lmmew_forward. */
int lmmew_backproject(lmmew_ctx *ctx, const lmmew_events *ev, const float *w, float *out,
                      hipStream_t stream);

/* Prepares list-mode data for OSEM: validates every event, sorts each
 * subset's events by (case, angle, line mask, bin or position, energy)
 * (stable; in the 3-D model by (case, angle, line mask, square block of the
 * detector, bin_z, bin, energy); the line mask is defined at
 * lmmew_plan_terms) and lays out the work tiles, the collimator-response factor of every (listed scatter point,
 * event) pair of each tile (event-tile floats per listed point: 35 MB for 50k
 * events at 64x64) and the per-subset scratch.  A plan holds one or more
 * independent cases (noise realisations or patients) that share the context's
 * attenuation map and sensitivity.
 *   ev            events of all cases, concatenated (device arrays).
 *   case_offsets  host int64 [n_cases+1] or NULL (one case): events of case
 *                 c are [case_offsets[c], case_offsets[c+1]).
 *   n_subsets     angle subsets, 1..n_angles.
 * The plan copies what it needs; the event arrays may be freed afterwards.
 * Synchronises the stream once.  Errors: EINVAL, ENOMEM, EDEVICE. */
int lmmew_plan_create(lmmew_ctx *ctx, const lmmew_events *ev, const int64_t *case_offsets,
                      int n_cases, int n_subsets, hipStream_t stream, lmmew_plan **out);

/* A plan whose cases have their own attenuation maps (patients): case c is
 * modelled with the tables of ctxs[c] (n_cases contexts that share the system
 * parameters and the support; they may differ in the map and hence in their
 * scatter points).  The plan belongs to ctxs[0]: pass ctxs[0] to the OSEM
 * calls, whose sens argument is then device [n_cases][n_subsets][n*n], case
 * c's block from lmmew_sensitivity(ctxs[c]).  Scatter model: with no network
 * selected on ctxs[0] every case uses the exact model (a network selected on
 * another case's context is then an error, EINVAL at the OSEM call); with one
 * selected, case c uses the network selected on ctxs[c], or ctxs[0]'s when
 * ctxs[c] has none (lmmew_set_scatter_model), so that each patient may carry
 * a network fitted to its own map.  The contexts must outlive the plan.  Otherwise
 * as lmmew_plan_create.  Errors: EINVAL (also for contexts with a different
 * system or support), ENOMEM, EDEVICE. */
int lmmew_plan_create_maps(lmmew_ctx *const *ctxs, const lmmew_events *ev,
                           const int64_t *case_offsets, int n_cases, int n_subsets,
                           hipStream_t stream, lmmew_plan **out);

/* Releases the plan (waits for all work on the device first, as
 * lmmew_destroy). */
int lmmew_plan_destroy(lmmew_plan *plan);

/* Cached-row mode (a mode of its own, outside the paper's matrix-free
 * iteration): with enable != 0 the rows a_jq of every subset are computed
 * once, with the context's current scatter model, into device memory owned by
 * the plan (n_events x support pixels padded to 64 x 4 bytes: 0.7 GB for 50k
 * events at 64x64); lmmew_osem_iter/_subiter/_graph then read them instead
 * of evaluating the model, which makes an iteration bound by HBM bandwidth.
 * Results are bitwise identical to the matrix-free iterations.  enable == 0
 * frees them.  After lmmew_set_scatter_model the cached rows are stale and the
 * OSEM calls fail with EINVAL until they are cached again.  Synchronises.
 * Errors: EINVAL, ENOMEM (also when the rows would leave less than 1 GiB of
 * device memory free), EDEVICE. */
int lmmew_plan_cache_rows(lmmew_ctx *ctx, lmmew_plan *plan, int enable, hipStream_t stream);

/* Runs n_iters iterations of list-mode OSEM (Eq. (18)-(20)): for every
 * subset s in order and every case c,
 *   p_j = sum_q a_jq lambda_c[q]                  (events j of case c in s)
 *   B_q = sum_{j, p_j > 0} a_jq / p_j
 *   lambda_c[q] <- lambda_c[q] * B_q / sens[s][q]  where sens[s][q] > 0.
 * The system model is evaluated afresh in every sub-iteration.
 *   sens     device [n_subsets][n*n] from lmmew_sensitivity (same n_subsets);
 *            [n_cases][n_subsets][n*n] for a plan from lmmew_plan_create_maps.
 *   lambda   device [n_cases][n*n], in: the current image, out: the image
 *            after n_iters iterations.  Initial values must be >= 0.
 *   stats    NULL, or host statistics; requesting them synchronises the
 *            stream at the end of the call.
 * Without stats the call only enqueues work.  Errors: EINVAL, EDEVICE,
 * ENUMERIC (a non-finite image value, reported only when stats are
 * requested). */
int lmmew_osem_iter(lmmew_ctx *ctx, lmmew_plan *plan, int n_iters, const float *sens,
                    float *lambda, lmmew_stats *stats, hipStream_t stream);

/* One sub-iteration of Eq. (18)-(20) for subset `subset` (0..n_subsets-1):
 * the same update as lmmew_osem_iter restricted to that subset.  Calling it
 * for subsets 0..n_subsets-1 in order is exactly one iteration, so a run can
 * stop after any sub-iteration and resume from (lambda, iteration, subset)
 * with a bitwise-identical result.  stats (optional) then holds one entry. */
int lmmew_osem_subiter(lmmew_ctx *ctx, lmmew_plan *plan, int subset, const float *sens,
                       float *lambda, lmmew_stats *stats, hipStream_t stream);

/* The same n_iters iterations as lmmew_osem_iter (no statistics), issued as
 * ONE hipGraph launch: on the first call (and whenever n_iters, sens, lambda
 * or the event tile differ from the previous call) the library captures the
 * whole launch sequence of every sub-iteration of every case into a graph
 * owned by the plan, then replays it.  The captured graph contains kernel
 * launches only.  Results are bitwise identical to lmmew_osem_iter.  The
 * arrays behind sens and lambda must stay allocated while the plan may
 * replay the graph.  Errors: EINVAL, EDEVICE. */
int lmmew_osem_graph(lmmew_ctx *ctx, lmmew_plan *plan, int n_iters, const float *sens,
                     float *lambda, hipStream_t stream);

/* Autotuner: times the per-event system-model kernel alone (it writes only
 * the plan's scratch) on the plan's largest subset at each event tile size
 * (16, 32, 64) with HIP events, keeps the fastest and returns it in *chosen.
 * With use_cache, a plan whose problem shape (support pixels, scatter
 * points, lines, angles, subsets, events per case and angle to a power of
 * two) was tuned before in this process reuses that choice without timing.
 * Synchronises the stream.  Errors: EINVAL, EDEVICE. */
int lmmew_autotune(lmmew_ctx *ctx, lmmew_plan *plan, int use_cache, hipStream_t stream,
                   int *chosen);

/* Tuning knobs of the per-event system-model kernel for a plan (chosen by
 * lmmew_autotune or set by hand).  event_tile: events per work tile, one of
 * 16, 32, 64.  Changing it rebuilds the plan's tiles (synchronises). */
int lmmew_plan_set_event_tile(lmmew_ctx *ctx, lmmew_plan *plan, int event_tile,
                              hipStream_t stream);
int lmmew_plan_get_event_tile(const lmmew_plan *plan);

/* Timing of the per-event system-model kernel (and of the scatter
 * surrogate's kernel when a network is selected): with profiling enabled,
 * every launch of those kernels made for this plan by lmmew_osem_iter or
 * lmmew_osem_subiter is bracketed by two HIP events recorded on the caller's
 * stream.  lmmew_plan_profile_read waits for the recorded launches, returns
 * the per-event kernel's summed duration (ms) and launch count, and starts a
 * new measurement; lmmew_plan_profile_read_kernels does the same for both
 * kernels: ms[0], launches[0] the per-event kernel, ms[1], launches[1] the
 * surrogate (host arrays of 2). */
int lmmew_plan_profile(lmmew_ctx *ctx, lmmew_plan *plan, int enable);
int lmmew_plan_profile_read(lmmew_ctx *ctx, lmmew_plan *plan, double *row_ms, int64_t *launches);
int lmmew_plan_profile_read_kernels(lmmew_ctx *ctx, lmmew_plan *plan, double *ms,
                                    int64_t *launches);

/* Number of algorithmic terms one OSEM iteration of the plan evaluates in
 * the per-event system-model kernel: for every (event, support pixel) pair,
 * one term per line for the unscattered path and one per (line, scatter
 * point) that is not dropped.  Two cuts drop terms whose value is negligible:
 * a scatter point whose Gaussian response puts the event's bin beyond 7
 * standard deviations (below 1.3e-12 of its peak), and a line whose
 * scattered photon cannot reach an energy near the event's: a line's
 * scattered energy lies between E_w / (1 + 2 E_w / electron_keV) and E_w,
 * and when the largest value of the energy-resolution Gaussian at the
 * event's energy over that range is below 2^-40 of the largest such value
 * over all lines, the event keeps only the line's unscattered term (the line
 * with the largest value is always kept; systems of up to three lines, with
 * more every line is kept).  The lines an event keeps form its line mask.
 *   out_terms      host: terms evaluated per iteration.
 *   out_full_terms host: terms of the unpruned model per iteration. */
int lmmew_plan_terms(const lmmew_plan *plan, double *out_terms, double *out_full_terms);

/* The line mask of an event of measured energy energy_keV under system sys
 * (host only, no device work): bit w is set when the event keeps line w's
 * scattered terms (see lmmew_plan_terms).  Returns the mask (>= 0), or
 * LMMEW_EINVAL for a NULL system, a line count outside 1..8 or a
 * non-finite energy. */
int lmmew_line_mask(const lmmew_system *sys, float energy_keV);

/* Measured issue rate of the per-event kernel's instruction chains on the
 * current device (the ceiling its roofline is reported against):
 *   kind 0: algorithmic terms per second -- one energy-Gaussian factor of a
 *           (line, path) pair of Eq. (3) at an event's energy, accumulated
 *           with the event's collimator-response factor: two FMAs, one
 *           exp2, one FMA, with the path parameters per lane and the event's
 *           energy and factor uniform over the wavefront;
 *   kind 1: FP32 fused multiply-adds per second (lane operations);
 *   kind 2: exp2 evaluations per second (lane operations).
 * 16 independent chains per lane, 8 waves per SIMD, 5 timed launches after
 * one warm-up.  Allocates and frees a small buffer; synchronises the stream.
 * Errors: EINVAL (kind outside 0..2, NULL rate), ENOMEM, EDEVICE. */
int lmmew_calibrate(int kind, hipStream_t stream, double *rate);

/* ---------------------------------------------------------------------------
 * Per-event rows
 * ------------------------------------------------------------------------- */

/* Full system rows for arbitrary events: rows[j][q] = a_jq over the n*n grid
 * (zero off the support), in input order.
 *   part  0: the context's scatter model (exact, or the surrogate when one
 *            is set with lmmew_set_scatter_model) plus the unscattered paths;
 *         1: exact once-scattered paths only; 2: unscattered paths only;
 *         3: exact model (ignores a surrogate).
 *   rows  device [ev->n][n*n] float, written.
 * Synchronises the stream.  Errors: EINVAL, ENOMEM, EDEVICE. */
int lmmew_rows(lmmew_ctx *ctx, const lmmew_events *ev, int part, float *rows, hipStream_t stream);

/* Rows of chosen events from one sub-iteration's system-model launch of a
 * plan: the launch lmmew_osem_iter makes for subset `subset` (the plan's
 * tiles, event tile, path table and the context's scatter model), written to
 * the plan's scratch, then rows[k][q] = a_jq of input event events[k]
 * (Eq. (3)) over the n*n grid (zero off the support).  For parity tests of
 * the rows at full size, in the configuration the OSEM iterations use.
 *   events  host int64 [n]: input indices (as given to lmmew_plan_create) of
 *           events of that subset.
 *   rows    device [n][n*n] float, written.
 * Synchronises the stream.  Errors: EINVAL (an event outside the subset or
 * out of range), ENOMEM, EDEVICE. */
int lmmew_plan_rows(lmmew_ctx *ctx, lmmew_plan *plan, int subset, const int64_t *events,
                    int64_t n, float *rows, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Scatter surrogate (an extension beyond the paper)
 *
 * A network that replaces the once-scattered part of a_jq (the sum over lines
 * and scatter points in Eq. (3)) for the context's attenuation map, while the
 * unscattered part stays exact.  Inputs of an (event, pixel) pair, in the
 * detector frame of the event's angle: (bin centre - pixel's lateral
 * projection)/R, pixel depth below the detector plane/R, pixel's lateral
 * projection/R, cos(angle), sin(angle), (E - 180 keV)/120 keV.
 * Architecture: 6 -> 128 -> 128 -> 128 -> 1, tanh-form GELU after each hidden
 * layer.  Training (lmmew_mlp_grad/_train/_fit): the 128x128 layers as BF16
 * MFMA with FP32 accumulation, the first and last layers in FP32, FP32 master
 * weights.  Inference inside OSEM: the first layer as BF16 MFMA with
 * high/low splitting (about FP32 accuracy), the 128x128 layers as FP16 MFMA
 * with FP32 accumulation and FP16 activations (its densities are closer to
 * the FP64 network than lmmew_mlp_forward's BF16 ones).  The output y is the
 * shifted logarithm of the density: density = max(exp(y + c0) - floor, 0).
 * Parameters (FP32 master copy, 34049 floats, in this order):
 *   W1[6][128] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] w4[128] b4[1],
 * W[i][o] mapping input unit i to output unit o.
 * ------------------------------------------------------------------------- */
#define LMMEW_MLP_PARAMS 34049

/* Creates a network for the context with Glorot-uniform weights (zero biases)
 * drawn from a counter-based generator seeded with seed.  Synchronises.
 * The surrogate models the planar system: EINVAL for a 3-D context (as for
 * lmmew_scatter_labels). */
int lmmew_mlp_create(lmmew_ctx *ctx, uint64_t seed, lmmew_mlp **out);
/* Releases the network (waits for all work on the device first).  Its
 * context may have been destroyed before it: lmmew_destroy detaches the
 * context's networks, which then only accept lmmew_mlp_destroy. */
int lmmew_mlp_destroy(lmmew_mlp *mlp);

/* Host copies of the FP32 parameters (NULL to skip) and the output shift c0
 * and floor.  set also resets the Adam state. */
int lmmew_mlp_get_params(const lmmew_mlp *mlp, float *params, double *c0, double *floor_);
int lmmew_mlp_set_params(lmmew_mlp *mlp, const float *params, double c0, double floor_);

/* Raw network output y for n feature rows.  feats: device [n][6] float;
 * y: device [n] float.  Synchronises. */
int lmmew_mlp_forward(lmmew_ctx *ctx, lmmew_mlp *mlp, const float *feats, int64_t n, float *y,
                      hipStream_t stream);

/* Gradient of the mean squared error (1/n) sum (y - target)^2 with respect to
 * the parameters, for one batch of n rows (n a multiple of 16, <= 2^24).
 *   grad: device [LMMEW_MLP_PARAMS] float; loss: host, may be NULL.
 * Synchronises. */
int lmmew_mlp_grad(lmmew_ctx *ctx, lmmew_mlp *mlp, const float *feats, const float *target,
                   int64_t n, float *grad, double *loss, hipStream_t stream);

/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error over
 * epochs passes of the n rows, shuffled each epoch (seeded), in batches of
 * `batch` rows (a multiple of 16; a trailing partial batch is dropped); the
 * step size decays from lr to lr/10 along a half cosine over the run.
 * epoch_loss: host [epochs] or NULL (mean loss of each epoch). */
int lmmew_mlp_train(lmmew_ctx *ctx, lmmew_mlp *mlp, const float *feats, const float *target,
                    int64_t n, int batch, int epochs, double lr, uint64_t seed,
                    double *epoch_loss, hipStream_t stream);

/* Training samples from the exact model: n_events events with bin and angle
 * uniform and energy uniform over the union of the windows (seeded), each
 * paired with every support pixel (Qm pixels): n_events*Qm samples in the
 * library's row order.  feats: device [n_events*Qm][6]; raw: device
 * [n_events*Qm], the exact once-scattered density. */
int lmmew_scatter_labels(lmmew_ctx *ctx, int64_t n_events, uint64_t seed, float *feats,
                         float *raw, hipStream_t stream);

/* Fits the network to given labels: floor = floor_frac x mean of raw, c0 =
 * mean of log(raw + floor), targets log(raw + floor) - c0, then
 * lmmew_mlp_train (seeded with seed).  floor_frac == 0 keeps the network's
 * current floor and c0 (fine-tuning a fitted network, e.g. one whose
 * parameters were copied with lmmew_mlp_set_params, on labels of another
 * map); EINVAL if it has none.  feats, raw: device, n rows, as written
 * by lmmew_scatter_labels of this or any context with the same system (so a
 * network can be trained on labels of several attenuation maps; the batch
 * shuffle mixes them).  Synchronises.  Errors: EINVAL, ENOMEM, EDEVICE. */
int lmmew_mlp_fit_labels(lmmew_ctx *ctx, lmmew_mlp *mlp, const float *feats, const float *raw,
                         int64_t n, int epochs, int batch, double lr, double floor_frac,
                         uint64_t seed, double *epoch_loss, hipStream_t stream);

/* lmmew_scatter_labels on this context's map for n_label_events events, then
 * lmmew_mlp_fit_labels. */
int lmmew_mlp_fit(lmmew_ctx *ctx, lmmew_mlp *mlp, int64_t n_label_events, int epochs, int batch,
                  double lr, double floor_frac, uint64_t seed, double *epoch_loss,
                  hipStream_t stream);

/* Factor on the scatter network's density for this context's cases
 * (default 1), the same for every energy window: in a plan over several maps
 * case c takes ctxs[c]'s factors, otherwise every case takes the plan
 * context's.  It calibrates a network with no attenuation-map input to one
 * patient's map (lmmew_scatter_scale_fit).
 * Errors: EINVAL (scale not positive and finite). */
int lmmew_set_scatter_scale(lmmew_ctx *ctx, double scale);

/* As lmmew_set_scatter_scale with one factor per energy window: an event's
 * density takes the factor of the first window (in the system's order) that
 * holds its energy.  scales: host array of n_windows factors, n_windows the
 * system's window count.  Errors: EINVAL (NULL, another count, a factor not
 * positive and finite). */
int lmmew_set_scatter_scale_windows(lmmew_ctx *ctx, const double *scales, int n_windows);

/* The factor that matches the network's total once-scattered density to the
 * exact model's over the given events on this context's map: *scale =
 * sum_j sum_q exact scattered a_jq / sum_j sum_q network density_jq (sums over
 * every support pixel, FP64), for example over a sample of one patient's own
 * recorded events.  mlp: a network of this context or of one with the same
 * system and support (it need not be selected).  Synchronises the stream.  Errors: EINVAL (no events,
 * continuous positions, NULL), ENUMERIC (a sum vanishes), ENOMEM, EDEVICE. */
int lmmew_scatter_scale_fit(lmmew_ctx *ctx, lmmew_mlp *mlp, const lmmew_events *ev,
                            double *scale, hipStream_t stream);

/* The factors of lmmew_scatter_scale_fit for each energy window: scales[w] =
 * the exact model's once-scattered density summed over the rows of the given
 * events whose energy lies in window w (the first that holds it) / the
 * network's over the same rows (FP64, every support pixel).  A window whose
 * events are absent, or whose sums vanish, takes the factor over all the
 * events.  scales: host array of n_windows, the system's window count.
 * Synchronises the stream.  Errors: as lmmew_scatter_scale_fit, and EINVAL
 * for another count. */
int lmmew_scatter_scale_fit_windows(lmmew_ctx *ctx, lmmew_mlp *mlp, const lmmew_events *ev,
                                    double *scales, int n_windows, hipStream_t stream);

/* Selects the scatter model that lmmew_osem_iter/_subiter/_graph,
 * lmmew_forward and lmmew_backproject use for this context: NULL for the
 * exact model, or a network of this context (kept by pointer: it must stay
 * alive while selected).  The network models binned events: a call on
 * events with continuous positions while a network is selected fails with
 * EINVAL. */
int lmmew_set_scatter_model(lmmew_ctx *ctx, lmmew_mlp *mlp);

/* Where OSEM, lmmew_forward, lmmew_backproject, lmmew_rows and the scale
 * fits evaluate this network (an extension of the surrogate; the appendix on
 * the computational requirements in 3-D, to which the Discussion (Sec. 5)
 * refers, names modelling scatter at a lower resolution as a way to cut the
 * cost, and the network's density varies slowly over a pixel).  grid = 1
 * (the default): at every support pixel.  grid = g in 2..8: at nodes placed on the centres of the pixels (g u, g v) for
 * every node any support pixel needs; a support pixel (ix, iy) takes the
 * bilinear interpolation of the four nodes around it, (ix / g, iy / g) and
 * the next ones in x and y (integer division), with weights from
 * fx = (ix mod g) / g and fy = (iy mod g) / g.  The density factors
 * (lmmew_set_scatter_scale*) apply to the node values.  About 1/g^2 of the
 * network evaluations; rows change by the interpolation error only.  Plans
 * using the network keep a node-value scratch of their largest subset's rows
 * times the node count (about Qm / g^2 floats per row), allocated on first
 * use.  Synchronises the device (the old node tables may still be read).
 * Errors: EINVAL (NULL, a network whose context was destroyed, grid outside
 * 1..8), EDEVICE/ENOMEM. */
int lmmew_mlp_set_grid(lmmew_mlp *mlp, int grid);

/* Number of positions at which the network is evaluated per event row: the
 * node count with a coarse grid, else the support size.  EINVAL for NULL. */
int lmmew_mlp_grid_nodes(const lmmew_mlp *mlp);

/* Scatter at a coarser pixel resolution for the exact model (the appendix on
 * the computational requirements in 3-D, to which the Discussion (Sec. 5)
 * refers, names modelling scatter at a lower resolution as a way to cut the
 * cost of the once-scattered term of Eq. (5)).  grid = 1 (the default): the scattered part of every row a_jq (Eq. (3)-(5))
 * at every support pixel.  grid = g in 2..8 (planar model): the scattered
 * part is evaluated only at node pixels and interpolated; the unscattered
 * part stays at every support pixel, and the sensitivity is unchanged.
 * Support pixel (ix, iy) takes the bilinear combination of the pixels
 * (g u0, g v0), (g u0 + g, g v0), (g u0, g v0 + g), (g u0 + g, g v0 + g),
 * u0 = ix / g, v0 = iy / g (integer division), with weights from
 * fx = (ix mod g) / g and fy = (iy mod g) / g; corners outside the support
 * or the grid are dropped and the remaining weights renormalised (a pixel
 * with no corner in the support keeps its own value).  A node pixel's value
 * is the one the full-resolution model gives it.  Applies to every row the
 * context's exact model produces: OSEM, lmmew_forward, lmmew_backproject,
 * lmmew_rows (parts 0, 1, 3), the surrogate's labels and scale fits.  In a
 * plan over several maps every context needs the same grid.  Plans keep a
 * node-value scratch of their largest subset's rows times the node count.
 * Synchronises the device (the old node tables may still be read) and the
 * stream.  Errors: EINVAL (NULL, grid outside 1..8, grid > 1 in 3-D),
 * ENOMEM, EDEVICE. */
int lmmew_set_scatter_pixel_grid(lmmew_ctx *ctx, int grid, hipStream_t stream);

/* Pixels at which the exact scattered part is evaluated per event row: the
 * node count with a coarse grid, else the support size.  EINVAL for NULL. */
int lmmew_scatter_pixel_grid_nodes(const lmmew_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Figures of merit for regional uptake (Sec. 3.1.4)
 * ------------------------------------------------------------------------- */

/* Uptake of each region in each image: out[c][k] = sum over the pixels q
 * with masks[k][q] != 0 of lambda[c][q], summed in FP64 (deterministic).
 *   lambda  device [n_cases][n*n] float;  masks  device [n_rois][n*n] uint8;
 *   out     host [n_cases][n_rois] double.
 * Synchronises.  Errors: EINVAL, ENOMEM, EDEVICE. */
int lmmew_roi_uptake(lmmew_ctx *ctx, const float *lambda, int n_cases, const uint8_t *masks,
                     int n_rois, double *out, hipStream_t stream);

/* Largest n_cases * n_rois that lmmew_roi_uptake_noalloc accepts. */
#define LMMEW_ROI_NOALLOC_MAX 65536

/* lmmew_roi_uptake for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc): the same kernel and the
 * same results (bitwise), with the per-(case, region) sums staged in a static
 * device array of LMMEW_ROI_NOALLOC_MAX doubles (512 KiB) that the library
 * holds on every device it runs on until the process ends, instead of a
 * buffer allocated per call.  The call allocates nothing and calls no
 * allocating routine; it still synchronises the stream to copy the sums to
 * out.  Every call on a device shares that device's array: calls that
 * overlap on one device (other host threads or streams) race and must be
 * serialised by the caller.
 * Errors: EINVAL (as lmmew_roi_uptake, and n_cases * n_rois >
 * LMMEW_ROI_NOALLOC_MAX), EDEVICE. */
int lmmew_roi_uptake_noalloc(lmmew_ctx *ctx, const float *lambda, int n_cases,
                             const uint8_t *masks, int n_rois, double *out, hipStream_t stream);

/* Ensemble figures of merit of Sec. 3.1.4 over S object realisations x N
 * noise realisations (N >= 2) for K regions (host arrays, no device work):
 *   est    [S][N][K] estimated uptake, truth [S][K] true uptake (nonzero);
 *   enrmse [K]  (1/S) sum_s sqrt(mean_n (est - y)^2) / y
 *   bias   [K]  (1/(S N)) sum_s sum_n (est - y) / y
 *   std_   [K]  (1/S) sum_s sqrt(sum_n (est - mean_n est)^2 / (N - 1)) / y
 * Any output pointer may be NULL.  Errors: EINVAL. */
int lmmew_roi_metrics(const double *est, const double *truth, int S, int N, int K, double *enrmse,
                      double *bias, double *std_);

#ifdef __cplusplus
}
#endif

#endif /* LMMEW_H */
