/*
 * nbreg.h -- C ABI of the MI355X (gfx950) Ahmad-Cohen regular-force library.
 *
 * The library computes, for an active block of bodies, the regular force (the
 * Newtonian acceleration from every body OUTSIDE the body's neighbour radius,
 * G = 1, no softening) together with its first time derivative (jerk), and
 * builds the neighbour list (the bodies INSIDE the radius) in the same pass.
 * This is the Ahmad-Cohen split of Wang et al. 2015 (NBODY6++GPU), section 2,
 * and the GPU regular-force step of section 3.2.1 (Table 1, "Reg."); the
 * all-particle Hermite prediction that feeds it is Table 1 "Pred." and
 * section 3.3.3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers are DEVICE pointers owned by the caller unless a name ends in
 *    _host.  Nothing is copied to or from the host except where stated.
 *  - Body state is structure-of-arrays FP64: a "[3][n] plane" array holds
 *    component k of body j at element k*n + j.  Per-row outputs are [3][n_i]
 *    planes with the same convention (plane stride n_i).
 *  - Every call is asynchronous on the context's stream and returns before
 *    the GPU work finishes; read outputs after synchronising that stream.
 *    Growing the context's scratch memory may synchronise the device.
 *    Calls on one context must not overlap in time: the context keeps device
 *    words of its own (the mixed-precision refinement counter) that each
 *    regular-force call uses.  Calls queued on the context's one stream are
 *    ordered; after nb_ctx_set_stream, order the new stream after the old
 *    one's pending work.
 *  - Return value: NB_OK (0) or a negative NB_ERR_* code.  Host-checkable
 *    argument errors are reported this way and launch nothing.  Nothing throws
 *    across the ABI.
 *  - Device-detected conditions are reported in the optional 'status' word
 *    (bit-or of NB_STATUS_*; the library ORs bits in, it never clears them, so
 *    the caller zeroes it) and, for list overflow, in the 'overflow' word
 *    (written 0 or 1 by the call itself).
 *  - A neighbour is decided by one canonical single-precision test, the same
 *    in every kernel and precision: with dx = x_j - x_i in FP64 (likewise dy,
 *    dz), fx = (float)dx, r2f = fmaf(fz, fz, fmaf(fy, fy, fx * fx)), body j
 *    (j != i) is a neighbour of row b iff r2f < (float)rs2[b].  Equality is
 *    regular.  rs2[b] <= 0 means "no neighbours".  The self pair is excluded.
 *  - Neighbour lists are in ascending body index.  A row with more than nb_cap
 *    neighbours keeps its first nb_cap (in ascending order); nb_count holds the
 *    true count and 'overflow' is set.  Forces never depend on nb_cap.
 */
#ifndef NBREG_H
#define NBREG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nb_ctx nb_ctx;

typedef enum {
    NB_FP64 = 0,
    NB_MIXED = 1,
    /* range markers only: they make every int a representable nb_precision,
     * so an out-of-range value passed through the ABI is a checked argument
     * error (NB_ERR_INVALID_ARG), not undefined behaviour in the library */
    NB_PRECISION_RANGE_MIN_ = -2147483647 - 1,
    NB_PRECISION_RANGE_MAX_ = 2147483647
} nb_precision;

enum {
    NB_OK = 0,
    NB_ERR_INVALID_ARG = -1, /* bad size, NULL required pointer, bad enum      */
    NB_ERR_HIP = -2,         /* a HIP runtime call failed                      */
    NB_ERR_OOM = -3,         /* scratch could not be grown (or exceeds limit)  */
    NB_ERR_UNSUPPORTED = -4, /* no gfx950 device, or an unsupported plan       */
    NB_ERR_TOO_LARGE = -5    /* block too large for the fixed workspace of     */
                             /* nb_regular_force_noalloc                       */
};

enum {
    NB_STATUS_OVERFLOW = 1,  /* some row has more neighbours than nb_cap       */
    NB_STATUS_BAD_INDEX = 2, /* some i_block entry outside [0, n); row zeroed  */
    NB_STATUS_NONFINITE = 4, /* some output is Inf/NaN (e.g. coincident bodies */
                             /* outside each other's radius)                   */
    NB_STATUS_BAD_LEVEL = 8  /* scheduler: a step level or list entry out of   */
                             /* range, or a prefix that is not the due block;  */
                             /* the list and offsets were left unchanged       */
};

/* ---- context ------------------------------------------------------------ */

/* Creates a context on HIP device 'device' that launches on 'hip_stream'
 * (a hipStream_t; NULL = the default stream).  Fails with NB_ERR_UNSUPPORTED
 * if the device is not gfx950. */
int nb_ctx_create(nb_ctx **out, int device, void *hip_stream);
/* Changes the stream later calls launch on. */
int nb_ctx_set_stream(nb_ctx *ctx, void *hip_stream);
/* Frees scratch, cached graphs and events.  Synchronises the stream first. */
int nb_ctx_destroy(nb_ctx *ctx);
const char *nb_error_string(int code);
int nb_version(void);

/* Plan override used by tests and the autotuner: 0 in a field means "choose
 * automatically".  mapping: 1 = one row per lane with j-tiles in LDS
 * (256-lane work-groups), 2 = 1, 2 or 4 rows per wavefront with j spread
 * over lanes (the smallest blocks), 3 = one row per lane in one-wave
 * work-groups with 64-body LDS tiles (automatic for blocks above 40 rows
 * whose rows fill 64-row tiles more than 1.2 times better than 256-row
 * ones, so at most 832 rows).  rows_per_lane: 1, 2 or 4 (mapping 1; rows per wave for mapping 2;
 * ignored by mapping 3).  splits: number of contiguous j ranges whose partial
 * sums are combined in FP64 (>= 1).  The override holds until changed; pass
 * all zeros to go back to automatic plans. */
int nb_ctx_set_plan(nb_ctx *ctx, int mapping, int rows_per_lane, int splits);
/* Describes the plan of the last nb_regular_force call into buf (text). */
int nb_ctx_last_plan(nb_ctx *ctx, char *buf, int len);
/* Upper bound on scratch bytes the context may hold (0 = no bound). */
int nb_ctx_set_scratch_limit(nb_ctx *ctx, int64_t bytes);

/* Kernel timing: when enabled, every launch (or launch sequence) of the
 * library's kernels is bracketed by HIP events on the context's stream.
 * nb_ctx_kernel_time synchronises those events and returns the summed
 * milliseconds and the launch count of one kernel class since the last reset:
 * 0 = regular force main kernel, 1 = cross-split reduce, 2 = predictor,
 * 3 = adjoint, 4 = batched, 5 = mixed-precision FP64 refinement,
 * 6 = irregular force (with its pack), corrector and potential,
 * 7 = block-step scheduler, 8 = radius control (update, compaction and
 * scatter; the recomputed rows count under 0, 1 and 5). */
int nb_ctx_enable_timing(nb_ctx *ctx, int on);
int nb_ctx_kernel_time(nb_ctx *ctx, int kernel_class, double *ms, int64_t *launches);
int nb_ctx_reset_timing(nb_ctx *ctx);
/* Mixed precision refinement: every NB_MIXED row also accumulates an estimate
 * of its FP32 rounding error (from the squared norms of its FP32 partial
 * sums); a row whose estimate times 'safety' exceeds tol times the norm of its
 * acc or jerk is recomputed in FP64 by a follow-up kernel on the same stream
 * (forces only; lists are already exact).  Defaults: tol 5e-6, safety 32.
 * tol = 0 turns the refinement off. */
int nb_ctx_set_mixed_tolerance(nb_ctx *ctx, double tol, double safety);
/* Test override of the refinement's buffer: at most 'rows' refined rows of a
 * single-block call (nb_regular_force, nb_regular_force_noalloc) keep chunk
 * partials, summed by the whole GPU; the others are refined one work-group
 * per row, chunk after chunk, to the same bits.  0 = automatic (as many rows
 * as 2^20 chunk partials hold); rows < 0 is NB_ERR_INVALID_ARG. */
int nb_ctx_set_refine_buffer_rows(nb_ctx *ctx, int32_t rows);
/* Number of rows the last NB_MIXED nb_regular_force call recomputed in FP64
 * (0 if refinement was off).  Synchronises the context's stream. */
int nb_ctx_last_refined_rows(nb_ctx *ctx, int32_t *rows);

/* ---- hot path ----------------------------------------------------------- */

/* Hermite predictor of all n bodies to block time t (section 3.3.3: every
 * body is predicted once for the regular force; the force and its first
 * derivative from the body's last step drive the prediction, section 2):
 *   dt = t - t0[j];  xp = x + v dt + a dt^2/2 + jrk dt^3/6;
 *   vp = v + a dt + jrk dt^2/2,
 * evaluated in FP64 in the fixed Horner order
 *   xp = fma(dt, fma(dt, fma(dt, jrk*C6, a*0.5), v), x),
 *   vp = fma(dt, fma(dt, jrk*0.5, a), v),  C6 = FP64 nearest 1/6,
 * so results are bit-reproducible.  x, v, a, jrk, xp, vp: [3][n] planes;
 * t0: [n].  m and m32 are optional (both NULL, or both set): m32[j] =
 * (float)m[j].  In-place (xp == x, vp == v) is allowed. */
int nb_predict(nb_ctx *ctx, int64_t n, double t, const double *x, const double *v,
               const double *a, const double *jrk, const double *t0, const double *m,
               double *xp, double *vp, float *m32);

/* Regular force + jerk + neighbour lists (section 2, section 3.2.1).
 * j-set: all n bodies, predicted positions xp and velocities vp ([3][n]
 * planes) and masses m ([n]).  Rows b = 0 .. n_i-1 are bodies i_block[b]
 * with squared neighbour radius rs2[b]; duplicate rows are allowed and are
 * computed independently.  For row b with i = i_block[b]:
 *   acc_b  = sum_{j regular} m_j r / |r|^3,
 *   jerk_b = sum_{j regular} m_j [ u / |r|^3 - 3 (r.u) r / |r|^5 ],
 * r = xp_j - xp_i, u = vp_j - vp_i, regular = not a neighbour and j != i.
 * prec = NB_FP64: all arithmetic in FP64.  prec = NB_MIXED: differences in
 * FP64, then r^-1 (hardware reciprocal square root), r^-2, r^-3 and the force
 * and jerk products in FP32, summed in short FP32 runs folded into FP64
 * running sums, with FP64 cross-split reduction; pairs closer than two
 * neighbour radii are evaluated in FP64, and rows whose rounding-error
 * estimate is too large are recomputed in FP64 (nb_ctx_set_mixed_tolerance).
 * Small blocks (n_i <= 40 under automatic plans) are latency-bound, and an
 * NB_MIXED request on them runs the FP64 kernels instead: no slower there,
 * no refinement, and results to the FP64 bar (nb_ctx_last_plan then reads
 * "prec=fp64 requested=mixed"; a plan set by nb_ctx_set_plan keeps the
 * mixed kernels).
 * Outputs: acc, jerk [3][n_i] FP64; nb_count [n_i] (true count); nb_list
 * [n_i][nb_cap] row-major (first min(count, nb_cap) entries of a row are
 * defined); *overflow (required) = 1 iff some count > nb_cap, else 0;
 * status (optional) gets NB_STATUS_* bits.  A row whose i_block entry is
 * outside [0, n) gets zero acc/jerk, count 0 and NB_STATUS_BAD_INDEX.
 * Errors: n <= 0 or n > INT32_MAX, n_i < 0, nb_cap < 0, NULL required
 * pointer (nb_list may be NULL only when nb_cap == 0), bad prec.
 * n_i == 0 is valid and only clears *overflow. */
int nb_regular_force(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                     const double *m, int32_t n_i, const int32_t *i_block,
                     const double *rs2, int32_t nb_cap, nb_precision prec, double *acc,
                     double *jerk, int32_t *nb_count, int32_t *nb_list, int32_t *overflow,
                     uint32_t *status);

/* Allocation-free variant of nb_regular_force, for callers that cannot
 * allocate device memory during the call: code being captured into a HIP
 * graph, tight serving or stepping loops, and harnesses that forbid
 * hipMalloc.  Same arguments, outputs, rules and kernels as nb_regular_force,
 * but the split partials, neighbour segments and refinement lists live in a
 * fixed device workspace that is part of the library itself (one copy per
 * GPU, nb_fixed_workspace_bytes() bytes, held from the first context created
 * on that GPU until the process ends) instead of context scratch.  The call
 * allocates nothing, creates no events and never synchronises.  When the
 * automatic (or forced) plan's scratch does not fit the workspace, the split
 * count is lowered until it does (results stay within the same tolerances;
 * FP64 sums may differ in the last bits from nb_regular_force, lists are
 * identical).  Errors as nb_regular_force, plus NB_ERR_TOO_LARGE when even a
 * single split does not fit (only NB_MIXED blocks of several million rows),
 * and NB_ERR_UNSUPPORTED if the workspace could not be located on the
 * context's device.  The workspace keeps the last call's contents; every
 * call on a GPU, from any context or stream, uses the same workspace, so
 * calls that overlap in time on one GPU race and must be serialised by the
 * caller (one stream, or events). */
int nb_regular_force_noalloc(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                             const double *m, int32_t n_i, const int32_t *i_block,
                             const double *rs2, int32_t nb_cap, nb_precision prec,
                             double *acc, double *jerk, int32_t *nb_count, int32_t *nb_list,
                             int32_t *overflow, uint32_t *status);
/* Size in bytes of the fixed workspace of nb_regular_force_noalloc (host
 * only; no GPU work). */
int nb_fixed_workspace_bytes(int64_t *bytes);

/* Adjoint of nb_regular_force (no counterpart in the paper): given upstream
 * weights w_a, w_j ([3][n_i] FP64), the gradient of
 *   L = sum_b w_a[:,b] . acc_b + w_j[:,b] . jerk_b
 * with respect to xp, vp ([3][n] planes) and m ([n]), with neighbour
 * membership frozen (the canonical test at the given xp decides membership
 * and is treated as constant).  FP64 throughout; pair terms are recomputed,
 * nothing per pair is stored.  gx, gv, gm are overwritten (bodies in no
 * regular pair get 0).  Same argument rules as nb_regular_force. */
int nb_regular_force_adjoint(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                             const double *m, int32_t n_i, const int32_t *i_block,
                             const double *rs2, const double *w_a, const double *w_j,
                             double *gx, double *gv, double *gm, uint32_t *status);

/* Batched ensemble: n_clusters independent clusters in one launch.  Cluster
 * c owns bodies [j_off_host[c], j_off_host[c+1]) of the concatenated xp, vp,
 * m arrays (planes of length n_total = j_off_host[n_clusters]) and rows
 * [i_off_host[c], i_off_host[c+1]) of i_block/rs2/outputs (n_rows =
 * i_off_host[n_clusters]).  Body indices in i_block and in nb_list are
 * GLOBAL indices into the concatenated arrays; a row's j-set is its own
 * cluster only.  The work of all clusters runs in one persistent kernel that
 * pulls (cluster, row-tile, j-range) items from a queue; the launch sequence
 * for a given shape is captured once into a HIP graph and replayed.
 * Offsets are host arrays of n_clusters+1 int64, non-decreasing, starting
 * at 0.  Outputs and rules as nb_regular_force. */
int nb_regular_force_batched(nb_ctx *ctx, int32_t n_clusters, const int64_t *j_off_host,
                             const int64_t *i_off_host, const double *xp,
                             const double *vp, const double *m, const int32_t *i_block,
                             const double *rs2, int32_t nb_cap, nb_precision prec,
                             double *acc, double *jerk, int32_t *nb_count,
                             int32_t *nb_list, int32_t *overflow, uint32_t *status);

/* Batched kernel shape override (tests and the batched tuner): the LDS tile
 * length (j bodies staged per tile), the work-group width in lanes, the rows
 * each lane holds, and the work cap (the ensemble's pair work is cut into
 * items of about 1/(items_per_cu x CUs) of the total, by j-splits of whole
 * 256-body units).  Built shapes (tile, lanes, rows_per_lane): (256, 256, 1)
 * (the default), (256, 256, 2), (128, 128, 1), (64, 64, 1), (512, 512, 1),
 * (256, 512, 1); others give NB_ERR_UNSUPPORTED.  items_per_cu in [1, 4096]
 * (0 = 64).  All zero = automatic (tuned shape if nb_autotune_batched has
 * tuned this ensemble, else the default).  Results do not depend on the
 * shape: a row's sums follow the j order of its cluster's splits, which
 * depend only on the split count. */
int nb_ctx_set_batched_shape(nb_ctx *ctx, int tile, int lanes, int rows_per_lane,
                             int items_per_cu);

/* Autotuner of the batched ensemble (an extension of the regular-force step
 * of section 3.2.1; the paper runs one cluster at a time): with the same
 * arguments as nb_regular_force_batched, times every built kernel shape with
 * work caps of 16, 64 and 256 items per CU (graph replays, best of three)
 * on the caller's own ensemble, and keeps the fastest for this ensemble
 * (keyed by precision, nb_cap and both offset arrays); later
 * nb_regular_force_batched calls on it use that shape.  The outputs are
 * written by every trial and finally by the tuned shape.  If cache_path
 * names a file written by an earlier run that holds this ensemble, its
 * entries are loaded instead (flags & 1 forces re-tuning); after tuning all
 * tuned ensembles of the context are written there.  Synchronises the
 * stream.  Errors as nb_regular_force_batched. */
int nb_autotune_batched(nb_ctx *ctx, int32_t n_clusters, const int64_t *j_off_host,
                        const int64_t *i_off_host, const double *xp, const double *vp,
                        const double *m, const int32_t *i_block, const double *rs2,
                        int32_t nb_cap, nb_precision prec, double *acc, double *jerk,
                        int32_t *nb_count, int32_t *nb_list, int32_t *overflow,
                        uint32_t *status, const char *cache_path, int flags);

/* Autotuner: times the candidate plans (rows per lane, splits, mapping) on
 * synthetic Plummer-like data for a ladder of block sizes at the given n,
 * for both precisions (for NB_MIXED blocks of up to 256 rows, also the FP64
 * kernels), and stores the fastest per (precision, n bucket, n_i bucket).
 * If cache_path names a readable file written by an earlier run (text, first
 * line "nbreg-tune 2"), the table is loaded from it instead (flags & 1
 * forces re-tuning); after tuning the table is written there.  Synchronises
 * the device. */
int nb_autotune(nb_ctx *ctx, int64_t n, const char *cache_path, int flags);

/* ---- the rest of the block step ---------------------------------------- */

/* Irregular force + jerk (section 2: the irregular force sums only the
 * neighbours): for row b with body i = i_block[b], the same pair terms as
 * nb_regular_force summed over the first min(nb_count[b], nb_cap) entries of
 * row b of nb_list ([n_i][nb_cap], as written by nb_regular_force).  FP64.
 * acc, jerk: [3][n_i].  Entries outside [0, n) or equal to i are skipped and
 * set NB_STATUS_BAD_INDEX; a bad i_block entry gives a zero row.  With the
 * lists of a regular-force call on the same state, regular + irregular is the
 * full Newtonian force and jerk.  For n_i >= n/128 the bodies are first
 * packed into context scratch (64 B per body, one cache line per neighbour
 * gather); the results are the same either way.  Errors: n <= 0 or
 * n > INT32_MAX, n_i < 0, nb_cap < 0, NULL required pointer. */
int nb_irregular_force(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                       const double *m, int32_t n_i, const int32_t *i_block, int32_t nb_cap,
                       const int32_t *nb_count, const int32_t *nb_list, double *acc,
                       double *jerk, uint32_t *status);

/* Fourth-order Hermite corrector of the integrator (section 2), entry-wise
 * over n entries with step h[n] (all other arrays [3][n] planes, FP64):
 *   v1 = v0 + h/2 (a0 + a1) + h^2/12 (j0 - j1)
 *   x1 = x0 + h/2 (v0 + v1) + h^2/12 (a0 - a1)
 *   a3 = (12 (a0 - a1) + 6 h (j0 + j1)) / h^3
 *   a2 = (-6 (a0 - a1) - h (4 j0 + 2 j1)) / h^2 + h a3   (second derivative at
 *        the end of the step)
 * where a0, j0 are the force and jerk at the start of the step and a1, j1 at
 * its end (evaluated on the predicted state).  Outputs may alias x0 / v0.
 * Errors: n <= 0 or n > INT32_MAX, NULL pointer. */
int nb_hermite_correct(nb_ctx *ctx, int64_t n, const double *h, const double *x0,
                       const double *v0, const double *a0, const double *j0, const double *a1,
                       const double *j1, double *x1, double *v1, double *a2, double *a3);

/* Potential (section 3.2.1; used for the energy check and the scaling to
 * N-body units, section 3.3.2): phi[i] = -sum_{j != i} m_j / |x_j - x_i|
 * (x: [3][n] plane, FP64) and, if energy is not NULL, *energy (one device
 * double) = 1/2 sum_i m_i phi_i, reduced in a fixed order.  1/|r| is the
 * hardware estimate refined by one Newton step (relative error below 5e-15;
 * the terms share one sign, so the sum keeps that bound).  Errors: n <= 0 or
 * n > INT32_MAX, NULL x, m or phi. */
int nb_potential(nb_ctx *ctx, int64_t n, const double *x, const double *m, double *phi,
                 double *energy);

/* ---- neighbour-radius control (Table A1: neighbour number toward NNBOPT) -- */

/* The paper steers each body's neighbour number toward the input parameter
 * NNBOPT.  Rule used here (uniform density: the count grows as the sphere's
 * volume): rs2 is scaled by f = (target / count)^(2/3), where the 2/3 power is
 * computed as the cube root of q*q by eight Newton steps
 *   y <- y - (y*y*y - x) / (3*y*y)   (as t = y*y; y - (t*y - x) / (3*t))
 * from y = 2^floor(e/3), q*q = frac * 2^e with frac in [0.5, 1), in IEEE FP64
 * without contraction, so results are reproducible bit for bit.
 *
 * nb_radius_update: next-step squared radii of a block, row by row:
 *   rs2_new[b] = rs2[b] * min(max(f, f_min), f_max),  target = nnbopt,
 *   count = max(nb_count[b], 1);  rows with rs2[b] <= 0 are copied unchanged.
 * nb_count, rs2, rs2_new: [n_i] device arrays; rs2_new may alias rs2.
 * Errors: n_i < 0, nnbopt < 1, f_min <= 0, f_max < f_min or not finite, NULL
 * arrays with n_i > 0. */
int nb_radius_update(nb_ctx *ctx, int32_t n_i, const int32_t *nb_count, const double *rs2,
                     int32_t nnbopt, double f_min, double f_max, double *rs2_new);

/* nb_regular_force_fit: nb_regular_force, then up to max_rounds rounds of:
 * every row with nb_count > nb_cap gets rs2[b] *= min(max(f, 1/4), 1) with
 * target = min(nnbopt, nb_cap), and those rows alone are recomputed with the
 * new radii (their acc, jerk, count and list replace the old ones).  rs2 is
 * IN/OUT: the caller's array holds the final radii.  Rounds stop when no row
 * overflows; *overflow reports the final state (status, which is only ever
 * OR-ed, keeps NB_STATUS_OVERFLOW from a round even when a later round
 * resolved it).  Each round synchronises the stream twice (to read the
 * overflow word and the number of rows).
 * rounds_host (optional, host) receives the number of rounds made.  Rows are
 * recomputed in ascending row order, so results are deterministic and a row's
 * result equals a plain nb_regular_force call with its final radius.
 * Arguments and outputs as nb_regular_force, plus: nb_cap >= 1, nnbopt >= 1,
 * max_rounds >= 0 (0: plain nb_regular_force). */
int nb_regular_force_fit(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                         const double *m, int32_t n_i, const int32_t *i_block, double *rs2,
                         int32_t nb_cap, nb_precision prec, int32_t nnbopt, int32_t max_rounds,
                         double *acc, double *jerk, int32_t *nb_count, int32_t *nb_list,
                         int32_t *overflow, uint32_t *status, int32_t *rounds_host);

/* ---- block-step scheduler: the sorting list (section 3.3.1) ------------- */

/* Every body has a step 2^-level[j] (level in [0, k_max], k_max <= 63).  The
 * sorting list is the body index list ordered by step from the smallest to
 * the largest (level descending), with boundary offsets
 *   level_end[L] = number of bodies with level >= L,  L = 0 .. k_max+1,
 * so the bodies of level L are order[level_end[L+1] : level_end[L]]; the
 * paper's I_off(L), the last list position of step 2^-L, is level_end[L]-1.
 * With synchronised block steps (every body's time a multiple of its step)
 * the bodies due at a block time whose coarsest dividing step is 2^-L are
 * the prefix order[0 : level_end[L]], which can be passed as i_block as is.
 *
 * nb_sched_build: full build from level[n] (device).  order [n] and level_end
 * [k_max+2] (device) are overwritten; bodies of equal level are listed by
 * ascending index.  A level outside [0, k_max] sets NB_STATUS_BAD_LEVEL and
 * leaves order and level_end unchanged.  Errors: n <= 0 or n > INT32_MAX,
 * k_max outside [0, 63], NULL required pointer. */
int nb_sched_build(nb_ctx *ctx, int64_t n, const int32_t *level, int32_t k_max, int32_t *order,
                   int32_t *level_end, uint32_t *status);

/* nb_sched_update: after the block of level L (the n_active = level_end[L]
 * bodies order[0 : n_active]) has been integrated and level[] holds their
 * new levels, re-sorts that prefix by the new levels and rewrites
 * level_end[L .. k_max+1]; the rest of the list and level_end[0 .. L-1] are
 * untouched.  O(n_active) work.  A new step must divide the block time, so
 * every new level must lie in [L, k_max]; bodies of one level may come out in
 * any order.  If a new level is out of that range, a list entry is outside
 * [0, n), or level_end[L] != n_active, NB_STATUS_BAD_LEVEL is set and order
 * and level_end are left unchanged.  n_active == 0 is a no-op.  Errors: as
 * nb_sched_build, plus L outside [0, k_max] or n_active outside [0, n]. */
int nb_sched_update(nb_ctx *ctx, int64_t n, int32_t n_active, int32_t L, const int32_t *level,
                    int32_t k_max, int32_t *order, int32_t *level_end, uint32_t *status);

/* nb_sched_next (host only, no GPU work): the offset search of Figure 1.
 * From the current block time t_now and a HOST copy of level_end, the
 * smallest step is that of the deepest occupied level kd, the next block time
 * is *t_new = t_now + 2^-kd, *level = the coarsest L whose step 2^-L divides
 * *t_new, and *n_active = level_end[L].  Errors (NB_ERR_INVALID_ARG): an
 * empty or non-monotone level_end, t_now negative, non-finite or not a
 * multiple of 2^-kd, or t_now too large for 2^-kd to change it. */
int nb_sched_next(double t_now, int32_t k_max, const int32_t *level_end_host, double *t_new,
                  int32_t *level, int32_t *n_active);

#ifdef __cplusplus
}
#endif
#endif /* NBREG_H */
