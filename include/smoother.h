/*
 * smoother.h -- C ABI of the MI355X (gfx950) parallel-in-time iterated smoother.
 *
 * The library computes the iterated extended (Taylor) or sigma-point
 * (statistical linear regression) Kalman smoother of Yaghoobi, Corenflos,
 * Hassan and Sarkka, "Parallel Iterated Extended and Sigma-Point Kalman
 * Smoothers" (ICASSP 2021), with the filter and the smoother of every
 * iteration evaluated as associative scans (Section 4, eq. 13-19).
 *
 * Problem (Section 3, eq. 4): for every track,
 *     x_k = f(x_{k-1}) + q_{k-1},   q ~ N(0, Q),      k = 1..T
 *     y_k = h(x_k) + r_k,           r ~ N(0, R),
 *     x_0 ~ N(m0, P0);
 * wanted: Gaussian approximations N(xbar_k, Pbar_k) of p(x_k | y_{1:T}),
 * k = 0..T, after M re-linearisations around the previous smoothed trajectory.
 *
 * f and h cannot cross a C ABI as device code, so they are chosen from a
 * compiled-in registry (sm_model) with a parameter block:
 *   SM_MODEL_LINEAR:      params = [F (nx*nx), c (nx), H (ny*nx), d (ny)],
 *                         row-major; f(x) = F x + c, h(x) = H x + d.
 *   SM_MODEL_CT_BEARINGS: params = [dt, (sx, sy, target) * ny]; the state is
 *                         nx/5 stacked coordinated-turn blocks
 *                         [px, py, vx, vy, omega]; sensor s measures
 *                         atan2(py - sy, px - sx) of block `target`.
 *                         Bearing innovations are wrapped to [-pi, pi) around
 *                         h(xbar_k) of the current linearisation point.
 *                         Supported: nx = 5 with ny = 2; and, with the Taylor
 *                         linearisation, k = nx / 5 stacked targets
 *                         (2 <= k <= 16) with two sensors per target and Q, R,
 *                         P0 (and init_cov) without terms between different
 *                         targets (|A_ij| <= 1e-12 sqrt(A_ii A_jj); smaller
 *                         terms are dropped).  Such targets do not interact,
 *                         the covariances stay block-diagonal, and the library
 *                         smooths each target as its own block (exact up to
 *                         rounding); off-block covariance outputs are zero.
 *                         Sigma-point rules couple stacked targets through
 *                         their regression residuals; with them, four targets
 *                         and eight sensors (nx = 20, ny = 8, FP64 or FP32,
 *                         any SPD Q, R, P0) run on an engine of the full state
 *                         in which one wavefront cooperates on each element;
 *                         its FP32 form keeps records, elements and scans in
 *                         FP32 and computes the regression in FP64.
 *
 * Conventions shared by every call:
 *   - Status: every call returns sm_status and never aborts or throws across the
 *     ABI; smoother_last_error() returns a message for the last failure.
 *   - Ownership: smoother_init copies every input; the caller keeps its buffers.
 *     The handle owns all device memory it allocates.  Result buffers are
 *     caller-owned, on the host (smoother_result) or on the device
 *     (smoother_result_device).
 *   - Layout: row-major; tracks are concatenated.  Track i has
 *     T_i = offsets[i+1] - offsets[i] >= 1 measurements and T_i + 1 states
 *     (slots) x_0..x_T; state arrays hold the slots of track 0, then track 1, ...
 *   - Failed tracks: a track whose iterate turns non-finite (for example from
 *     a broken caller-supplied trajectory) gets a NaN change statistic, and
 *     the call that asked for the delta returns SM_ENUMERIC; the other tracks
 *     of the batch are unaffected and their results stay valid, since every
 *     track's prior and end elements restart both scans (Section 4).
 *   - Streams: all device work of a handle is queued on the stream given to
 *     smoother_init (NULL = the default stream).  One handle per host thread at
 *     a time; handles on different streams are independent.
 */
#ifndef SMOOTHER_H_
#define SMOOTHER_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smoother* smoother_t;

typedef enum {
  SM_OK = 0,
  SM_EINVAL = 1,    /* invalid argument; decided on the host before device work */
  SM_ENOMEM = 2,    /* device allocation failed or exceeds max_device_bytes */
  SM_EDEVICE = 3,   /* HIP runtime error */
  SM_ENUMERIC = 4,  /* non-finite iterate (see smoother_track_deltas) */
  SM_ESTATE = 5     /* call not valid for this handle (e.g. NULL handle) */
} sm_status;

typedef enum { SM_MODEL_LINEAR = 0, SM_MODEL_CT_BEARINGS = 1 } sm_model;

/* Linearisation (Section 3): first-order Taylor at the previous smoothed mean
 * (eq. 10, IEKS) or statistical linear regression with sigma points of the
 * previous smoothed mean and covariance (eq. 7-9, IPLS). */
typedef enum { SM_LIN_TAYLOR = 0, SM_LIN_CUBATURE = 1, SM_LIN_UNSCENTED = 2 } sm_lin;

typedef enum { SM_FP64 = 0, SM_FP32 = 1 } sm_precision;

/* SM_SCAN_PARALLEL: prefix/suffix associative scans (eq. 15, eq. 19).
 * SM_SCAN_SEQUENTIAL: the same linearised model filtered and smoothed by the
 * sequential Kalman/RTS recursions, one lane per track (comparison baseline). */
typedef enum { SM_SCAN_PARALLEL = 0, SM_SCAN_SEQUENTIAL = 1 } sm_scan;

/* How the parallel scans carry the covariance-like blocks of the elements.
 * SM_FORM_COVARIANCE: as matrices, the elements (A, b, C, eta, J) and
 * (E, g, L) of eq. 13-19.  SM_FORM_SQRT: as lower-triangular factors
 * C = U U^T, J = Z Z^T, L = D D^T, with the operators of eq. 15 and eq. 19
 * rewritten on the factors (new factors from LQ decompositions, no
 * covariance is formed and re-factorised, no difference of covariances is
 * taken); algebraically the same results, in more arithmetic.  Outputs are
 * covariances in both forms.  Eq. 15 needs I + C_i J_j invertible, not C_i
 * positive definite: the factor form takes a positive semi-definite Q, whose
 * zero-variance directions become zero columns of the factor of Q', while
 * the covariance form factorises C_i and needs Q positive definite. */
typedef enum { SM_FORM_COVARIANCE = 0, SM_FORM_SQRT = 1 } sm_form;

typedef struct {
  int32_t nx, ny;                 /* state / measurement dimension */
  int32_t n_tracks;               /* >= 1 */
  const int64_t* offsets;         /* host [n_tracks+1], offsets[0] = 0, strictly increasing */
  int32_t model;                  /* sm_model */
  const double* params;           /* host [n_params], see sm_model */
  int32_t n_params;
  const double* Q;                /* host [nx*nx], symmetric positive definite; with
                                     SM_FORM_SQRT positive semi-definite (a state component
                                     without process noise; the MAP objective then refuses) */
  const double* R;                /* host [ny*ny], symmetric positive definite */
  const double* m0;               /* host [n_tracks*nx] */
  const double* P0;               /* host [n_tracks*nx*nx], each symmetric positive definite */
  const double* y;                /* host [offsets[n_tracks]*ny], y_1..y_T of each track */
  int32_t n_iter;                 /* M, iterations run by smoother_iterate(h, 0) */
  int32_t lin;                    /* sm_lin */
  double ut_alpha, ut_beta, ut_kappa;  /* unscented parameters (lambda = alpha^2 (n+kappa) - n);
                                          beta is accepted and unused: one weight set */
  int32_t precision;              /* sm_precision */
  int32_t scan;                   /* sm_scan */
  const double* init_mean;        /* optional host [S*nx], S = sum(T_i+1); NULL = m0 broadcast */
  const double* init_cov;         /* optional host [S*nx*nx]; NULL = P0 broadcast */
  int64_t max_device_bytes;       /* 0 = no cap; otherwise SM_ENOMEM if the plan needs more */
  int32_t tile_lanes;             /* scan schedule: lanes per tile (64 or 256; 0 = auto) */
  int32_t lane_slots;             /* scan schedule: consecutive slots per lane (1..32; 0 = auto) */
  int32_t use_graph;              /* 1: iterations of the parallel path are replayed from a HIP graph
                                     captured on the first call; 0: launched one kernel at a time */
  double lm_lambda;               /* Levenberg-Marquardt damping (Section 3, damped Gauss-Newton
                                     extension): >= 0, finite; 0 = the undamped iterated smoother.
                                     Each iteration also observes every state x_k of every track
                                     through x_k + r, r ~ N(0, I/lm_lambda), with the previous
                                     iterate xbar_k as the value: this adds (lm_lambda/2)|x_k - xbar_k|^2
                                     to the objective.  Fixed points are those of the undamped
                                     smoother.  Every engine and scan mode supports it with
                                     SM_FORM_COVARIANCE; SM_FORM_SQRT needs 0. */
  int32_t form;                   /* sm_form; SM_FORM_SQRT runs on the parallel scan of the
                                     single-block engines (nx = 5 coordinated turn, the linear
                                     models) and on stacked targets with the Taylor linearisation,
                                     without damping; otherwise SM_EINVAL */
  int32_t freeze_converged;       /* 1: smoother_iterate_until takes every track that has converged
                                     (or failed) out of its later iterations: the track's result is
                                     its iterate of the iteration at which it converged, and tiles
                                     whose tracks are all out are skipped.  Batches on the parallel
                                     scan of the single-block engines; elsewhere ignored.  0: every
                                     track is iterated until the last one has converged. */
} sm_problem;

/* Fills *pb with defaults: n_tracks = 1, n_iter = 10, lin = SM_LIN_TAYLOR,
 * ut_alpha = 1, ut_beta = 0, ut_kappa = 1, FP64, parallel scan, no init, no cap,
 * automatic scan schedule, HIP-graph replay, no damping, covariance form. */
void smoother_problem_defaults(sm_problem* pb);

/* Validates the problem on the host (dimensions supported by the compiled
 * kernels, offsets, finite inputs, positive-definite Q, R, P0), allocates
 * device memory, copies the inputs to the device on `hip_stream` and sets the
 * initial trajectory (eq. 4 prior broadcast, or init_mean/init_cov).
 * On success *out is a new handle; on failure *out is NULL and the status says
 * why (the message is available from smoother_last_error(NULL)). */
sm_status smoother_init(const sm_problem* pb, void* hip_stream, smoother_t* out);

/* Scan-schedule autotuner: for every candidate schedule (tile_lanes 64 or
 * 256, lane_slots 1, 2, 4, 8 or 16) builds a handle for *pb on hip_stream, runs
 * one warm-up iteration and then three timed rounds of `iters` iterations (HIP
 * events around the graph replays; the best round counts), releases the
 * handle, and returns the fastest schedule in
 * *tile_lanes / *lane_slots and its time per iteration in *ms_per_iter
 * (nullable).  pb->tile_lanes, lane_slots and n_iter are ignored; the result
 * is meant for the same fields of the problem given to smoother_init.  The
 * schedule returned is the one the engine ran: the square-root form and the
 * full-state (nx = 20) engine fix the tile width at 64 lanes, and candidates
 * that run alike are timed once.
 * Candidates that fail (e.g. over max_device_bytes) are skipped; if none runs,
 * the last failure is returned.  Messages go to smoother_last_error(NULL). */
sm_status smoother_autotune(const sm_problem* pb, void* hip_stream, int32_t iters, int32_t* tile_lanes,
                            int32_t* lane_slots, double* ms_per_iter);

/* As smoother_autotune, through a per-process cache: a problem of the same
 * shape (device, model, nx, ny, lin, precision, form, freeze_converged,
 * whether lm_lambda is zero, use_graph, max_device_bytes, iters, and the
 * track offsets) seen before
 * returns the schedule and time measured then, without building a handle;
 * *from_cache (nullable) is 1 then and 0 after a measurement.  The cache is
 * shared by the host threads of the process (guarded) and holds one entry
 * per shape until smoother_autotune_cache_clear.  Errors as
 * smoother_autotune; failures are not cached. */
sm_status smoother_autotune_cached(const sm_problem* pb, void* hip_stream, int32_t iters, int32_t* tile_lanes,
                                   int32_t* lane_slots, double* ms_per_iter, int32_t* from_cache);

/* Empties the cache of smoother_autotune_cached. */
void smoother_autotune_cache_clear(void);

/* Runs `k` more iterations (k <= 0: the iterations left up to n_iter).  Each
 * iteration re-linearises around the current trajectory (Section 3), builds the
 * filtering elements (eq. 13-14) and combines them with a prefix scan
 * (eq. 15), builds the smoothing elements (eq. 16-18) and combines them with
 * a suffix scan (eq. 19).  Work is queued on the handle's stream; when
 * max_delta_out is not NULL the call waits and stores
 * max_{tracks,k,j} |xbar_k,j^(i) - xbar_k,j^(i-1)| of the last iteration run.
 * iters_done_out (nullable) receives the total number of iterations so far.
 * Returns SM_ENUMERIC when max_delta_out was requested and is not finite. */
sm_status smoother_iterate(smoother_t h, int32_t k, double* max_delta_out, int32_t* iters_done_out);

/* Iteration driver with the convergence rule: runs iterations (as
 * smoother_iterate) until every track's trajectory change
 * max_{k,j} |xbar_k,j^(i) - xbar_k,j^(i-1)| has been below tol at least once,
 * or max_iter iterations have run in this call.  With the problem's
 * freeze_converged, a track that has converged is not iterated again in this
 * call (its trajectory stays the iterate at which it converged); all tracks
 * are iterated again by later calls.  Waits for each iteration's
 * per-track deltas (one small copy through pinned host memory), so it returns
 * as soon as the last track has converged.  *iters_run (nullable) receives the
 * iterations run; track_iters (nullable, host [n_tracks]) the 1-based
 * iteration of this call at which each track first fell below tol, 0 if it
 * did not.  A track whose delta turns non-finite has failed: it is not waited
 * for (its entry stays 0), the other tracks run on, and the call returns
 * SM_ENUMERIC with the outputs filled.  Returns SM_EINVAL for tol <= 0 or
 * max_iter < 1. */
sm_status smoother_iterate_until(smoother_t h, double tol, int32_t max_iter, int32_t* iters_run,
                                 int32_t* track_iters);

/* One filtering pass (Section 2: the filter is the prefix of the filtering
 * elements, eq. 13-15) linearised at the current trajectory as an iteration
 * would be, without damping, and without the smoothing half.  Outputs (host,
 * each nullable): filt_mean [S*nx] and filt_cov [S*nx*nx] the filtered moments
 * x*_k, P*_k of every slot (slot 0 of a track holds m0, P0); track_loglik
 * [n_tracks] log p(y_{1:T}) of the linearised model, the sum over k of the log
 * Gaussian predictive density N(ytil_k; H_k m-_k + d_k, S_k) from the filtered
 * moments of slot k-1 (the normalising constants that eq. 14 leaves out; for a
 * linear model, the exact log marginal likelihood).  Bearing measurements
 * enter unwrapped around h(xbar_k), as in the iteration.  The trajectory, the
 * iteration count and the per-track deltas are unchanged.  Waits for the
 * stream.  On the nx = 20 sigma-point engine one wavefront builds each slot's
 * predictive density. */
sm_status smoother_filter(smoother_t h, double* filt_mean, double* filt_cov, double* track_loglik);

/* MAP objective of the current trajectory of every track (Section 3: the
 * function whose Gauss-Newton iterations are the iterated extended smoother):
 *   J(x_{0:T}) = 1/2 |x_0 - m0|^2_{P0^-1}
 *              + sum_{k=1..T} 1/2 |x_k - f(x_{k-1})|^2_{Q^-1} + 1/2 |y_k - h(x_k)|^2_{R^-1},
 * bearing residuals y_k - h(x_k) taken modulo 2 pi in [-pi, pi).  Waits for
 * the handle's stream; track_cost is host [n_tracks].  Evaluated in the
 * handle's precision per slot and summed per track in double, in a fixed
 * order.  SM_EINVAL for a NULL track_cost, or when Q is not positive definite
 * (the process residuals are weighed by Q^-1). */
sm_status smoother_objective(smoother_t h, double* track_cost);

/* Levenberg-Marquardt iterations (Section 3, the damped Gauss-Newton
 * extension of the iterated extended smoother) with Marquardt's damping
 * schedule, every track on its own: each iteration is one pass damped by
 * the track's lambda (the previous iterate observed with covariance
 * I/lambda, as lm_lambda does); the pass is kept when the track's objective
 * (smoother_objective) does not rise by more than 1e-12 |J| (1e-6 for SM_FP32,
 * the rounding of J), and lambda is divided by nu; otherwise the track's
 * trajectory is put back and lambda = min(lambda * nu, 1e16).  lambda starts
 * at lambda0 for every track.  A track has converged at the first kept pass
 * whose largest change max_{k,j} |xbar^(i) - xbar^(i-1)| is below tol while
 * its lambda is at most lambda0.  Runs until every track has converged or
 * max_iter passes; rejected passes count.  *iters_run (nullable) receives the
 * passes run, track_iters (nullable, host [n_tracks]) the 1-based pass of
 * convergence (0 = none), track_cost (nullable, host [n_tracks]) the final
 * objective.  The problem's lm_lambda is not used during the call and is used
 * again by later calls of smoother_iterate.  Covariances are those of the last
 * kept damped pass; one more smoother_iterate with lm_lambda = 0 gives the
 * undamped ones at the result.  A track whose objective is not finite at the
 * start has failed: it is not waited for (convergence entry 0, cost not
 * finite), the other tracks run on, and the call returns SM_ENUMERIC with the
 * outputs filled.  Needs the Taylor linearisation (SM_EINVAL otherwise, or for
 * invalid arguments: lambda0 > 0 and nu > 1 finite, tol > 0, max_iter >= 1).
 * Waits for the stream twice per pass. */
sm_status smoother_iterate_lm(smoother_t h, double lambda0, double nu, double tol, int32_t max_iter,
                              int32_t* iters_run, int32_t* track_iters, double* track_cost);

/* Waits for the handle's stream and copies the current trajectory to host
 * buffers: mean [S*nx], cov [S*nx*nx] (full symmetric matrices); either may be
 * NULL.  S = sum(T_i + 1), slots of track 0 first. */
sm_status smoother_result(smoother_t h, double* mean, double* cov);

/* As smoother_result, into caller-owned device buffers (same layouts, double
 * for SM_FP64 handles, float for SM_FP32 handles), queued on the handle's
 * stream without a host wait. */
sm_status smoother_result_device(smoother_t h, void* d_mean, void* d_cov);

/* Replaces the current trajectory -- the linearisation points of the next
 * iteration (Section 3) -- with caller-owned device data, queued on the
 * handle's stream without a host wait: means d_mean [S*nx] in the handle's
 * precision (double for SM_FP64, float for SM_FP32); covariances from d_cov
 * [S*nx*nx] (symmetrised), else the host matrix cov_const [nx*nx] (double,
 * symmetric positive definite) at every slot, else each track's P0.  Giving
 * both d_cov and cov_const is SM_EINVAL.  The iteration count restarts at 0
 * and the per-track deltas are cleared.  The device data are not inspected: a
 * non-finite value surfaces as SM_ENUMERIC from the next smoother_iterate
 * that asks for the delta.  Used to start from a learned initial trajectory
 * (warmstart.h, ws_trajectory). */
sm_status smoother_set_trajectory_device(smoother_t h, const void* d_mean, const void* d_cov,
                                         const double* cov_const);

/* Per-track maximum |xbar^(i) - xbar^(i-1)| of the last iteration, host
 * [n_tracks]; waits for the stream. */
sm_status smoother_track_deltas(smoother_t h, double* deltas);

/* Per-kernel timing record filled by smoother_profile. */
typedef struct {
  char name[40];        /* kernel family, e.g. "scan_up_filter" */
  int32_t launches;     /* launches timed */
  double total_ms;      /* sum of HIP-event durations of those launches */
  int64_t positions;    /* sum over launches of the slots / scan positions processed */
} sm_kernel_time;

/* Runs k iterations exactly like smoother_iterate(h, k, NULL, NULL) but with a
 * HIP event pair recorded on the handle's stream around every kernel launch,
 * waits, and reports per-kernel-family totals in out[0..*n_out-1] (at most cap
 * records).  The iterations advance the trajectory like any others. */
sm_status smoother_profile(smoother_t h, int32_t k, sm_kernel_time* out, int32_t cap, int32_t* n_out);

/* As smoother_profile, with every kernel launched `repeat` times (1..64) back
 * to back between its event pair; total_ms then sums, over the launches
 * counted in `launches`, the mean duration of the repeats, so the latency of
 * the event records and of one dispatch is spread over the repeats.  A
 * kernel that computes its outputs from buffers it does not write leaves the
 * same result after a repeat (the per-track change statistic is a maximum);
 * the one kernel that overwrites its input (the nx = 20 engine's forward
 * down-sweep, which stores each slot's smoothing element over its filtering
 * element) runs once.  So the trajectory, the deltas and the iteration count
 * come out as from smoother_iterate(h, k).  SM_EINVAL for repeat outside
 * 1..64. */
sm_status smoother_profile_repeat(smoother_t h, int32_t k, int32_t repeat, sm_kernel_time* out, int32_t cap,
                                  int32_t* n_out);

/* Number of slots S, tracks and the device bytes held by the handle. */
sm_status smoother_info(smoother_t h, int64_t* n_slots, int32_t* n_tracks, int64_t* device_bytes);

/* Scan schedule in use: lanes per tile, slots per lane, number of tiles. */
sm_status smoother_schedule(smoother_t h, int32_t* tile_lanes, int32_t* lane_slots, int64_t* tiles);

/* Allocation-free variant of smoother_init + smoother_iterate(h, 0) +
 * smoother_result_device + smoother_destroy, for callers that cannot
 * allocate device memory (serving loops, harnesses that forbid hipMalloc).
 * Runs pb->n_iter iterations from the prior broadcast and writes the final
 * trajectory to caller-owned device buffers d_mean [S*nx] and d_cov
 * [S*nx*nx] (layouts of smoother_result_device; double for SM_FP64, float
 * for SM_FP32).  max_delta_out (nullable) receives the last iteration's
 * largest change, as smoother_iterate reports it.
 *
 * Every buffer of the plan is carved out of one static device array of the
 * library (64 MiB per GPU, held from the library's load on that GPU until
 * the process ends); nothing is allocated: no hipMalloc, hipFree, pinned host
 * memory or HIP graph.  Limits, rejected with SM_EINVAL and a message before
 * any device work: at most 36864 slots (sum over tracks of T_i + 1) and 1024
 * tracks; the single-block engines only (nx = 5 coordinated turn, or the
 * compiled linear models); no init_mean/init_cov; lane_slots 0 or 1.
 * tile_lanes, lin, precision, scan and lm_lambda are honoured; use_graph and
 * max_device_bytes are ignored.
 *
 * Queued on hip_stream, and the call waits for that stream before it
 * returns.  The static array is shared by every call on the same GPU and
 * keeps the last call's contents (each call initialises what it reads):
 * calls that overlap on one GPU -- from several host threads, or on several
 * streams -- race and must not be made.  Errors as smoother_init
 * (smoother_last_error(NULL)); SM_ENUMERIC when max_delta_out was requested
 * and is not finite. */
sm_status smoother_solve_static(const sm_problem* pb, void* hip_stream, void* d_mean, void* d_cov,
                                double* max_delta_out);

/* Message for the last failure of a call on h (h = NULL: the last failure of
 * smoother_init, smoother_autotune or smoother_solve_static on this thread).
 * Valid until the next call on h. */
const char* smoother_last_error(smoother_t h);

/* Releases the handle and its device memory; NULL-safe. */
void smoother_destroy(smoother_t h);

/* Library version string. */
const char* smoother_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMOOTHER_H_ */
