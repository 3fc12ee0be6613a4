/*
 * stencil5d -- temporally blocked Jacobi-style stencil sweeps on MI355X (gfx950).
 *
 * C ABI of libstencil5d.so.  Plain C types only; no exception, abort or exit
 * ever crosses it: every entry point returns a status code and leaves a
 * detail string for s5d_last_error().
 *
 * The operation (AN5D, Background "Stencil Computation"; Table 3 for the
 * star/box stencils; Fig. 4 and "Host Code" under "Code Generation" for the
 * double-buffered time loop):
 *
 *   A[2] are two padded grids of ndim axes.  Axis 0 is the outermost
 *   (slowest-varying, C order) axis; it is also the axis the kernels stream
 *   along ("Implementation": the loop after the time loop is the streaming
 *   dimension).  Extents are interior[a] + 2*radius: the border of width
 *   `radius` on every face, both faces of axis 0 included, holds the fixed
 *   boundary values and is never written.  For t = 0 .. steps-1 every interior
 *   cell p receives
 *
 *       A[(t+1) % 2][p] = sum_k coeffs[k] * A[t % 2][p + o_k]
 *
 *   and the result is A[steps % 2], exactly where the modulo double buffer of
 *   the C program leaves it ("Host Code").
 *
 *   Offsets o_k come in ONE canonical order: lexicographic in (d0, d1[, d2]),
 *   each component in [-radius, radius], axis 0 first.  A box stencil keeps
 *   all (2r+1)^ndim offsets; a star stencil keeps the 2*r*ndim + 1 offsets
 *   with at most one non-zero component.  coeffs[k] belongs to offset o_k.
 *
 * How it is computed (AN5D, "Execution Model" and "Optimizations"): each GPU
 * launch advances b_T time steps at once.  A tile of the plane normal to axis
 * 0 streams along axis 0; every arriving plane is pushed into the 2*radius+1
 * output planes it feeds, so each fused time level holds 2*radius partial
 * sums in registers.  The tile overlaps its neighbours by b_T*radius cells on
 * each side and only its compute region is stored.  Every output sums its
 * terms in the canonical order above, so the result equals the plain loop up
 * to the rounding of the fused multiply-adds the kernels use (float64:
 * relative error far below 1e-12 for the workloads in the test-suite), and
 * every blocking choice gives the same bits.
 */
#ifndef STENCIL5D_H
#define STENCIL5D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
typedef int32_t s5d_status;
#define S5D_OK 0           /* success */
#define S5D_EINVAL 1       /* an argument is invalid (null, out of range, aliased) */
#define S5D_EUNSUPPORTED 2 /* valid, but no kernel of this library covers it */
#define S5D_ENOMEM 3       /* host allocation failed */
#define S5D_EDEVICE 4      /* a HIP runtime call failed; see s5d_last_error() */
#define S5D_EBUDGET 5      /* a memory budget would be exceeded */
#define S5D_ECANCELED 6    /* a served request was cancelled (s5d_server_cancel) */
#define S5D_ETIMEDOUT 7    /* a persistent batch's bounded wait ran out (s5d_batch_status) */

/* Stencil shape (Background "Stencil Computation"). */
#define S5D_STAR 0
#define S5D_BOX 1

/* Storage and arithmetic type of the grids. */
#define S5D_F32 0
#define S5D_F64 1

/* Accumulation of the stencil terms. */
#define S5D_ACC_PLAIN 0       /* one fused multiply-add per term, working precision */
#define S5D_ACC_COMPENSATED 1 /* float32 only: error-free products and sums
                                 (compensated dot product), one final rounding */

/* What a time step computes for an interior cell p (AN5D Table 3, the
 * synthetic and the general benchmarks).  f is the previous time level. */
#define S5D_EXPR_LINEAR 0   /* sum_k c_k f[p + o_k]: the star and box stencils.
                               coeffs: the n points' weights in canonical order */
#define S5D_EXPR_DIV 1      /* (sum_k c_k f[p + o_k]) / c0: j2d5pt (the program of
                               Fig. 4), j2d9pt, j2d9pt-gol, j3d27pt.  coeffs: the n
                               weights, then c0 (n_coeffs = n + 1).  Blocked kernels
                               for the 2D star of radius 1 and 2, the 2D box and the
                               3D box of radius 1, float32 and float64, plain
                               accumulation */
#define S5D_EXPR_GRADIENT 2 /* gradient2d, 2D star of radius 1 only:
                               cc f[p] + 1 / sqrt(c0 + sum_n (f[p] - f[n])^2) over the
                               four axis neighbours n in canonical order, each
                               operation rounded on its own (no fused multiply-add).
                               coeffs: cc, c0 (n_coeffs = 2) */
#define S5D_EXPR_VARCOEF 3  /* sum_k C[k][q] f[p + o_k]: every interior cell has its
                               own weights.  C is a device array passed to
                               s5d_run_fields; coeffs is unused (n_coeffs = 0).  2D
                               star of radius 1 and 2 and 2D box of radius 1 */

/* Problem descriptor.  Set struct_size = sizeof(s5d_desc). */
typedef struct s5d_desc {
    uint32_t struct_size;
    int32_t ndim;        /* 2 or 3 */
    int32_t radius;      /* stencil radius r >= 1 */
    int32_t shape;       /* S5D_STAR or S5D_BOX */
    int32_t dtype;       /* S5D_F32 or S5D_F64 */
    int32_t accum;       /* S5D_ACC_PLAIN or S5D_ACC_COMPENSATED (LINEAR only) */
    int64_t interior[3]; /* interior extents, axis 0 first; entries beyond ndim ignored */
    int64_t steps;       /* number of time steps T >= 0 */
    const double *coeffs;/* host pointer, n_coeffs values (see S5D_EXPR_*) in canonical
                            offset order; copied by s5d_plan_create, not retained */
    int64_t n_coeffs;    /* LINEAR: star 2*radius*ndim + 1, box (2*radius + 1)^ndim;
                            DIV: that + 1; GRADIENT: 2; VARCOEF: 0 */
    int32_t expr;        /* S5D_EXPR_* */
    int32_t reserved;    /* 0 */
} s5d_desc;

/* Blocking parameters (AN5D "Execution Model", "Division of Streaming
 * Dimension"; Table 5 header).  A zero field lets the library choose.
 * Set struct_size = sizeof(s5d_tuning). */
typedef struct s5d_tuning {
    uint32_t struct_size;
    int32_t bt;             /* temporal blocking degree b_T: time steps fused per launch */
    int32_t tile0;          /* 2D: b_S along axis 1; 3D: b_S along axis 1 (rows) */
    int32_t tile1;          /* 3D: b_S along axis 2 (columns); 2D: unused */
    int32_t stream_chunk;   /* h_SN: axis-0 length of one stream block (2D:
                               each of 8 bands of ceil(I0/8) rows, one per
                               XCD, ends in blocks of h_SN/2 rows when
                               h_SN >= 32) */
    int32_t cells_per_lane; /* consecutive cells of the last axis owned by one lane */
    int32_t rows_per_wave;  /* 3D: consecutive axis-1 rows held by one wave */
    int32_t waves_per_eu;   /* reserved: must be 0 (S5D_EINVAL otherwise) */
    int32_t kernel;         /* S5D_KERNEL_*: which kernel family runs the sweep */
} s5d_tuning;

/* Kernel families (s5d_tuning.kernel). */
#define S5D_KERNEL_AUTO 0    /* temporally blocked where compiled, else direct; direct
                                also where it measured faster: a plain-accumulation
                                2D star or box of radius <= 2, or 3D 7-point star,
                                whose tuning asks for bt = 1 and nothing else; the
                                compensated 3D stars of radius <= 2; the float32
                                125-point and compensated 27-point boxes */
#define S5D_KERNEL_BLOCKED 1 /* b_T fused steps per launch (AN5D "Execution Model") */
#define S5D_KERNEL_DIRECT 2  /* one step per launch, every radius 1..4 and shape: 2D stars
                                and boxes of radius <= 2 and 3D stars stream whole
                                rows, the others work from an LDS-staged tile (the
                                plan's bt is 1) */

typedef struct s5d_plan s5d_plan; /* opaque; immutable once created */

/* Validate `desc`, copy its coefficients and fix the blocking parameters.
 * `tuning` may be NULL (all fields chosen by the library).  On success *out
 * receives a plan that the caller releases with s5d_plan_destroy.  Errors:
 * S5D_EINVAL for malformed descriptors or tunings, S5D_EUNSUPPORTED for
 * stencils or tunings without a kernel, S5D_EDEVICE if no HIP device is
 * usable.  Nothing is enqueued. */
s5d_status s5d_plan_create(const s5d_desc *desc, const s5d_tuning *tuning, s5d_plan **out);

/* Release a plan (NULL is accepted). */
void s5d_plan_destroy(s5d_plan *plan);

/* The blocking parameters the plan uses (`chosen`, may be NULL) and the
 * size in bytes of one padded grid buffer (`bytes_per_buffer`, may be NULL). */
s5d_status s5d_plan_query(const s5d_plan *plan, s5d_tuning *chosen, int64_t *bytes_per_buffer);

/* Run the whole sweep of `plan` on device buffers.
 *   buf0: device pointer, padded grid in C order (dtype of the plan), holding
 *         the initial state including the boundary.
 *   buf1: device pointer, same size, distinct and not overlapping buf0; its
 *         contents are ignored.  The library first copies buf0's boundary
 *         cells into it.
 *   stream: a hipStream_t (NULL = the null stream).  Work is enqueued
 *         asynchronously; a kernel fault surfaces at the caller's next
 *         synchronisation with that stream.
 *   result_index: may be NULL; receives steps % 2, the buffer that holds the
 *         result once the stream has drained (steps = 0 enqueues nothing and
 *         leaves buf0 untouched).
 * The caller owns both buffers and must keep them alive until the stream has
 * drained.  Errors are detected before anything is enqueued (S5D_EINVAL),
 * except launch failures (S5D_EDEVICE), which may leave a partial sweep. */
s5d_status s5d_run(const s5d_plan *plan, void *buf0, void *buf1, void *stream,
                   int32_t *result_index);

/* s5d_run for plans whose weights vary from cell to cell (S5D_EXPR_VARCOEF),
 * which s5d_run rejects (S5D_EINVAL).
 *   fields: device pointer, n_points arrays of the interior's extents
 *           (I0 x I1, C order, the plan's dtype), weight k of every cell
 *           first: fields[k * I0 * I1 + q] is the weight of offset k (canonical
 *           order) for the interior cell with 0-based interior index q.  Read
 *           by every round; the caller keeps it allocated and unchanged until
 *           the stream has drained.
 * Everything else is as for s5d_run.  fields must be NULL for other plans. */
s5d_status s5d_run_fields(const s5d_plan *plan, void *buf0, void *buf1, const void *fields, void *stream,
                          int32_t *result_index);

/* ---- Performance model and autotuner ----
 *
 * The model follows AN5D's "Performance Model": per launch, count the vector
 * ALU work, the HBM traffic and the LDS traffic of every wave (all lanes
 * compute every fused level; lanes outside the grid move no data; LDS carries
 * the 3D edge-row exchange), divide each by the device's rate (VALU 64
 * lane-operations per clock per CU in float32 and float64 alike, as the
 * kernels use no packed float32 instructions; HBM 6.0e12 B/s sustained, LDS
 * 128 B per clock per CU), take the largest and divide by the slot efficiency
 * 1 / (max(1, s/g) + 0.75 min(1, s/g)) for g workgroups and s resident slots
 * (an idle part of the machine when g < s, else a tail of about 0.75
 * workgroup durations as the last ones finish unevenly).  The whole sweep is
 * the sum over its rounds. */
typedef struct s5d_model {
    uint32_t struct_size; /* = sizeof(s5d_model) */
    int32_t bound;        /* largest term of the first round's kind: 0 ALU, 1 HBM, 2 LDS */
    double seconds;       /* predicted time of the whole sweep */
    double t_alu, t_hbm, t_lds; /* summed over rounds, before the slot efficiency */
    double eff_cu;        /* slot efficiency of the first (full-depth) round */
    double hbm_bytes;     /* predicted HBM traffic of the whole sweep */
    double valu_ops;      /* lane-operations of the whole sweep */
    int64_t workgroups;   /* workgroups of the first round */
} s5d_model;

s5d_status s5d_plan_model(const s5d_plan *plan, s5d_model *out);

typedef struct s5d_tune_report {
    uint32_t struct_size; /* = sizeof(s5d_tune_report) */
    int32_t n_candidates; /* configurations the model ranked */
    int32_t n_measured;   /* of which timed on the GPU */
    int32_t reserved;
    double model_best_seconds;       /* model time of its top-ranked candidate */
    double best_seconds_per_step;    /* measured time of the winner (-1 if none measured) */
    double default_seconds_per_step; /* measured time of the library's default choice */
} s5d_tune_report;

/* Choose the blocking (b_T, tile, cells per lane, rows per wave, stream block
 * length h_SN) for `desc` (AN5D "Performance Model" and "Tuning"): enumerate
 * every compiled variant of the stencil with a ladder of stream block
 * lengths, rank them by the model, time the best top_k on the GPU (two full
 * rounds each, on scratch buffers the tuner allocates and frees), and keep
 * the fastest, or the library's default if none beats it.  top_k = 0 trusts
 * the model alone.  The winner goes to *best and, unless it is the choice a
 * plan without tuning gets already, into the process-wide cache,
 * from which s5d_plan_create takes it whenever it is given no tuning for a
 * descriptor with the same stencil, dtype, accumulation and power-of-two
 * bucket of every extent.  Synchronous on `stream`. */
s5d_status s5d_autotune(const s5d_desc *desc, int32_t top_k, void *stream, s5d_tuning *best,
                        s5d_tune_report *report);

/* Write / merge / empty the tuning cache (a small text file, one entry per line).
 * The first s5d_plan_create of a process merges the autotuner's choices
 * measured on MI355X at the benchmark sizes into the cache: the file
 * tuning_gfx950.txt beside the library, or the file the environment variable
 * S5D_TUNING_FILE names (an empty value: none).  A missing or malformed file
 * leaves the library's built-in defaults in place. */
s5d_status s5d_tune_cache_save(const char *path);
s5d_status s5d_tune_cache_load(const char *path);
void s5d_tune_cache_clear(void);

/* ---- Batched execution of many independent sweeps ----
 *
 * Many grids of uneven sizes (each with its own plan: stencil, extents,
 * steps, blocking) advance together.  Each grid follows exactly the rounds
 * s5d_run would give it, so its result is bit-identical to running it alone;
 * at each round index the rounds of all grids that share a kernel variant
 * form ONE launch, whose workgroups are spread over the grids by a device
 * table built at creation.  Small grids thereby share the machine instead of
 * each under-filling it (AN5D "Execution Model": the thread blocks of a launch
 * are independent, whichever grid they belong to). */
typedef struct s5d_batch s5d_batch; /* opaque */

#define S5D_BATCH_GRAPH 1 /* flag: capture the whole sequence into a HIP graph on the
                             first run and replay it with one graph launch */
#define S5D_BATCH_PERSISTENT 2 /* flag: one persistent launch per stencil family
                             (element type, accumulation, shape, radius, cells
                             per lane) runs every round of that family's grids.
                             Its workgroups (at most as many as are resident at
                             once) take (grid, round, workgroup) items from a
                             device queue ordered by round index; a grid's round
                             k starts once every workgroup of its round k-1 has
                             finished, with no device-wide barrier between round
                             indices.  Results are bit for bit those of s5d_run.
                             2D blocked plans of the families the library
                             builds (plain float32 stars r <= 2 and 9-point
                             boxes, plain float64 stars r <= 2, default cells per
                             lane; b_T up to the family's deepest); any other
                             plan gives S5D_EUNSUPPORTED at creation.  A waiting
                             workgroup polls at most a bounded number of times
                             (s5d_batch_set_wait_limit); s5d_batch_status reports
                             a wait that ran out. */

/* Build a batch over n grids.  plans[i] (not retained: it may be destroyed
 * afterwards; the batch keeps a reference to whatever device state of the
 * plan its launches read, such as the coefficient table of a direct kernel),
 * buf0[i] and buf1[i] (device pointers, as for s5d_run) describe
 * grid i; the buffers are bound to the batch, must stay allocated while it
 * exists, and no two buffers of the batch may overlap.  The device tables are
 * allocated with hipMalloc on the current device and uploaded synchronously.
 * Errors: S5D_EINVAL (bad arguments, overlapping buffers), S5D_EUNSUPPORTED,
 * S5D_ENOMEM, S5D_EDEVICE.  n = 0 gives a batch that does nothing. */
s5d_status s5d_batch_create(const s5d_plan *const *plans, void *const *buf0, void *const *buf1,
                            int32_t n, int32_t flags, s5d_batch **out);

/* Enqueue every grid's whole sweep on `stream` (a hipStream_t of the batch's
 * device; NULL = null stream).  As for s5d_run, buf0[i] must hold grid i's
 * initial state and result_index (n entries, may be NULL) receives
 * steps_i % 2.  Asynchronous; a batch may be run again once its inputs have
 * been reset.  Runs of one batch on different streams must not overlap. */
s5d_status s5d_batch_run(s5d_batch *batch, void *stream, int32_t *result_index);

/* Launches per run (the one boundary-copy launch that covers every grid
 * included) and the number of round indices (may be NULL). */
s5d_status s5d_batch_query(const s5d_batch *batch, int32_t *n_launches, int32_t *n_round_steps);

/* Persistent batches: the number of persistent launches (stencil families),
 * and their workgroups and work items summed over the launches (each may be
 * NULL; all 0 for other batches).  Errors: S5D_EINVAL (NULL batch). */
s5d_status s5d_batch_persistent_info(const s5d_batch *batch, int32_t *n_launches, int64_t *workgroups,
                                     int64_t *items);

/* Persistent batches (S5D_BATCH_PERSISTENT): synchronise `stream` (the
 * stream of the last run), then read the launches' status.  S5D_OK if every
 * dependency wait of the last run was satisfied, S5D_ETIMEDOUT if a wait ran
 * out of polls (the run stopped early and its results are incomplete; the
 * batch may be run again), S5D_EDEVICE if the synchronisation failed.  For
 * other batches, S5D_OK after the synchronisation. */
s5d_status s5d_batch_status(s5d_batch *batch, void *stream);

/* Persistent batches: the most polls (each about a microsecond) a workgroup
 * spends waiting for its grid's previous round before it gives up and the run
 * stops with S5D_ETIMEDOUT.  polls >= 0; the default, 2^24, is seconds, far
 * above any legitimate wait.  Takes effect at the next run (a captured graph
 * is captured again).  Errors: S5D_EINVAL (NULL batch, polls < 0). */
s5d_status s5d_batch_set_wait_limit(s5d_batch *batch, int64_t polls);

/* Wait for the device to drain, then release the batch (NULL accepted). */
void s5d_batch_destroy(s5d_batch *batch);

/* Create, run on `stream`, synchronise that stream and destroy: a batched
 * s5d_run for one-off use.  Synchronous. */
s5d_status s5d_run_batch(const s5d_plan *const *plans, void *const *buf0, void *const *buf1,
                         int32_t n, void *stream, int32_t *result_index);

/* ---- Serving loop: continuous batching of sweep requests ----
 *
 * A server owns HIP streams and the device memory of the grids it holds.
 * Requests (a plan and an initial grid) queue in arrival order.  Each call of
 * s5d_server_tick
 *   1. drops the running requests that were cancelled (FAILED, S5D_ECANCELED);
 *   2. admits queued requests in FIFO order while the two buffers of the next
 *      one fit the HBM budget (and max_running allows it): stream-ordered
 *      allocation, copy of the initial grid, boundary copy.  A request whose
 *      admission fails becomes FAILED and admission goes on with the next;
 *   3. advances every running request by one round of its own schedule, all
 *      of them in one batched launch per kernel variant (the variants of one
 *      round spread over n_streams streams), so new arrivals join at round
 *      boundaries and every result is bit-identical to the request run alone
 *      with s5d_run.  A request's round counts as done only once its launch
 *      has been enqueued: if a launch cannot be enqueued, requests with a
 *      round in it become FAILED and the others are unaffected (if nothing of
 *      the tick was enqueued, no request moves and the tick may be retried);
 *   4. records when requests whose last round was just enqueued complete
 *      (GPU clock, on the server's time axis).
 * At most three ticks are in flight: a tick waits for the tick three before
 * it.  Times are seconds since s5d_server_create on the host's steady clock.
 * A server is not thread-safe: calls on one server must not overlap. */
typedef struct s5d_server s5d_server; /* opaque */

typedef struct s5d_server_config {
    uint32_t struct_size;     /* = sizeof(s5d_server_config) */
    int32_t max_running;      /* requests running at once; 0 = no limit */
    int64_t hbm_budget_bytes; /* device memory for the grids of admitted requests */
    int32_t rounds_per_tick;  /* rounds of each running request per tick; 0 = adaptive:
                                 ceil(8 / running), at most 16, so that a tick carries
                                 enough launches while few requests run */
    int32_t n_streams;        /* streams the launches of one round spread over, 1..4;
                                 0 = 4 */
    int32_t fail_admit_every; /* testing: k > 0 makes every k-th admission fail as if
                                 its allocation had failed; 0 = off */
    int32_t fail_tick_every;  /* testing: k > 0 makes the launch of the last round of
                                 every k-th tick with work fail before it is enqueued;
                                 0 = off */
} s5d_server_config;

/* Request states. */
#define S5D_REQ_QUEUED 0
#define S5D_REQ_RUNNING 1
#define S5D_REQ_DONE 2     /* finished; result held if it was kept */
#define S5D_REQ_RELEASED 3 /* result fetched, memory returned */
#define S5D_REQ_FAILED 4   /* will not finish (status says why); memory returned */

typedef struct s5d_request_info {
    uint32_t struct_size; /* = sizeof(s5d_request_info) */
    int32_t state;        /* S5D_REQ_* */
    int32_t result_index; /* steps % 2 */
    int32_t status;       /* S5D_OK, or why a FAILED request failed */
    int64_t updates;      /* interior cells x steps */
    int64_t rounds_done;  /* rounds enqueued so far */
    double t_arrival, t_admit, t_done; /* seconds; -1 if not yet */
    int32_t init_in_use;  /* 1 while the server may still read the request's init */
    int32_t reserved;
} s5d_request_info;

typedef struct s5d_server_stats {
    uint32_t struct_size; /* = sizeof(s5d_server_stats) */
    int32_t reserved;
    int64_t submitted, queued, running, done, failed;
    int64_t bytes_in_use, bytes_peak; /* grid memory held (both buffers per request) */
    int64_t ticks, launches;          /* ticks with work, batched launches they made */
    int64_t updates_done;             /* cell updates of the finished requests */
    double latency_p50, latency_p99;  /* t_done - t_arrival over finished requests, nearest rank */
    double makespan;                  /* last completion - first arrival */
} s5d_server_stats;

/* Create a server on the current device.  Errors: S5D_EINVAL, S5D_ENOMEM,
 * S5D_EDEVICE. */
s5d_status s5d_server_create(const s5d_server_config *config, s5d_server **out);

/* Wait for the server's stream, free everything it holds (NULL accepted). */
void s5d_server_destroy(s5d_server *server);

/* The server clock: seconds since creation. */
s5d_status s5d_server_now(const s5d_server *server, double *seconds);

/* Queue a request.  The plan is copied (the caller may destroy it).  `init`
 * (host or device memory, plan's padded grid, boundary included) is read on
 * the server's stream after the request is admitted, so it must stay valid
 * and unchanged until s5d_server_request reports init_in_use = 0 (or the
 * request is FAILED).  S5D_EUNSUPPORTED if a round of the plan has no batched
 * kernel.  `arrival` stamps the request on the server clock
 * (negative: now).  With keep_result != 0 the result stays on the device until
 * s5d_server_fetch; otherwise it is dropped when the request completes.
 * S5D_EBUDGET if the request alone exceeds the budget. */
s5d_status s5d_server_submit(s5d_server *server, const s5d_plan *plan, const void *init,
                             double arrival, int32_t keep_result, int64_t *id);

/* One tick (see above; with rounds_per_tick != 1, step 2 repeats).  n_running / n_queued (may be NULL) receive the
 * counts after it.  n_running = 0 with n_queued > 0 means the next queued
 * request does not fit beside the kept results: it waits until they are
 * fetched. */
s5d_status s5d_server_tick(s5d_server *server, int32_t *n_running, int32_t *n_queued);

/* Cancel a request: a queued one becomes FAILED at once, a running one at the
 * start of the next tick (its buffers are freed after the work already
 * enqueued for it); finished requests are left as they are.  Status
 * S5D_ECANCELED is recorded for it. */
s5d_status s5d_server_cancel(s5d_server *server, int64_t id);

/* Wait for all enqueued work and record the completions. */
s5d_status s5d_server_sync(s5d_server *server);

/* State and timestamps of one request. */
s5d_status s5d_server_request(const s5d_server *server, int64_t id, s5d_request_info *info);

/* Copy a finished, kept result into `dst` (host or device memory, one padded
 * grid) and release the request's buffers.  Synchronous. */
s5d_status s5d_server_fetch(s5d_server *server, int64_t id, void *dst);

/* Counters, latency percentiles and makespan. */
s5d_status s5d_server_get_stats(const s5d_server *server, s5d_server_stats *out);

/* Error and norm reductions in float64 between a computed grid and a
 * reference, for checking a sweep against an independent result on the GPU
 * (the relative error measure of the accuracy evaluation).  Over the n
 * elements g = got[i], o = ref[i], with d = |g - o| formed in float64, `out`
 * receives S5D_NORMS_COUNT doubles:
 *   out[0] = max d,   out[1] = max |o|,
 *   out[2] = max (d / |o|), taking d itself where o = 0,
 *   out[3] = sqrt(sum d^2 / n),   out[4] = sqrt(sum o^2 / n).
 * A NaN in g or o propagates into out[0], out[2] and out[3].  n = 0 gives zeros.
 *   got, ref: device pointers, n elements of got_dtype / ref_dtype (S5D_F32 or
 *             S5D_F64), 16-byte aligned (any torch allocation is).
 *   out: device pointer, S5D_NORMS_COUNT doubles, 8-byte aligned; every value
 *        is written, so it needs no clearing.
 *   workspace: device memory of at least s5d_error_norms_workspace_bytes(n)
 *        bytes (at most 80 KiB), not overlapping out; the caller owns it and
 *        must not reuse it before the stream has passed this call.
 * Asynchronous on `stream` (a hipStream_t; NULL = null stream); two kernel
 * launches, no allocation and no host synchronisation, so the call may be
 * captured in a HIP graph.  The result is a deterministic function of the
 * inputs and n.  Errors: S5D_EINVAL before anything is enqueued,
 * S5D_EDEVICE if a launch fails. */
#define S5D_NORMS_COUNT 5
int64_t s5d_error_norms_workspace_bytes(int64_t n); /* -1 if n < 0 */
s5d_status s5d_error_norms(const void *got, int32_t got_dtype, const void *ref, int32_t ref_dtype,
                           int64_t n, double *out, void *workspace, int64_t workspace_bytes,
                           void *stream);

/* s5d_error_norms without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same inputs, outputs, results (bit for
 * bit) and errors as s5d_error_norms, except:
 *   - the first-pass partials go to a fixed scratch array in device memory
 *     that the library holds for each GPU until the process ends
 *     (2048 x 5 doubles = 80 KiB; the first pass never uses more than 2048
 *     workgroups, so every n >= 0 fits; a larger need would be rejected
 *     with S5D_EINVAL);
 *   - the scratch of the current device is used, and a non-NULL `stream`
 *     must belong to that device (S5D_EINVAL otherwise);
 *   - no call allocates or frees memory; the scratch keeps the last call's
 *     partials, and every value the final pass reads is written by the same
 *     call first, so nothing needs clearing.
 * Calls that overlap on one GPU (on different streams, or from several
 * threads without ordering) share that scratch and race: order them on one
 * stream, or use s5d_error_norms with a workspace of their own. */
s5d_status s5d_error_norms_noalloc(const void *got, int32_t got_dtype, const void *ref, int32_t ref_dtype,
                                   int64_t n, double *out, void *stream);

/* Human-readable name of a status code (static storage). */
const char *s5d_status_string(s5d_status status);

/* Detail of the last error raised on the calling thread ("" if none). */
const char *s5d_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL5D_H */
