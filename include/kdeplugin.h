/*
 * libkdeplugin — PLUGIN bandwidth selection for univariate Gaussian kernel
 * density estimation on AMD Instinct MI355X (gfx950).
 *
 * The method is the two-stage plug-in selector of Section 3, Algorithm 1 of
 * Gramacki, Sawerwain and Gramacki, "FPGA-Based Bandwidth Selection for Kernel
 * Density Estimation Using High Level Synthesis Approach" (arXiv:1505.02100):
 *
 *   Step I    V = sum (X_i - mean)^2 / (n - 1),  sigma = sqrt(V)
 *   Step II   Psi8 = 105 / (32 sqrt(pi) sigma^9)
 *   Step III  g1 = (-2 K6(0) / (mu2 Psi8 n))^(1/9),      K6(0) = -15/sqrt(2 pi)
 *   Step IV   Psi6(g1) = (n^2 g1^7)^-1 sum_i sum_j K6((X_i - X_j)/g1)
 *   Step V    g2 = (-2 K4(0) / (mu2 Psi6 n))^(1/7),      K4(0) = 3/sqrt(2 pi)
 *   Step VI   Psi4(g2) = (n^2 g2^5)^-1 sum_i sum_j K4((X_i - X_j)/g2)
 *   Step VII  h = (R(K) / (mu2^2 Psi4 n))^(1/5),         R(K) = 1/(2 sqrt(pi)), mu2 = 1
 *
 * with K6(x) = (x^6 - 15x^4 + 45x^2 - 15) phi(x), K4(x) = (x^4 - 6x^2 + 3) phi(x)
 * and phi the standard normal density (equation (2)).  The double sums are
 * evaluated in the symmetric form of equations (6)-(7): twice the strict upper
 * triangle i < j plus the diagonal n K(0), which is added analytically.
 *
 * Conventions for every entry point:
 *  - Integer return values: KDE_OK (0) on success, a negative KDE_E* code on
 *    failure.  Functions returning double return NaN on failure.  In both
 *    cases kde_last_error() / kde_last_error_message() hold the reason
 *    (thread-local).  No C++ exception crosses this interface.
 *  - The caller owns every input and output buffer.  The library never keeps
 *    a pointer to caller data after a synchronous call returns.
 *  - Samples x are contiguous arrays of n values.  KDE_MEM_HOST means an
 *    ordinary host pointer; KDE_MEM_DEVICE means a pointer to memory on the
 *    context's GPU (for example a torch tensor's data_ptr()).
 *  - A kde_stream is a hipStream_t passed as void*; NULL is the null stream.
 *  - Every call on a context is synchronous with respect to the host unless
 *    its comment says otherwise (kde_plugin_bandwidth_batch on device
 *    samples and device-accessible results); work is enqueued on the given
 *    stream and the call waits for that work before returning.
 *  - A context is not thread-safe: use one context per host thread.  The
 *    literal calls kde_psi() and kde_plugin_bandwidth() use a process-wide
 *    default context guarded by a mutex.
 *  - Results are deterministic: the same samples give bitwise-identical
 *    results on every call, alone or inside any batch, for a given context
 *    configuration (precision and tile shape).
 */
#ifndef KDEPLUGIN_H
#define KDEPLUGIN_H

#include <stdint.h>

#if defined(__GNUC__)
#define KDE_API __attribute__((visibility("default")))
#else
#define KDE_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define KDE_OK 0
#define KDE_EINVAL (-1)      /* null pointer, n < 2 (Step I divides by n-1), r not in {4,6},
                                g not finite and positive, bad enum value               */
#define KDE_ENONFINITE (-2)  /* NaN or Inf among the samples (or their sum overflows)     */
#define KDE_EDEGENERATE (-3) /* sigma = 0 (constant sample: Psi8 of Step II is infinite),
                                or Psi6 >= 0 / Psi4 <= 0, which exact arithmetic excludes
                                (Psi6 < 0 < Psi4 for every sample), i.e. numerical failure */
#define KDE_ENOMEM (-4)      /* device or host allocation failed, or over memory budget   */
#define KDE_EDEVICE (-5)     /* HIP runtime error; the message names the call             */
#define KDE_ETIMEOUT (-6)    /* an in-kernel wait for a previous stage exceeded its limit */
#define KDE_EBUSY (-7)       /* server: request not finished yet / queue full             */

/* ------------------------------------------------------------------ enums */
#define KDE_FP64_PLAIN 0 /* pair sums in FP64 with the printed polynomials and FP64 exp      */
#define KDE_FP32_COMP 1 /* the production precision: pair terms in FP32 (exp2 on the
                           transcendental unit, Hermite factors in y^2 with exact integer
                           coefficients) with error-compensated per-thread sums.  The
                           compensation is blocking, not Kahan's algorithm: each FP32
                           accumulator takes at most 4 terms, four of them are added
                           pairwise in FP32 (16 terms) and the result is folded into an
                           FP64 lane sum, so the FP32 rounding error of a partial stays
                           that of 16 terms whatever n is (Kahan's update would cost 3
                           more VALU operations per pair, the fold 0.3).  Moments,
                           cross-block sums (exact, in fixed point) and Steps I-III, V,
                           VII in FP64.  The one systematic error left by construction
                           is the FP32 rounding of log2(e)/2 (relative 1.3e-8) in the
                           exponent                                                      */
#define KDE_FP32_COMP_EXACT 2 /* as KDE_FP32_COMP with log2(e)/2 carried as two FP32
                                 terms (one more VALU op per pair)                       */
#define KDE_FP32_POLYEXP 3 /* as KDE_FP32_COMP with 2^t evaluated by a degree-6 minimax
                              polynomial (Remez exchange, FP32 coefficients, relative
                              error 1.6e-8) on the FMA pipes instead of the
                              transcendental unit, after t = n + f, n = round(t)      */
#define KDE_Q32_32 4 /* the FPGA design's arithmetic (Section 4.2), emulated: z-scored
                        samples and the pair-stage quantities in Q32.32 fixed point
                        (truncating products, exact sums), the Gaussian factor from a
                        degree-7 minimax polynomial in Q32.32; moments, cross-item sums
                        and Steps I-III, V, VII in FP64.  Integer VALU work: slow, for
                        studying the fixed-point design's accuracy                    */

#define KDE_MEM_HOST 0
#define KDE_MEM_DEVICE 1

#define KDE_F64 0
#define KDE_F32 1

typedef struct kde_ctx kde_ctx;
typedef void* kde_stream;

typedef struct {
    int32_t device;     /* HIP device ordinal (default 0)                                  */
    int32_t precision;  /* KDE_FP64_PLAIN (default), KDE_FP32_COMP, KDE_FP32_COMP_EXACT,
                           KDE_FP32_POLYEXP or KDE_Q32_32                                 */
    int64_t mem_budget; /* bytes of device workspace this context may hold; 0 = no limit    */
    const char* tune_table; /* path of an autotune table written by kde_autotune, or NULL
                               for the built-in tile configuration                          */
    int32_t rows_per_lane;   /* 0 = from the tune table / default; else 1, 2 or 4          */
    int32_t blocks_per_cu;   /* 0 = from the tune table / occupancy (and, with neither
                                set, launches at KDE_FP32_COMP and one row per lane whose
                                pair stage holds 2^34 pairs or more -- one sample of about
                                185 000 or more, or a large batch -- run on a kernel built
                                for four waves per SIMD, with four blocks per CU); else
                                1..16 on the three-wave kernel                              */
    int32_t target_items;    /* 0 = default; pair work items per stage for large n         */
    int32_t wait_limit_us;   /* 0 = default; else the longest an in-kernel wait for an
                                earlier stage may take, in microseconds, before the sample
                                fails with KDE_ETIMEOUT.  The default is 20 s plus the time
                                of the launch's largest work item at a rate far below any
                                measured one (so huge samples are never cut off)           */
    int64_t pair_budget;     /* 0 = default; else pair items of about this many pairs for
                                every n (overrides target_items and the tune table)         */
} kde_options;

/* The outputs of Algorithm 1 for one sample.  psi6/psi4 are the estimates of
 * Steps IV and VI; psi8 is Step II's normal-scale estimate. */
typedef struct {
    double h;       /* Step VII bandwidth (for kde_psi_ex-style calls: NaN)            */
    double mean;    /* sample mean                                                      */
    double sigma;   /* Step I standard deviation (divisor n - 1)                        */
    double psi8;    /* Step II                                                          */
    double g1;      /* Step III                                                         */
    double psi6;    /* Step IV                                                          */
    double g2;      /* Step V                                                           */
    double psi4;    /* Step VI                                                          */
    int32_t status; /* KDE_OK or the KDE_E* code for this sample                        */
    int32_t reserved;
} kde_result;

/* -------------------------------------------------------------- utilities */
KDE_API const char* kde_version(void);
KDE_API int kde_last_error(void);                  /* last status set on this thread */
KDE_API const char* kde_last_error_message(void);  /* human-readable detail for it   */
KDE_API const char* kde_strerror(int code);

/* Fill *opt with the defaults listed above. */
KDE_API void kde_options_init(kde_options* opt);

/* Create a context on opt->device (opt may be NULL for defaults).  The
 * context owns its device workspace (work lists, per-item partial sums,
 * per-sample state), cached hipGraphs and the tile configuration. */
KDE_API int kde_ctx_create(kde_ctx** out, const kde_options* opt);
KDE_API void kde_ctx_destroy(kde_ctx* ctx);

/* Tile configuration actually in use: rows per lane, threads per block,
 * rows per tile, persistent blocks per CU. */
KDE_API int kde_ctx_config(const kde_ctx* ctx, int32_t* rows_per_lane, int32_t* block_threads,
                   int32_t* tile_rows, int32_t* blocks_per_cu);

/* Device time in milliseconds of the last synchronous call's launch on this
 * context (persistent kernel and the few-hundred-byte state read-back,
 * replayed as one graph; the reset of the states for the next call follows
 * it), measured with HIP events on the caller's stream; -1 if none yet. */
KDE_API double kde_ctx_last_device_ms(const kde_ctx* ctx);

/* Launch shape of the persistent kernel of the last call on this context
 * (single, batch or no-allocation): its blocks (256 threads each) and the waves per SIMD the kernel is
 * built for (3, or 4 for the default precision at R = 1 on launches whose
 * pair stage holds 2^34 pairs or more, when the context chose its own tile
 * configuration).
 * KDE_EINVAL if the context has launched nothing yet. */
KDE_API int kde_ctx_last_launch(const kde_ctx* ctx, int32_t* blocks, int32_t* waves_per_simd);

/* Device timeline of sample `sample` of the last synchronous call on this
 * context: ms[k] (k < KDE_NUM_STAGES; the caller provides that many) =
 * milliseconds from the start of the sample's first work item to the moment
 * stage k published its result (k = 0: mean, 1: sigma and g1 (Steps I-III;
 * Step I takes one pass, so entries 0 and 1 are equal), 2: Psi6 and g2
 * (Steps IV-V), 3: Psi4 and h (Steps VI-VII)); -1 for a stage that did not
 * run.  From the GPU's 100 MHz clock. */
#define KDE_NUM_STAGES 4
KDE_API int kde_ctx_last_timeline(const kde_ctx* ctx, int64_t sample, double* ms);

/* ------------------------------------------------------- literal calls */

/* Psi_r(g) of equations (6)-(7) (Steps IV/VI with a caller-chosen g) for
 * r in {4, 6}: host pointer x[0..n), n >= 1, g > 0.  Any finite sample is
 * valid: n = 1 gives K^(r)(0) / g^(r+1), and ties are ordinary K^(r)(0) terms
 * (Step I only centres the data here, so a sample without spread is no
 * error).  Synchronous, FP64 plain, default context.  Returns NaN on error
 * (null x, n < 1, r not in {4, 6}, g not finite and positive, NaN or Inf in
 * x). */
KDE_API double kde_psi(const double* x, int64_t n, int r, double g);

/* h of Algorithm 1 (Steps I-VII) for host samples x[0..n), n >= 2.
 * Synchronous, FP64 plain, default context.  Returns NaN on error. */
KDE_API double kde_plugin_bandwidth(const double* x, int64_t n);

/* --------------------------------------------------------- context calls */

/* Psi_r(g) of equations (6)-(7) for samples x[0..n), n >= 1 (as kde_psi),
 * r in {4, 6}, g > 0, with x in host or device memory (mem_kind
 * KDE_MEM_HOST/DEVICE) as FP64 or FP32 values (dtype KDE_F64/F32), in the
 * context's precision.  *out receives the value.  Errors as kde_psi, plus
 * KDE_ENOMEM / KDE_EDEVICE.  Synchronous. */
KDE_API int kde_psi_ex(kde_ctx* ctx, const void* x, int64_t n, int r, double g, int mem_kind,
               int dtype, kde_stream stream, double* out);

/* Algorithm 1 for one sample; *out receives every intermediate.  The result's
 * status field repeats the return code.  Synchronous. */
KDE_API int kde_plugin_bandwidth_ex(kde_ctx* ctx, const void* x, int64_t n, int mem_kind, int dtype,
                            kde_stream stream, kde_result* out);

/* Algorithm 1 for count independent samples xs[k][0..ns[k]) (all host or all
 * device pointers, FP64), in ONE launch of the persistent kernel (replayed
 * from a cached hipGraph when the same batch is seen again).  out[k] is
 * filled for every k; the return value is KDE_OK when the launch itself
 * succeeded, and per-sample failures are reported in out[k].status.  Each
 * out[k] is bitwise identical to what kde_plugin_bandwidth_ex returns for the
 * same sample on the same context.
 *
 * Asynchronous when the samples are device memory (mem_kind KDE_MEM_DEVICE)
 * and out is device-accessible (memory on the context's GPU, or pinned host
 * memory from hipHostMalloc): the call enqueues the launch and the writing
 * of out[0..count) on `stream` and returns; the caller synchronizes the
 * stream before reading out, and keeps xs[k] and out alive until then.  A
 * later call on the same context (any stream) is ordered after this one's
 * use of the shared work list where it needs to be, so calls on several
 * streams may be in flight at once.  Otherwise (host samples, or out in
 * ordinary pageable host memory) the call returns when out is filled. */
KDE_API int kde_plugin_bandwidth_batch(kde_ctx* ctx, const void* const* xs, const int64_t* ns,
                               int64_t count, int mem_kind, kde_result* out, kde_stream stream);

/* --------------------------------------------------- no-allocation variant */

/* kde_plugin_bandwidth_ex for callers that cannot allocate memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It calls no hipMalloc, hipFree, hipHostMalloc or other allocating routine
 * and no host synchronization; it only enqueues kernels on `stream`.
 *   x, n, dtype: the sample, n >= 2, FP64 or FP32 (KDE_F64/KDE_F32), in device
 *     memory on the context's GPU.
 *   out: one kde_result in device-accessible memory (device memory on the
 *     context's GPU, or pinned host memory from hipHostMalloc), written on
 *     the stream.  Per-sample failures (KDE_ENONFINITE, KDE_EDEGENERATE,
 *     KDE_ETIMEOUT) are reported in out->status, with out->h = NaN.
 *   Asynchronous: the call returns once the work is enqueued; the caller
 *   synchronizes the stream before reading out, and keeps x and out alive
 *   until then.  The result is bitwise what kde_plugin_bandwidth_ex returns
 *   for the same sample on the same context.  kde_ctx_last_device_ms and the
 *   timeline are not updated.  The persistent kernel is always the
 *   three-wave build, which uses no scratch (private) memory, so the launch
 *   never makes the HIP runtime grow its scratch pool.
 *   Scratch: the work list, per-item partial sums, state and ticket live in a
 *   static device array of KDE_NOALLOC_SCRATCH_BYTES (about 13 MiB) that each
 *   GPU the library runs on holds once until the process ends; its address is
 *   taken when the first context is created on the device.  Every call on a
 *   GPU (from any context or thread) uses that one array, so calls whose work
 *   overlaps on one GPU race: order them on one stream, or synchronize between
 *   them.  Each call clears what must start at zero before it runs.
 *   Limit: the work list of the sample (Step I chunks plus the pair items of
 *   Steps IV and VI for the context's tile configuration) must fit in
 *   KDE_NOALLOC_MAX_ITEMS items; the default configuration needs at most
 *   about 209000 for any n.
 *   Errors (returned, nothing enqueued): KDE_EINVAL (null pointer, n < 2,
 *   bad dtype, x not device memory of the context's GPU, out not
 *   device-accessible, work list over the limit), KDE_EDEVICE (a launch
 *   failed, or the scratch is not set up on the device). */
#define KDE_NOALLOC_MAX_ITEMS 262144
#define KDE_NOALLOC_SCRATCH_BYTES 13634816
KDE_API int kde_plugin_bandwidth_noalloc(kde_ctx* ctx, const void* x, int64_t n, int dtype,
                                         kde_stream stream, kde_result* out);

/* ---------------------------------------------- work decomposition / shards */

/* Number of pair work items of one Psi stage for a sample of size n on this
 * context (the decomposition depends on n and the tile configuration only). */
KDE_API int64_t kde_psi_num_items(const kde_ctx* ctx, int64_t n);

/* Rectangle of the pair matrix covered by pair item `item`: rows [r0, r1),
 * columns [c0, c1), of which only the pairs with column > row are summed. */
KDE_API int kde_psi_item_geometry(const kde_ctx* ctx, int64_t n, int64_t item, int64_t* r0,
                          int64_t* r1, int64_t* c0, int64_t* c1);

/* Partial sum of one Psi stage over the contiguous pair items
 * [item_begin, item_end):  *partial = sum over those items' pairs i < j of
 * K^(r)((x_i - x_j)/g), in the context's precision; each item's FP64 partial
 * is added exactly in 128-bit fixed point with a resolution of 2^-64 (so the
 * total does not depend on the order of the items, and a partial is exact to
 * within 2^-64 per item on top of the items' own rounding).
 * This is one shard of Step IV/VI: the shards of a partition of
 * [0, kde_psi_num_items) add up to the full strict-upper-triangle sum.
 * Synchronous. */
KDE_API int kde_psi_range(kde_ctx* ctx, const void* x, int64_t n, int r, double g, int mem_kind,
                  int dtype, int64_t item_begin, int64_t item_end, kde_stream stream,
                  double* partial);

/* ------------------------------------------------------ density evaluation */

/* The kernel density estimate of equation (1) with the Gaussian kernel of
 * equation (2), for a bandwidth h (for example the one kde_plugin_bandwidth
 * selected):
 *     out[k] = (n h)^-1 sum_i phi((y[k] - x[i]) / h),    k = 0 .. m-1,
 * on a grid of points or at the samples themselves.
 *   x, n, mem_kind, dtype: the n >= 1 samples, as for the other calls.
 *   y, m: m >= 0 evaluation points (FP64); out: m FP64 results.  y and out
 *     are both host memory (y_mem_kind = KDE_MEM_HOST) or both device memory
 *     on the context's GPU (KDE_MEM_DEVICE).
 *   Precision from the context: KDE_FP64_PLAIN evaluates the definition in
 *     FP64.  The FP32 precisions take runs of 32 consecutive points: where
 *     they are evenly spaced (a grid with spacing up to about 0.3 h), a
 *     sample's 32 terms come from four exp2 and a geometric recurrence in
 *     FP32 (exponents formed in FP64), otherwise each term takes one exp2 of
 *     an FP32 exponent (centred per group of 64 points; groups spread over
 *     more than about 9 h take the differences in FP64); short FP32 sums are
 *     added in FP64: relative error per point below 1e-5.  Results are
 *     deterministic.
 *   Errors: KDE_EINVAL (null pointer, n < 1, m < 0, h not finite and
 *     positive, bad enum), KDE_ENONFINITE (NaN or Inf among x or y; out is
 *     then undefined), KDE_ENOMEM, KDE_EDEVICE.  Synchronous. */
KDE_API int kde_eval_ex(kde_ctx* ctx, const void* x, int64_t n, int mem_kind, int dtype, const double* y,
                        int64_t m, int y_mem_kind, double h, kde_stream stream, double* out);

/* kde_eval_ex on host arrays with the process-wide default context (FP64). */
KDE_API int kde_eval(const double* x, int64_t n, const double* y, int64_t m, double h, double* out);

/* ----------------------------------------------------------------- server */

/* A continuous-batching server: requests (one sample each) may be submitted
 * at any time; the server admits them (first come first served, or smallest
 * n first) into at most max_active slots against a device-memory budget,
 * keeps admitted samples resident on the device, and runs steps.  A step is
 * one launch of the persistent kernel over the next work items of the
 * active requests up to step_pairs pair evaluations, taken round-robin
 * (processor sharing, the default) or in priority order (KDE_FILL_PRIORITY),
 * so a request that arrives while others run joins at the next step and its
 * work overlaps theirs on the device.  Each result is
 * bitwise what kde_plugin_bandwidth_ex returns for the same sample on the
 * same context.  Steps are queued two deep on the server's own stream.
 * A server uses its context exclusively; neither is thread-safe. */
#define KDE_SERVE_FCFS 0
#define KDE_SERVE_SJF 1
/* How a step's pair budget is shared among the active requests: */
#define KDE_FILL_SHARE 0    /* round-robin, one pair item per request per turn (processor sharing) */
#define KDE_FILL_PRIORITY 1 /* in admission-key order (FCFS: oldest first; SJF: fewest remaining
                               pair evaluations first, with the same aging), each request taking
                               all it can before the next: finishes requests instead of spreading
                               the device over all of them                                       */

typedef struct kde_server kde_server;

typedef struct {
    int64_t mem_budget;  /* device bytes of admitted requests: their samples (copied in, or
                            left in caller device memory) and partial sums (default 8 GiB)    */
    int64_t step_pairs;  /* pair evaluations per step across all requests (default 2^34)     */
    int32_t max_active;  /* requests on the device at once (default 64)                       */
    int32_t policy;      /* KDE_SERVE_FCFS (default) or KDE_SERVE_SJF admission order         */
    int64_t aging_ms;    /* KDE_SERVE_SJF: a queued request's key is log2 of its pair count
                            minus one per aging_ms of waiting, so large requests overtake newer
                            small ones instead of starving; 0 = pure smallest first (default)  */
    int32_t fill;        /* KDE_FILL_SHARE (default) or KDE_FILL_PRIORITY                     */
    int32_t reserved;
} kde_server_options;

typedef struct {
    int64_t id;          /* the id kde_server_submit returned                                 */
    int64_t n;
    kde_result result;   /* as kde_plugin_bandwidth_ex would return it                       */
    double t_submit_ms;  /* host steady clock (ms) at submission, admission, and at the step  */
    double t_admit_ms;   /* retirement that observed the result                               */
    double t_done_ms;
} kde_completion;

typedef struct {
    int32_t active, queued, inflight_steps;
    int32_t failed_steps;  /* steps that could not run (their requests completed with an error) */
    int64_t steps, arena_used, completed_unread;  /* arena_used: bytes counted against the budget */
    double pairs_done;   /* n(n-1) summed over completed requests                             */
    double pairs_issued; /* pair evaluations (i < j) of every item launched so far           */
} kde_server_stats;

KDE_API void kde_server_options_init(kde_server_options* opt);
/* Allocates the arena (mem_budget bytes) on ctx's device. */
KDE_API int kde_server_create(kde_server** out, kde_ctx* ctx, const kde_server_options* opt);
/* Waits for the server's stream, then frees everything it owns. */
KDE_API void kde_server_destroy(kde_server* srv);
/* Queue one FP64 sample x[0..n) (host or device memory).  Host samples are
 * copied to the device at admission, so x must stay valid until the request
 * is admitted (device samples: until it completes).  For a device sample,
 * `producer` is the stream whose work writes x (NULL: the null stream): the
 * server records an event there at submission and its own stream waits for
 * it before the first step that reads x, so the sample may still be in
 * flight when it is submitted (ignored for host samples).  *id identifies the
 * request.  KDE_ENOMEM if it could never fit the memory budget. */
KDE_API int kde_server_submit(kde_server* srv, const void* x, int64_t n, int mem_kind, kde_stream producer,
                              int64_t* id);
/* Remove a request that is still queued; KDE_EBUSY once admitted. */
KDE_API int kde_server_cancel(kde_server* srv, int64_t id);
/* Retire finished steps, admit queued requests, and launch the next step if
 * fewer than two are queued.  block != 0 waits when the device is the
 * bottleneck (two steps queued, or nothing new to launch).  stats may be NULL. */
KDE_API int kde_server_step(kde_server* srv, int32_t block, kde_server_stats* stats);
/* Move up to max finished requests into out[]; *got receives the count. */
KDE_API int kde_server_poll(kde_server* srv, kde_completion* out, int32_t max, int32_t* got);
/* Step until every submitted request has finished. */
KDE_API int kde_server_drain(kde_server* srv);

/* Failure handling.  A step that cannot run (its kernel launch fails) fails
 * the requests it lists: each completes with that status (h = NaN) once no
 * earlier step still in flight can write its memory, and its slot and memory
 * are freed; the other requests are unaffected and complete as usual.
 * (Per-request failures found on the device -- KDE_ENONFINITE,
 * KDE_EDEGENERATE, KDE_ETIMEOUT -- are reported in that request's result.)
 * kde_server_fail_next_step makes the next step that has work fail with
 * `code` (a negative KDE_E* value) without launching it, for tests of this
 * path; KDE_EINVAL for a non-negative code. */
KDE_API int kde_server_fail_next_step(kde_server* srv, int32_t code);

/* ------------------------------------------------------------- autotuner */

/* Search the tile configuration for opt->precision on opt->device (opt may
 * be NULL for the defaults): rows per lane R in {1, 2, 4} (tile height 256 R),
 * persistent blocks per CU (0 = the context's own choice, the occupancy
 * limit, one below it; table value 0 leaves the choice, including the
 * four-wave kernel for large samples, to the context) and the size of the
 * pair items.  Each candidate is timed with HIP events on the launch
 * stream (median of reps launches) on synthetic normal samples with the
 * sizes ns[0..count):
 *   mode KDE_TUNE_SINGLE: every size alone, one selection per launch; the
 *     (R, blocks per CU) with the least total time wins, with the best item
 *     count per size (table key "targets");
 *   mode KDE_TUNE_BATCH: all samples in one kde_plugin_bandwidth_batch
 *     launch; items are sized to a pair budget B (table key "pair_budget").
 * For KDE_FP32_COMP the search also times the other way to evaluate 2^t in
 * the pair terms, the Remez minimax polynomial on the FMA pipes (the kernels
 * of KDE_FP32_POLYEXP), and records the faster as "exp_poly" (0: v_exp_f32,
 * 1: the polynomial); a context created with such a table uses it.
 * The table is written to out_path as JSON and read back through
 * kde_options.tune_table.  R, the blocks per CU and the item sizes do not
 * change what is computed; the exponential's choice changes results at the
 * rounding level only (both within the FP32 bounds).  For a given table
 * results are deterministic.  verbose != 0 prints every timing to stderr.
 * Synchronous. */
#define KDE_TUNE_SINGLE 0
#define KDE_TUNE_BATCH 1
KDE_API int kde_autotune(const kde_options* opt, const int64_t* ns, int32_t count, int32_t mode,
                 int32_t reps, const char* out_path, int32_t verbose);

#ifdef __cplusplus
}
#endif

#endif /* KDEPLUGIN_H */
