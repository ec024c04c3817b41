/*
 * sketch.h -- C ABI of the MI355X (gfx950) matrix-sketch library.
 *
 * The library maintains Frequent-Directions (FD) sketches of row streams on
 * one GPU.  Each time a sketch's 2*ell-row buffer fills, it is shrunk: the
 * buffer is factorised, the ell-th largest squared singular value is
 * subtracted from every squared singular value (clamped at zero) and an
 * (ell-1)-row sketch is rebuilt (paper Sec. 2.3 "Frequent Directions";
 * the FD reduce of Algorithm "AeroSketch: Update").  With SK_SHRINK_RAND the exact
 * SVD is replaced by the randomized factorisation of Algorithm "Simultaneous
 * Iteration" (Sec. 2.2) applied to the buffer, with the Gaussian test matrix
 * on the d side (Omega, d x k) drawn from Philox4x64-10.
 *
 * Problem statements served (paper Sec. 2.1):
 *   - persistent stream sketch (SK_PERSISTENT): cov-error of the whole stream;
 *   - sliding window (SK_WINDOW): Algorithm "ML-AeroSketch", window of the
 *     last window_N rows;
 *   - at-the-time persistent sketch (SK_ATTP, Sec. 4.1): Algorithm "ATTP
 *     Sketch using AeroSketch", the sketch of any earlier prefix of the
 *     stream (sketch_query_at);
 *   - distributed streams: per-site sketches combined by sketch_merge
 *     (Lemma "Decomposability"), or tracked continuously by the protocol
 *     of Algorithm "P5" (SK_P5, Sec. 4.3): m simulated sites and their
 *     coordinator on one GPU (p5_update);
 *   - approximate matrix multiplication over a sliding window (SK_COD,
 *     Sec. 4.2): Algorithm "AeroSketchCOD Framework" on pairs (x_i, y_i)
 *     (cod_update, cod_query).
 *
 * Conventions (all entry points):
 *   - Matrices are row-major.  A row block is n_rows x d with leading
 *     dimension ld >= d (elements).
 *   - on_device != 0: the pointer is device memory of the sketch's GPU;
 *     otherwise host memory.  The caller owns every input and output buffer;
 *     the library owns all sketch state and scratch (allocated at create).
 *   - Work is ordered on the sketch's HIP stream.  sketch_update returns once
 *     the work is enqueued; device inputs must stay valid until sketch_sync,
 *     a query, or a later call on the same handle has returned.  Host inputs
 *     are copied before sketch_update returns.
 *   - sketch_query blocks until B_out holds the result.
 *   - Errors: no exception crosses the ABI.  On SK_EINVAL / SK_ESHAPE /
 *     SK_EUNSUPPORTED the sketch state is unchanged.  A failed HIP call or a
 *     non-converged eigen-solve makes the handle sticky-SK_EDEVICE.
 *     sketch_last_error() returns a thread-local message for the last
 *     failing call on the calling thread.
 *   - Threading: one handle must not be used by two threads at once;
 *     distinct handles are independent.
 *   - Query output: ell rows; B_out^T B_out is the sketch (rows in descending
 *     norm, signs arbitrary).  Compare B^T B, never B.
 */
#ifndef SKETCH_H
#define SKETCH_H
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SK_EXPORT __attribute__((visibility("default")))
#else
#define SK_EXPORT
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sketch_s* sketch_t; /* opaque, library-owned */

typedef enum {
    SK_OK = 0,
    SK_EINVAL = -1,       /* bad argument (NULL, negative size, ld < d, ...)   */
    SK_ENOMEM = -2,       /* device or host allocation failed / over budget     */
    SK_EDEVICE = -3,      /* HIP error or eigen-solver failure (sticky)         */
    SK_ESHAPE = -4,       /* shapes of two sketches do not match                */
    SK_EUNSUPPORTED = -5, /* operation not defined for this kind of sketch      */
    SK_ESTATE = -6        /* call out of order (e.g. time moving backwards)     */
} sk_status;

typedef enum { SK_F64 = 0, SK_F32 = 1, SK_BF16 = 2 } sk_dtype;
typedef enum { SK_PERSISTENT = 0, SK_WINDOW = 1, SK_ATTP = 2, SK_P5 = 3, SK_COD = 4 } sk_kind;
typedef enum { SK_SHRINK_EXACT = 0, SK_SHRINK_RAND = 1 } sk_shrink;

typedef struct {
    int32_t d;            /* row dimension, >= 1                                  */
    int32_t ell;          /* sketch rows (buffer holds 2*ell), >= 2              */
    int32_t kind;         /* sk_kind                                             */
    int32_t shrink;       /* sk_shrink (persistent sketches)                     */
    int32_t state_dtype;  /* SK_F64 or SK_F32: dtype of the resident buffer      */
    int32_t proj_dtype;   /* SK_F64, SK_F32 or SK_BF16: dtype of C*Omega inputs  */
    int32_t q;            /* power steps of simul_iter (>= 0)                    */
    int32_t oversample;   /* k = min(ell + oversample, 2*ell, d)                 */
    int64_t window_N;     /* SK_WINDOW: window length in rows                    */
    double R;             /* SK_WINDOW: bound on squared row norms (>= 1)        */
    uint64_t seed;        /* Philox key word 0                                   */
    uint64_t stream_id;   /* Philox key word 1                                   */
    int32_t device;       /* HIP device ordinal                                  */
    int32_t use_given_stream; /* 1: order work on hip_stream even when it is NULL
                                 (the default stream); 0: NULL means a stream
                                 owned by the library                           */
    void* hip_stream;     /* hipStream_t to order work on                        */
    /* SK_WINDOW, SK_ATTP and SK_P5: probability amplification of the dump step
     * (Algorithm "Probability Amplification", analysed in the appendix on the
     * amplified estimation).  Every doubling step of a dump runs amplify_r
     * simul_iter candidates (candidate h draws its test matrix from counter
     * word 3 = 0x200 + 32 j + s + 0x1000 h at level j, step s; h = 0 is the
     * plain call); each candidate keeps its leading directions whose estimate
     * reaches theta, and amplify_s power iterations on its residual
     * C' - C' Z_h Z_h^T (start vectors from counter word 3 = 0x100000 +
     * 0x10000 g + 0x1000 h + 32 j + s, ceil(log2 d) + 1 steps) estimate its
     * top squared singular value; the candidate with the smallest estimate
     * (the first on ties) decides the step.  1 <= amplify_r <= 16,
     * 0 <= amplify_s <= 16; (1, 0) (the value sketch_config_init sets) is
     * the plain dump step.  SK_P5 applies it at every site; persistent
     * sketches require (1, 0).                                             */
    int32_t amplify_r;
    int32_t amplify_s;
    int32_t sites;        /* SK_P5: number of sites m, 1..4096                  */
    int32_t d_y;          /* SK_COD: dimension of the second stream (d is d_x)   */
    double theta;         /* SK_COD: dump threshold (> 0)                        */
} sketch_config;

/* Fills *cfg with defaults: exact FP64 persistent sketch, q = 1, no
 * oversampling, seed 0, device 0, library-owned stream.  d and ell are 0 and
 * must be set by the caller. */
SK_EXPORT sk_status sketch_config_init(sketch_config* cfg);

/* Creates a sketch; allocates all device state up front.
 * SK_EINVAL for bad fields; SK_ENOMEM if allocation fails or the
 * library-wide memory budget (sketch_set_memory_budget) would be exceeded. */
SK_EXPORT sk_status sketch_create(const sketch_config* cfg, sketch_t* out);

/* Appends n_rows rows (n_rows x d, leading dimension ld, element type dtype)
 * to the stream.  Rows are copied into the buffer (converted to the state
 * dtype, round-to-nearest-even); every time the buffer reaches 2*ell rows a
 * shrink runs (the FD reduce of Algorithm "AeroSketch: Update").  n_rows == 0 is a
 * no-op.  For SK_WINDOW sketches each row advances time by one. */
SK_EXPORT sk_status sketch_update(sketch_t h, const void* rows, int64_t n_rows, int64_t ld,
                        int32_t dtype, int32_t on_device);

/* Same for sparse rows in CSR form: indptr (n_rows + 1, int64, indptr[0] may
 * be non-zero), column indices (int32, in [0, d)), values (float32).
 * Duplicate indices within a row are summed in the order they appear in
 * the row (FP64 sum, then one rounding to the state dtype); the result does
 * not depend on thread timing.  Persistent sketches only. */
SK_EXPORT sk_status sketch_update_csr(sketch_t h, const int64_t* indptr, const int32_t* indices,
                            const float* values, int64_t n_rows, int32_t on_device);

/* Writes the ell x d sketch (row-major, dtype SK_F64 or SK_F32) to B_out.
 * Persistent: f_ell of the buffer rows, i.e. one exact shrink of the current
 * buffer when it holds >= ell rows (the final step of Algorithm "AeroSketch: Query").
 * Window: the query of Algorithm "ML-AeroSketch" for the window (T-N, T].
 * Non-destructive. */
SK_EXPORT sk_status sketch_query(sketch_t h, void* B_out, int32_t dtype, int32_t on_device);

/* SK_ATTP only (Sec. 4.1, Algorithm "ATTP Sketch using AeroSketch";
 * Theorem "ATTP"): writes the ell x d sketch of A_t, the first t rows of the
 * stream, 0 <= t <= T (T = rows seen), to B_out (row-major, SK_F64 or
 * SK_F32, host or device as on_device).  The sketch keeps one AeroSketch
 * whose dump threshold is eps ||A_i||_F^2 (eps = 2 / ell) when row i
 * arrives and every snapshot it ever dumped; B_out^T B_out is the restored
 * matrix of the snapshots taken at times <= t (plus the residual's Gram
 * when t = T) shrunk by its ell-th eigenvalue, with covariance error
 * O(eps) ||A_t||_F^2 w.h.p.  Blocks until B_out is written.  SK_EINVAL for t
 * outside [0, T] (state unchanged); SK_EUNSUPPORTED for other kinds.
 * sketch_query on an SK_ATTP sketch is sketch_query_at(T). */
SK_EXPORT sk_status sketch_query_at(sketch_t h, int64_t t, void* B_out, int32_t dtype, int32_t on_device);

/* SK_WINDOW only: moves time to t_now >= current time without rows and
 * expires what left the window.  SK_EUNSUPPORTED on persistent sketches,
 * SK_EINVAL (state unchanged) if t_now is in the past. */
SK_EXPORT sk_status window_advance(sketch_t h, int64_t t_now);

/* dst absorbs each source sketch in order: the non-zero rows of the source's
 * query are appended to dst as ordinary rows (stack and re-shrink, Lemma
 * "Decomposability").  Sources are unchanged.  SK_ESHAPE if d differs;
 * persistent sketches only. */
SK_EXPORT sk_status sketch_merge(sketch_t dst, const sketch_t* srcs, int32_t n_src);

/* Binary-tree merge of n_src sketches (same d and ell) into dst, which must be
 * empty: level by level, pairs (2i, 2i+1) in index order are stacked and
 * shrunk; the shrinks of one level run as one batched launch. */
SK_EXPORT sk_status sketch_merge_tree(sketch_t dst, const sketch_t* srcs, int32_t n_src);

/* Blocks until all work enqueued on h has finished; reports deferred device
 * errors (e.g. a non-converged eigen-solve). */
SK_EXPORT sk_status sketch_sync(sketch_t h);

/* Waits for outstanding work and frees the sketch.  NULL is a no-op. */
SK_EXPORT sk_status sketch_destroy(sketch_t h);

/* Thread-local message of the last failing call ("" if none). */
SK_EXPORT const char* sketch_last_error(void);

typedef struct {
    int64_t rows_seen;    /* rows appended so far (time for windows)              */
    int64_t fill;         /* rows in the buffer now                                */
    int64_t shrinks;      /* shrinks run so far                                    */
    int64_t device_bytes; /* device memory owned by the sketch                     */
    int32_t k;            /* target rank of the randomized shrink (0 if exact)     */
    int32_t levels;       /* window levels (1 for persistent sketches)             */
} sketch_info_t;

SK_EXPORT sk_status sketch_info(sketch_t h, sketch_info_t* info);

/* SK_WINDOW and SK_ATTP: counters of one level: [0] snapshots dumped,
 * [1] raw rows stored, [2] directions dumped, [3] rows in the level's FD
 * buffer, [4] queue length, [5] FD reduces.  SK_P5: level j is site j, and
 * [1] counts the rows it sent as they are, [4] is 0.  SK_COD: level 0, [1]
 * is 0, [3] the buffer rows, [4] the live snapshots, [5] the COD reduces. */
SK_EXPORT sk_status window_stats(sketch_t h, int32_t level, int64_t* stats6);

/* SK_P5 only (Sec. 4.3, Algorithm "P5"; Theorem "dist"): n_rows rows (rows,
 * n_rows x d, leading dimension ld, dtype SK_F64 / SK_F32 / SK_BF16, host or
 * device as on_device) arrive in order, row e at site sites[e] (host array
 * of n_rows ints in [0, m)).  Per row at site j: the site adds |a|^2 to its
 * counter F_j and sends it when F_j >= (eps / m) Fhat_j (eps = 2 / ell);
 * the coordinator adds it to Fhat and broadcasts Fhat at every m-th such
 * message, received by every site before the row's next step.  Then the
 * site's AeroSketch (2 ell x d FD buffer, dump threshold (eps / m) Fhat_j,
 * the theorem's per-site threshold) takes the row, and every snapshot it
 * dumps, (Z, Z^T C'^T C'), goes to the coordinator, which adds
 * Z W + W^T Z^T - Z (W Z) Z^T to its d x d matrix B.  While Fhat_j = 0 a
 * row goes to the coordinator as it is (B += a^T a).  Site j's random
 * draws are those of an SK_ATTP sketch with stream_id 4096 stream_id + j.
 * The sites' steps run together on the GPU; the result equals processing
 * the rows one by one.  Blocks until done.  SK_EINVAL (state unchanged) for
 * a site outside [0, m); SK_EUNSUPPORTED for other kinds (sketch_update on
 * an SK_P5 sketch is SK_EUNSUPPORTED too).  sketch_query returns B's
 * eigen-decomposition shrunk by its ell-th eigenvalue. */
SK_EXPORT sk_status p5_update(sketch_t h, const int32_t* sites, const void* rows, int64_t n_rows, int64_t ld,
                              int32_t dtype, int32_t on_device);

/* SK_COD only (Sec. 4.2, Algorithm "AeroSketchCOD Framework"; Theorem
 * "sw-amm"): n pairs arrive in order, x_i = row i of X (n x d, leading
 * dimension ldx) and y_i = row i of Y (n x d_y, ldy), both of dtype SK_F64 /
 * SK_F32 / SK_BF16 in host or device memory as on_device.  The sketch keeps
 * FD-style buffers A (2 ell x d) and B (2 ell x d_y) whose product A^T B
 * tracks the window's X_W^T Y_W: a pair is appended, the
 * co-occurring-directions reduce (the product's SVD shrunk by its ell-th
 * singular value, split evenly between A and B) runs when the buffers hold
 * 2 ell rows (ell - 1 remain), a power iteration estimates the top singular
 * value s1 of A^T B, and when s1 >= theta / 2 the doubling loop (k = 2, 4,
 * ...; left directions Z by simul_iter on A^T B with Philox counter word 3 =
 * 0x200 + step, right directions H and the estimates by simul_iter on its
 * transpose with 0x400 + step) dumps the directions whose singular-value
 * estimate reaches theta as a snapshot (Z, Z^T M, M H, H) and removes them
 * from A and B.  Snapshots leave after window_N pairs.  Blocks until done.
 * Requires d, d_y <= 4096, min(d, d_y) <= 512, ell <= 256, window_N >= 1,
 * theta > 0; SK_EUNSUPPORTED for other kinds. */
SK_EXPORT sk_status cod_update(sketch_t h, const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t n,
                               int32_t dtype, int32_t on_device);

/* SK_COD only: the query of Algorithm "AeroSketchCOD Framework": M_W = A^T B
 * plus every live snapshot's Z (Z^T M) + (M H) H^T - Z (Z^T M H) H^T; with its
 * SVD U S V^T, A_out = U sqrt(max(S - s_ell, 0)) (d x ell, row-major) and
 * B_out = V sqrt(max(S - s_ell, 0)) (d_y x ell), dtype SK_F64 or SK_F32, host
 * or device as on_device.  A_out B_out^T approximates X_W^T Y_W; compare
 * products, never the factors.  Blocks until written. */
SK_EXPORT sk_status cod_query(sketch_t h, void* A_out, void* B_out, int32_t dtype, int32_t on_device);

/* SK_COD only: the restored product M_W (d x d_y, FP64, row-major) before
 * the query's shrink, host or device as on_device. */
SK_EXPORT sk_status cod_product(sketch_t h, void* M_out, int32_t on_device);

/* SK_P5 only: [0] counter messages, [1] broadcasts, [2] snapshot messages,
 * [3] dumped directions, [4] rows sent as they are, [5] words sent (1 per
 * counter message, m per broadcast, d per row sent as it is, 2 d per
 * direction), [6] FD reduces over all sites, [7] rows seen. */
SK_EXPORT sk_status p5_stats(sketch_t h, int64_t* stats8);

/* SK_P5 only: the coordinator's Fhat (host double, may be NULL) and B
 * (d x d FP64 row-major, host or device as on_device, may be NULL).
 * Blocks until written. */
SK_EXPORT sk_status p5_coordinator(sketch_t h, double* fhat, void* gram, int32_t on_device);

/* Library-wide cap (bytes) on device memory held by live sketches; 0 = no
 * cap.  sketch_create returns SK_ENOMEM instead of exceeding it.  Used for
 * admission control by a serving loop. */
SK_EXPORT sk_status sketch_set_memory_budget(int64_t bytes);
SK_EXPORT int64_t sketch_memory_in_use(void);

/* Batched update: count sketches, each with its own device row block
 * (rows[i], n[i] rows, ld[i] = its d).  All sketches must share one HIP
 * stream and device.  Ingest and the shrinks that fall due are grouped
 * across sketches: one launch per pipeline stage serves every sketch whose
 * buffer filled at that point, whatever its d and ell. */
SK_EXPORT sk_status sketch_update_batch(sketch_t* hs, const void* const* rows, const int64_t* n,
                              int32_t count, int32_t dtype);
/* The same for CSR rows on the device (as sketch_update_csr with
 * on_device = 1): sketch i takes n[i] rows from indptr[i] (n[i] + 1 int64
 * offsets into indices[i] / values[i]; int32 column indices < d, FP32
 * values).  Used for many sites of a distributed stream on one GPU; each
 * sketch's result is bitwise the same as with its own sketch_update_csr. */
SK_EXPORT sk_status sketch_update_csr_batch(sketch_t* hs, const int64_t* const* indptr,
                                            const int32_t* const* indices, const float* const* values,
                                            const int64_t* n, int32_t count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * sketch_update_batch (dense rows on the device, same results bit for bit),
 * but the call allocates nothing.  The batch's task records (one per ingest
 * segment and per shrink) go into a static device array of
 * SK_NOALLOC_MAX_TASKS records (about 1.4 MiB, held by each GPU the library
 * runs on until the process ends) instead of the library's growable task
 * arena; the records are staged from host memory before the call returns.
 * SK_EINVAL, with the state unchanged, when the batch needs more records than
 * that.  All calls on one GPU share the array: calls that overlap on one GPU
 * (different streams or threads) race; calls on one stream are ordered. */
#define SK_NOALLOC_MAX_TASKS 16384
SK_EXPORT sk_status sketch_update_batch_noalloc(sketch_t* hs, const void* const* rows, const int64_t* n,
                                                int32_t count, int32_t dtype);

/* ---- serving ---------------------------------------------------------------
 * A request loop over many resident stream sketches on one GPU: streams are
 * admitted while the device-memory budget allows (others wait, first come
 * first served); bursts of rows are submitted with their arrival time; each
 * server_tick polls finished work, admits waiting streams and launches one
 * batched update (sketch_update_batch) for every stream that has pending
 * rows, so bursts that arrive while the GPU is busy join the next tick while
 * the host plans it.  A burst is complete -- its rows are queryable -- when
 * the batch holding its last rows has finished on the device.  Not
 * thread-safe: one driver thread per server. */
typedef struct sk_server_s* sk_server_t;

typedef struct {
    int32_t device;
    int32_t max_inflight;         /* ticks in flight at once (>= 1; default 2)   */
    int64_t memory_budget;        /* device bytes for admitted streams, 0 = none */
    int64_t max_rows_per_tick;    /* rows of one burst per tick, 0 = unlimited   */
    void* hip_stream;             /* stream for all work (see use_given_stream)  */
    double (*clock)(void* ctx);   /* seconds; NULL: steady clock + HIP events    */
    void* clock_ctx;
    int32_t use_given_stream;     /* 1: hip_stream as given, also NULL (the null
                                     stream); 0: NULL means a server-owned one   */
    int32_t max_shrinks_per_tick; /* rows of one stream per tick are also capped
                                     at this many shrinks' worth ((ell + 1) rows
                                     each; 64 / ell times as many for ell < 64),
                                     0 = no cap: keeps ticks short, so small
                                     bursts do not wait behind large ones      */
} sk_server_config;

typedef struct {
    int64_t ticket;
    int64_t stream;               /* server stream id                            */
    int64_t rows;
    double arrival;               /* as submitted                                */
    double launched;              /* clock when its first rows were launched     */
    double done;                  /* clock when its last rows finished           */
} sk_completion;

typedef struct {
    int64_t admitted, waiting, closed;
    int64_t bytes_in_use;
    int64_t ticks, batches, pending_bursts, inflight;
    int64_t rows_done;
} sk_server_stats;

SK_EXPORT sk_status server_config_init(sk_server_config* cfg);
SK_EXPORT sk_status server_create(const sk_server_config* cfg, sk_server_t* out);
/* Registers a stream with the given sketch configuration (its stream and
 * device fields are overridden by the server's).  The stream is admitted at
 * once if the budget allows, else it waits; *id is valid either way and
 * bursts may be submitted to a waiting stream. */
SK_EXPORT sk_status server_open(sk_server_t s, const sketch_config* cfg, int64_t* id);
/* Queues a burst of n device rows (dtype, leading dimension = the stream's
 * d).  The rows must stay valid until the burst completes. */
SK_EXPORT sk_status server_submit(sk_server_t s, int64_t id, const void* rows, int64_t n,
                                  int32_t dtype, double arrival, int64_t* ticket);
/* One scheduling step (non-blocking unless max_inflight ticks are on the
 * device).  *launched receives the number of bursts that got rows. */
SK_EXPORT sk_status server_tick(sk_server_t s, int32_t* launched);
/* Completed bursts since the last poll (up to max). */
SK_EXPORT sk_status server_poll(sk_server_t s, sk_completion* out, int32_t max, int32_t* n);
/* Runs ticks until every submitted burst of admitted streams has completed. */
SK_EXPORT sk_status server_drain(sk_server_t s);
/* Query of an admitted stream (blocks). */
SK_EXPORT sk_status server_query(sk_server_t s, int64_t id, void* B_out, int32_t dtype,
                                 int32_t on_device);
/* Ends a stream.  New bursts are refused at once; queued bursts still run,
 * and the sketch is released when they have completed (a waiting stream is
 * dropped with its bursts, which are reported with done = -1).  A released
 * sketch's memory is reused for the next admitted stream of the same shape
 * (d, ell, kind, dtypes, q, oversample) or freed when a waiting stream of
 * another shape needs the budget. */
SK_EXPORT sk_status server_close(sk_server_t s, int64_t id);
SK_EXPORT sk_status server_stats(sk_server_t s, sk_server_stats* out);
/* The server's clock in seconds (the fake clock when one is configured);
 * arrival times are given in this time base. */
SK_EXPORT double server_now(sk_server_t s);
SK_EXPORT sk_status server_destroy(sk_server_t s);

/* ---- failure injection (tests of the error paths) ---------------------------
 * Records one non-converged eigen-solve in the sketch's device status words,
 * in stream order after the work queued so far, exactly as a failing solver
 * would; nothing else changes.  The next sketch_sync / sketch_query then
 * returns SK_EDEVICE and the handle turns sticky.  Persistent sketches only
 * (SK_EUNSUPPORTED otherwise).  The server form acts on an admitted stream's
 * sketch (SK_ESTATE if the stream is not admitted).  Lets a test exercise
 * the failure path without making a kernel fail. */
SK_EXPORT sk_status sketch_debug_fail_solver(sketch_t h);
SK_EXPORT sk_status server_debug_fail_solver(sk_server_t s, int64_t id);

/* ---- profiling -------------------------------------------------------------
 * Per-stage GPU time of the pipeline, measured with HIP events recorded on
 * the sketch's stream around every launch of the enabled stages.  Disabled by
 * default.  Stage bits: */
enum {
    SK_STAGE_INGEST = 1u << 0,    /* row copy into the buffer                    */
    SK_STAGE_OMEGA = 1u << 1,     /* Philox test matrix                          */
    SK_STAGE_GRAM = 1u << 2,      /* buffer Gram C C^T (split-K + reduce)         */
    SK_STAGE_PROJECT = 1u << 3,   /* C Omega (split-K + reduce)                   */
    SK_STAGE_CHOLQR = 1u << 4,    /* CholeskyQR of the iterate                    */
    SK_STAGE_CORE_GEMM = 1u << 5, /* power steps, Rayleigh-Ritz and Z = Q U       */
    SK_STAGE_EIG = 1u << 6,       /* symmetric eigen-solve                        */
    SK_STAGE_THRESHOLD = 1u << 7, /* delta and the rebuild matrix                 */
    SK_STAGE_REBUILD = 1u << 8,   /* B' = T C                                     */
    SK_STAGE_EIG_BACK = 1u << 9,  /* eigenvectors back to the matrix's basis      */
    SK_STAGE_EIG_REDUCE = 1u << 10, /* tridiagonal reduction of the eigen-solve   */
    SK_STAGE_ALL = 0x7ffu
};

typedef struct {
    char name[24];
    int64_t calls;        /* launches timed                                  */
    double total_ms;      /* summed event-to-event time                      */
} sketch_stage_time;

/* Enables (mask != 0) or disables event timing of the given stages for h and
 * clears the accumulated times. */
SK_EXPORT sk_status sketch_profile_enable(sketch_t h, uint32_t stage_mask);

/* Waits for h's stream and returns up to max_entries accumulated stage times
 * (only stages with at least one timed launch).  *n_out receives the count.
 * Entries after the stages report solver counters of the last cooperative
 * eigen-solve ("eig_sweeps" etc.) in total_ms with calls = 0. */
SK_EXPORT sk_status sketch_profile_read(sketch_t h, sketch_stage_time* out, int32_t max_entries,
                              int32_t* n_out);

#ifdef __cplusplus
}
#endif
#endif
