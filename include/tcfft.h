/*
 * tcfft.h -- C ABI of the MI355X (gfx950) matrix-core FP16 FFT library
 * (libtcfft.so).  Plain C: no HIP or torch types in any signature; streams are
 * passed as `void*` holding a hipStream_t (NULL = the default stream).
 *
 * Method: tcFFT (Li, Cheng, Lin, arXiv 2104.11471).  A transform is a chain of
 * merging processes X_out = F_N1 . (T (.) X_in) (Sec. 2.1, Eq. 3) with
 * radix-16 DFT-matrix products on the matrix cores and radix-2/4/8 on the
 * vector ALU (Sec. 3.1), grouped into passes that exchange data through LDS
 * inside a pass and through HBM between passes (Sec. 3.2), with coalesced
 * strided access (Sec. 4.2).
 *
 * What is computed (Sec. 2.1, Eq. 1): for every transform b of the batch,
 *     Y_b[k] = 2^-S * sum_n x_b[n] * exp(dir * 2*pi*i * n*k / N)
 * with dir = TCFFT_FORWARD (-1) or TCFFT_INVERSE (+1), unnormalised except for
 * the exact power-of-two output scale 2^-S reported by tcfft_plan_scale_log2().
 * 2D transforms (Sec. 3.1) use the separable sum over a row-major nx-by-ny
 * array whose second dimension (ny) is contiguous.
 *
 * Data layouts (all device memory, caller-owned, 16-byte aligned):
 *   TCFFT_PREC_FP16        interleaved complex FP16 (re, im), 4 B per point;
 *                          1D element (b, n) at b*N + n, 2D (b, x, y) at
 *                          (b*nx + x)*ny + y.
 *   TCFFT_PREC_SPLIT_FP16  two such planes in one buffer: hi plane of B*N
 *                          points, then lo plane of B*N points; the value is
 *                          hi + 2^-11 * lo.
 *   TCFFT_PREC_FP32_RADIX2 interleaved complex FP32 (the plain radix-2
 *                          comparator path), 8 B per point.
 *   TCFFT_PREC_FP64        interleaved complex FP64, 16 B per point: the
 *                          radix-16 blocks on the FP64 matrix core
 *                          (v_mfma_f64_16x16x4f64), twiddles in FP64, no
 *                          output scale (S = 0); 1D only, N = 16..4096, one
 *                          launch; not for the server (UNSUPPORTED there).
 * Output is in natural order, in the same layout as the input.  in == out is
 * allowed (in-place).
 *
 * Errors: every entry point returns a status code; nothing aborts.  Nothing
 * prints unless the environment variable TCFFT_LOG is set (non-empty, not
 * "0"): then plan creation writes each plan's JSON description (as
 * tcfft_plan_describe) and every failing entry point its status to stderr.
 * Kernel faults surface asynchronously at the caller's next synchronisation.
 * Testing hook: while TCFFT_TEST_FAIL_ALLOC is set, every device allocation
 * of plan and server creation fails (ALLOC), so callers can exercise their
 * allocation-failure paths.
 */
#ifndef TCFFT_H_
#define TCFFT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tcfft_plan_s* tcfft_plan; /* opaque, owned by the library */

typedef enum {
  TCFFT_OK = 0,
  TCFFT_ERR_INVALID_ARG = 1, /* null/misaligned pointer, batch <= 0, bad dir/precision */
  TCFFT_ERR_UNSUPPORTED = 2, /* size outside the supported set (see tcfft_plan_create) */
  TCFFT_ERR_NO_DEVICE = 3,   /* no gfx950 device visible */
  TCFFT_ERR_ALLOC = 4,       /* device allocation failed */
  TCFFT_ERR_LAUNCH = 5,      /* a kernel launch was rejected by the runtime */
  TCFFT_ERR_INTERNAL = 6,
  TCFFT_ERR_TIMEOUT = 7,     /* serving: the request waited in the queue past queue_timeout_us */
  TCFFT_ERR_CANCELLED = 8    /* serving: the request was cancelled before it was admitted */
} tcfft_status;

#define TCFFT_FORWARD (-1)
#define TCFFT_INVERSE (+1)

enum {
  TCFFT_PREC_FP16 = 0,        /* FP16 storage, FP16 matrix-core products, FP32 accumulation */
  TCFFT_PREC_SPLIT_FP16 = 1,  /* hi+lo FP16 pairs, compensated products (precision recovery) */
  TCFFT_PREC_FP32_RADIX2 = 2, /* plain FP32 radix-2 Stockham, one launch per stage (comparator) */
  TCFFT_PREC_FP64 = 3         /* FP64 storage, FP64 matrix-core products (Sec. 7: wider types) */
};

enum {
  TCFFT_FLAG_NO_SCALE = 1u, /* S = 0: literally unnormalised (may overflow FP16 for large N) */
  TCFFT_FLAG_TUNE = 4u,     /* time every planner candidate on the device and keep the fastest */
  TCFFT_FLAG_REAL = 8u      /* real data: FORWARD is real-to-complex, INVERSE complex-to-real */
};

/*
 * Creates a plan (Sec. 3.1 and Fig. 1: the plan picks the merging kernels once,
 * the execution function runs them many times).
 *   out        receives the plan handle (set to NULL on failure)
 *   rank       1, 2 or 3
 *   dims       rank values: {N}, {nx, ny} or {nx, ny, nz} (last index
 *              contiguous); powers of two.  1D: 16 <= N <= 2^27.
 *              2D: 16 <= nx <= 2048, 16 <= ny <= 16384.
 *              3D: 16 <= nx, ny <= 2048, 16 <= nz <= 16384 (a row pass over
 *              nz, then column passes over ny and over nx).
 *   batch      number of transforms, >= 1 (batch * points <= 2^31 per plan)
 *   dir        TCFFT_FORWARD or TCFFT_INVERSE
 *   precision  TCFFT_PREC_*
 *   flags      TCFFT_FLAG_* bit set
 * Real transforms (TCFFT_FLAG_REAL; rank 1, 32 <= N <= 2^27, FP16 or split
 * precision).  With M = N/2, a real sequence x of N values is stored as M
 * complex words (word m holds x[2m] in its real half and x[2m+1] in its
 * imaginary half); the spectrum is the first M+1 bins X[0..M] of the N-point
 * DFT (the rest follow by Hermitian symmetry), M+1 complex words per
 * transform.  FORWARD reads batch*M words and writes batch*(M+1); INVERSE
 * reads batch*(M+1) words (the imaginary parts of X[0] and X[M] are ignored)
 * and writes batch*M words holding N * x * 2^-S.  Input and output must not
 * overlap (lines of M and M + 1 words cannot be rewritten in place).  The plan
 * runs an M-point
 * complex transform plus one elementwise pass (Eq. 2 with a radix-2 split of
 * the real sequence into its even and odd points); split precision stores
 * both buffers as a hi plane then a lo plane.
 * Allocates the plan's device tables (DFT-matrix operands, twiddles generated
 * in FP64 on the device) and its workspace on the current device; the tables
 * are generated on a private stream that the call waits for (other streams
 * are not synchronised).  With TCFFT_FLAG_TUNE, or when the tuning cache holds
 * a choice for this key, the planner's knobs come from the autotuner.
 * Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, ALLOC, LAUNCH.
 */
tcfft_status tcfft_plan_create(tcfft_plan* out, int rank, const int64_t* dims, int64_t batch,
                               int dir, int precision, unsigned flags);

/* The paper's plan functions (Sec. 3.1): forward FP16 plans of nx points
 * (1D) or nx-by-ny arrays (2D, ny contiguous). */
tcfft_status tcfft_plan_1d(tcfft_plan* out, int64_t nx, int64_t batch);
tcfft_status tcfft_plan_2d(tcfft_plan* out, int64_t nx, int64_t ny, int64_t batch);

/*
 * Executes a plan (the "execution function" of Fig. 1): reads `in`, writes
 * `out` (device pointers of tcfft_plan_input_bytes() and
 * tcfft_plan_output_bytes(), 16-byte aligned; in == out allowed for complex
 * plans, real plans need disjoint buffers), enqueued asynchronously on `stream` (a
 * hipStream_t or NULL).  One exec per plan may be in flight at a time (the
 * plan's workspace is shared).
 * Errors: INVALID_ARG (null plan/pointer, misalignment, overlapping buffers of
 * a real plan), LAUNCH.
 */
tcfft_status tcfft_exec(tcfft_plan plan, const void* in, void* out, void* stream);

/*
 * Mixed-size batch execution: job j runs plans[j] on (in[j], out[j]), all jobs
 * enqueued on one stream.  Jobs of any sizes and precisions mix.  Each job's
 * result is bitwise equal to tcfft_exec of that job alone.  Jobs are
 * independent: no job may write a buffer another job of the call reads or
 * writes (shared read-only inputs are fine).  A plan that holds a workspace
 * (multi-pass plans; real plans whose spectrum step is a separate pass) may
 * appear in only one job of a call, since its jobs would write the same
 * intermediate; single-pass plans may repeat.
 *
 * Launch structure (Sec. 3.1, Fig. 1: the plan fixes each transform's passes
 * once).  When every pass of every job is one of the variants compiled into
 * the fused kernel (the default FP16 and split plans of 1D N <= 2^22 and 2D
 * arrays up to 2048 x 2048, 256-thread variants), one kernel runs all
 * variants: by default one launch per (pass level, precision, LDS class)
 * with one workgroup per tile, pass l of every job after pass l-1 of every
 * job (stream order).  TCFFT_FUSED=2 in the environment instead makes it one
 * launch per (precision, LDS class) for all levels: workgroups take tiles
 * from an atomic counter in (level, job) order and a tile of pass l of a job
 * first waits until every tile of pass l-1 of that job has finished (a wait
 * bounded by the wall clock, 1 s by default or TCFFT_FUSED_WAIT_US
 * microseconds; a wait that runs out fails the whole launch, which then
 * drains, and is counted by tcfft_fused_wait_failures).  Otherwise (other
 * variants, real plans with a fused spectrum step, the single-pass 65536
 * kernel, or TCFFT_FUSED=0) one persistent launch per (level, variant) reads
 * a device-resident descriptor table.  FP32 radix-2 and FP64 jobs run as
 * their own launches first; chunked FP16 plans run on their own.
 * Errors: as tcfft_exec; INVALID_ARG for njobs < 0, null arrays or a
 * workspace-holding plan listed twice; ALLOC when the descriptor table cannot
 * be allocated (stream-ordered).
 */
tcfft_status tcfft_exec_many(const tcfft_plan* plans, const void* const* in, void* const* out,
                             int njobs, void* stream);

/*
 * For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): tcfft_exec_many with its
 * descriptor tables in a static device array of TCFFT_STATIC_SCRATCH_BYTES
 * per GPU (held until the process ends) instead of a stream-ordered
 * allocation, written by kernels from their arguments instead of a copy from
 * pinned host memory.  It calls no hipMalloc, hipFree or other allocating
 * routine.  Same jobs, rules and results as tcfft_exec_many (bitwise equal);
 * every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (different streams, no ordering between them) race; calls on one stream
 * are ordered.  Plans must be created beforehand (plan creation allocates).
 * Errors: as tcfft_exec_many; INVALID_ARG for njobs > TCFFT_STATIC_MAX_JOBS;
 * NO_DEVICE when the array's address cannot be taken.
 */
#define TCFFT_STATIC_SCRATCH_BYTES (1u << 20)
#define TCFFT_STATIC_MAX_JOBS 1024
tcfft_status tcfft_exec_many_static(const tcfft_plan* plans, const void* const* in,
                                    void* const* out, int njobs, void* stream);

/*
 * Runs only the first `npasses` passes of a multi-pass FP16 or split plan and
 * writes that pass's result to `out` (used to check the intermediate against
 * the decomposition of Sec. 2.1, Eq. 3).  After pass 1 of a long 1D plan with
 * first pass length N1 and M = N / N1, transform b holds at b*N + m*N1 + k1
 *     2^-s1 * W_N^{m k1} * sum_{n1 < N1} x[b][n1*M + m] * W_N1^{n1 k1},
 * with s1 the pass's scale exponent (tcfft_plan_describe, "passes"[0].scale);
 * after the row pass of a 2D plan it holds the row transforms in natural
 * order.  npasses equal to the plan's pass count is tcfft_exec.  `in` and
 * `out` must differ.  Errors: as tcfft_exec;
 * INVALID_ARG for npasses outside [1, passes] or in == out; UNSUPPORTED for
 * the FP32 comparator and real plans.
 */
tcfft_status tcfft_exec_passes(tcfft_plan plan, const void* in, void* out, int npasses,
                               void* stream);

/*
 * One device's share of a distributed 1D transform (the single-GPU kernels of
 * a multi-device four-step FFT; the paper's Sec. 6 names distributed FFT
 * frameworks as the place its kernels plug into).  The length N is split as
 * N = N1 * M (Sec. 2.1, Eq. 3 with n = n1 M + m and k = k1 + N1 k'), N1 the
 * first factor of the library's own long-1D plan (tcfft_plan_describe,
 * "shard_n1"), and the M columns m are dealt out to G = nshards devices in
 * slabs of M/G; device g = shard holds m = g M/G + m_l, m_l < M/G.  With
 * n1l = N1/G and ml = M/G, per transform b of the batch (all offsets in
 * complex points, b * N/G apart):
 *   step 1  in:  x[n1 M + g ml + m_l] at n1 ml + m_l            ([N1][ml])
 *           out: Z[k1][m] = 2^-s1 W_N^{m k1} sum_{n1} x[n1 M + m] W_N1^{n1 k1}
 *                at h (ml n1l) + m_l n1l + k1_l, k1 = h n1l + k1_l
 *                ([G][ml][n1l]: block h is the contiguous chunk for device h)
 *   exchange (the caller's all-to-all): device h receives block h of every
 *           device g and concatenates them in g order, giving [M][n1l]
 *           (row m = g ml + m_l)
 *   step 2  in:  that [M][n1l] array on device h
 *           out: X[k' N1 + h n1l + k1_l] * 2^-S at k' n1l + k1_l ([M][n1l])
 * s1 is passes[0].scale of the description and S = tcfft_plan_scale_log2().
 * Layouts as tcfft_exec (FP16 or split; split buffers hold the hi plane of
 * batch * N/G points, then the lo plane); every buffer of both steps holds
 * batch * N/G points (tcfft_plan_buffer_bytes).  Requires N > 16384,
 * nshards a power of two >= 2 with N1/nshards >= 4 and M/nshards >= 8,
 * 0 <= shard < nshards; TCFFT_FLAG_NO_SCALE allowed, TUNE ignored, REAL
 * rejected.  tcfft_exec, tcfft_exec_passes and tcfft_exec_many refuse shard
 * plans (UNSUPPORTED / INVALID_ARG): the two steps surround an exchange.
 * tcfft_exec_shard runs step 1 or 2; `in` and `out` must differ.
 * Errors: INVALID_ARG (bad shard, step, pointers), UNSUPPORTED (sizes),
 * NO_DEVICE, ALLOC, LAUNCH.  tcfft_shard_dry_run is the device-free planner
 * (returns the JSON length, or -(status)).
 */
tcfft_status tcfft_plan_create_shard(tcfft_plan* out, int64_t n, int64_t batch, int dir,
                                     int precision, int nshards, int shard, unsigned flags);
tcfft_status tcfft_exec_shard(tcfft_plan plan, int step, const void* in, void* out, void* stream);
int tcfft_shard_dry_run(int64_t n, int64_t batch, int dir, int precision, int nshards, int shard,
                        unsigned flags, char* buf, size_t len);

/* Releases the plan and its device memory (synchronises the device first:
 * the plan's tables may be read by work on any stream, and freeing device
 * memory waits for the device anyway).  NULL is accepted.  Errors: none
 * besides INTERNAL. */
tcfft_status tcfft_plan_destroy(tcfft_plan plan);

/* S such that out = DFT(in) * 2^-S (0 for NO_SCALE and the FP32 path); -1 for NULL. */
int tcfft_plan_scale_log2(tcfft_plan plan);

/* Bytes of the larger of the plan's input and output buffers (they are equal
 * for complex plans); 0 for NULL. */
size_t tcfft_plan_buffer_bytes(tcfft_plan plan);

/* Bytes of the plan's input buffer and of its output buffer (they differ for
 * real plans: M versus M+1 complex words per transform); 0 for NULL. */
size_t tcfft_plan_input_bytes(tcfft_plan plan);
size_t tcfft_plan_output_bytes(tcfft_plan plan);

/* Device workspace bytes held by the plan; 0 for NULL. */
size_t tcfft_plan_workspace_bytes(tcfft_plan plan);

/* Number of kernel launches of one exec; -1 for NULL. */
int tcfft_plan_num_launches(tcfft_plan plan);

/*
 * Writes a JSON description of the plan (passes, radices, kernels, scale) into
 * buf (NUL-terminated, truncated to len).  Returns the length the full text
 * needs (excluding the NUL), or -1 for NULL.
 */
int tcfft_plan_describe(tcfft_plan plan, char* buf, size_t len);

/*
 * Runs only the planner (no device needed) and writes the JSON description
 * the same arguments would produce.  Returns the needed length, or -(status)
 * when the arguments are rejected.
 */
int tcfft_plan_dry_run(int rank, const int64_t* dims, int64_t batch, int dir, int precision,
                       unsigned flags, char* buf, size_t len);

/*
 * Autotuner (plan "wisdom").  A plan created with TCFFT_FLAG_TUNE times every
 * candidate the planner can build for its (rank, dims, batch rounded down to a
 * power of two, precision) -- threads per workgroup, column-block width,
 * factorisation of long lengths -- on scratch device buffers and keeps the
 * fastest; the choice is cached in-process and reused by later plans with the
 * same key (tuned or not).
 *   tcfft_tune_candidates  JSON array of the candidate plans (no device);
 *                          returns the needed length or -(status).
 *   tcfft_tune_cache_size  number of cached choices.
 *   tcfft_tune_cache_save  writes the cache as text; INVALID_ARG if the file
 *                          cannot be written.
 *   tcfft_tune_cache_load  merges a saved cache; INVALID_ARG on a bad file.
 *   tcfft_tune_cache_clear forgets every cached choice.
 */
int tcfft_tune_candidates(int rank, const int64_t* dims, int64_t batch, int precision, char* buf,
                          size_t len);
int tcfft_tune_cache_size(void);
tcfft_status tcfft_tune_cache_save(const char* path);
tcfft_status tcfft_tune_cache_load(const char* path);
void tcfft_tune_cache_clear(void);

/*
 * Serving: continuous batching of mixed-size requests (not a paper item; the
 * scheduler feeds tcfft_exec_many-style grouped launches).
 *
 * A server owns `nslots` slots; a slot is a HIP stream, an event and a device
 * workspace arena of `arena_bytes` (0 = mem_budget_bytes / nslots).  Requests
 * are queued FIFO.  Whenever a slot is idle, the scheduler thread admits the
 * longest queue prefix (at most max_batch_jobs requests) whose bytes -- input
 * + output payload + workspace of every request in flight -- stay within
 * mem_budget_bytes and whose workspaces fit the slot's arena, and launches it
 * as one grouped execution; batches in different slots overlap on the GPU.
 * Completion is detected by polling the slot events; each request gets
 * submit / start / done timestamps (steady clock, ns, see tcfft_server_now_ns).
 * Plans are created per shape on first use (or ahead of time with
 * tcfft_server_prepare) and shared by all slots.  Each result is bitwise the
 * result of tcfft_exec of the same request alone (same kernels).
 */
typedef struct tcfft_server_s* tcfft_server;

typedef struct {
  int nslots;              /* 1..16 concurrent batches (HIP streams) */
  int max_batch_jobs;      /* >= 1 requests per batch */
  size_t mem_budget_bytes; /* > 0: payload + workspace of all requests in flight */
  size_t arena_bytes;      /* workspace arena per slot; 0 = mem_budget_bytes / nslots */
  int use_graphs;          /* nonzero: each slot captures its grouped launches as a HIP graph
                              once a kernel-variant sequence recurs, and replays it
                              (descriptor tables are rewritten in device memory per batch) */
  int batch_window_us;     /* while other slots are busy, hold a batch until its oldest
                              request has waited this long (0 = dispatch at once) */
  int queue_timeout_us;    /* > 0: a request still queued (not admitted) this long after its
                              submission completes with TCFFT_ERR_TIMEOUT instead of running */
} tcfft_server_config;

typedef struct {
  int rank;             /* 1 or 2 */
  int64_t dims[2];      /* {N, ignored} or {nx, ny} */
  int64_t batch;        /* transforms in this request */
  int dir;              /* TCFFT_FORWARD / TCFFT_INVERSE */
  int precision;        /* TCFFT_PREC_FP16 or TCFFT_PREC_SPLIT_FP16 */
  const void* in;       /* device buffers in the layouts of tcfft_exec, 16-byte aligned, */
  void* out;            /* owned by the caller and untouched by it until completion */
  uint64_t tag;         /* returned in the completion record */
} tcfft_request;

typedef struct {
  uint64_t tag;
  int status;           /* tcfft_status of the request */
  int batch_jobs;       /* requests in the batch that carried it */
  int64_t t_submit_ns, t_start_ns, t_done_ns;
  int batch_id;
} tcfft_completion;

typedef struct {
  int64_t submitted, completed, rejected, batches, max_batch_jobs;
  int64_t max_inflight_bytes, inflight_bytes, queued, plans;
} tcfft_server_stats;

/* Creates a server on the current device and starts its scheduler thread.
 * Errors: INVALID_ARG (bad config), NO_DEVICE, ALLOC (streams/arenas). */
tcfft_status tcfft_server_create(tcfft_server* out, const tcfft_server_config* cfg);
/* Creates the plans of these request shapes now (buffers are not used). */
tcfft_status tcfft_server_prepare(tcfft_server s, const tcfft_request* reqs, int n);
/* Enqueues a request (thread-safe, non-blocking).  Errors: INVALID_ARG,
 * UNSUPPORTED (size), ALLOC (the request alone exceeds the budget or an
 * arena: it could never be admitted). */
tcfft_status tcfft_server_submit(tcfft_server s, const tcfft_request* req);
/* Moves up to `max` completion records into `out`; returns how many, or
 * -(status) on bad arguments. */
int tcfft_server_poll(tcfft_server s, tcfft_completion* out, int max);
/* Cancels every queued (not yet admitted) request with this tag: each
 * completes with TCFFT_ERR_CANCELLED.  Requests already launched run to
 * completion.  Returns how many were cancelled, or -(status) for a NULL
 * server. */
int tcfft_server_cancel(tcfft_server s, uint64_t tag);
/* Waits until nothing is queued or in flight (timeout_ms < 0: forever);
 * INTERNAL on timeout. */
tcfft_status tcfft_server_wait_idle(tcfft_server s, int64_t timeout_ms);
tcfft_status tcfft_server_get_stats(tcfft_server s, tcfft_server_stats* st);
/* Stops the scheduler (queued, unadmitted requests are dropped), waits for
 * in-flight batches and frees everything.  NULL is accepted. */
tcfft_status tcfft_server_destroy(tcfft_server s);
/* The steady clock of the timestamps, in ns. */
int64_t tcfft_server_now_ns(void);

/* Static text for a status code. */
const char* tcfft_status_string(tcfft_status s);

/*
 * Diagnostics of the fused batch path in its dependency mode (tcfft_exec_many
 * with TCFFT_FUSED=2): the number of dependency waits, on the current device
 * since the library was loaded, that ran past their bound and failed their
 * launch.  Synchronous (a device copy);
 * *count is untouched on error.  Errors: INVALID_ARG (null), NO_DEVICE.
 */
tcfft_status tcfft_fused_wait_failures(unsigned* count);

/* Library version string. */
const char* tcfft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TCFFT_H_ */
