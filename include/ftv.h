/*
 * ftv.h -- C ABI of the MI355X (gfx950) heterogeneity-aware majority voter.
 *
 * The voter of Kicherer & Karl, "Heterogeneity-aware Fault Tolerance using a
 * Self-Organizing Runtime System": after a task has been run more than once
 * (dual-modular redundancy and its k-replica generalisation, Sec. IV-D), the
 * voter compares the replicas' results and determines the presumable correct
 * result.  Values of integer type are compared bit-wise; floating-point values
 * are equal when they differ by no more than a programmer-set maximum, because
 * diverse kernels on diverse processing units order and round differently
 * (Sec. IV-D; the paper's experiments allow 0.1% in single precision).  The type a
 * buffer is registered with selects its compare method (Sec. IV-E).  The voter
 * is itself an ordinary task that can run on any device (Sec. IV-D), here one
 * MI355X.
 *
 * Conventions for every call:
 *  - Buffer pointers are DEVICE pointers unless the parameter says "host".
 *    The caller owns all buffers; the library owns only its context workspace
 *    and, for the server, the output buffers it hands out until ftv_release.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls enqueue work and return; outputs are valid once the stream has
 *    been synchronised.  Inputs must stay alive and unchanged until then.
 *  - Return value: FTV_OK (0) or a negative FTV_E_* code.  No call throws or
 *    aborts.  ftv_last_error() returns a thread-local description of the last
 *    failure on the calling thread.
 *  - A context is used by one host thread at a time.  Its calls may be issued
 *    on different streams: per-task and block votes count in accumulators of
 *    their stream's own (at most 64 streams per context, FTV_E_BUSY beyond),
 *    and a batched or mixed-memory call on another stream than the previous
 *    one of its kind is ordered after that one on the device (they share the
 *    context's tables and staging).  The server calls (ftv_submit / ftv_poll /
 *    ftv_release / ftv_server_get_stats) are thread-safe.
 */
#ifndef FTV_H
#define FTV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define FTV_OK 0
#define FTV_E_INVALID (-1)  /* bad argument (NULL pointer, size, tolerance) */
#define FTV_E_DTYPE (-2)    /* unknown value type, or tolerance illegal for it */
#define FTV_E_K (-3)        /* replica count outside [2, FTV_MAX_K] */
#define FTV_E_ALIGN (-4)    /* pointer misaligned for the requested call */
#define FTV_E_HIP (-5)      /* a HIP runtime call failed (text in ftv_last_error) */
#define FTV_E_NOMEM (-6)    /* allocation failed, or request exceeds the budget */
#define FTV_E_BUSY (-7)     /* server queue full; context stream slots exhausted */
#define FTV_E_NOTREADY (-8) /* ftv_poll: request still in flight */
#define FTV_E_CLOSED (-9)   /* server shutting down / unknown ticket */
#define FTV_E_MISMATCH (-10) /* redundant voters disagree with no majority among them;
                                no voter unit left for a placed vote */

/* ---- value types (Sec. IV-E: registration carries the value type) --------- */
#define FTV_F32 0
#define FTV_F64 1
#define FTV_I32 2
#define FTV_I64 3

/* ---- tolerance kinds (Sec. IV-D) ------------------------------------------ */
#define FTV_TOL_EXACT 0 /* bit-wise; the only kind for integer types */
#define FTV_TOL_ULP 1   /* |key(a) - key(b)| <= max_ulp, key = signed-magnitude
                           bits as two's complement (+0 and -0 both 0) */
#define FTV_TOL_REL 2   /* |a-b| <= delta*max(|a|,|b|) or |a-b| <= abs_floor,
                           evaluated in IEEE binary64, round-to-nearest-even,
                           no fused multiply-add, no flush-to-zero */

/* ---- verdicts ------------------------------------------------------------- */
#define FTV_UNANIMOUS 0        /* every pair of replicas agrees everywhere */
#define FTV_TASK_MAJORITY 1    /* replica `winner` agrees with a strict majority
                                  of the replicas over the whole task */
#define FTV_ELEMENT_MAJORITY 2 /* every element has a strict majority; only the
                                  consensus buffer is a valid result */
#define FTV_UNRESOLVED 3       /* some element has no majority: re-execute */

#define FTV_MAX_K 7
#define FTV_MASK_NOMAJ 0x80 /* mask bit 7: element without a strict majority */

/* Tolerance.  NaN equals any NaN; an infinity equals only the same infinity;
 * +0 equals -0 (ULP and REL).  EXACT compares bit patterns. */
typedef struct ftv_tol {
  int32_t kind;      /* FTV_TOL_* */
  uint32_t reserved; /* must be 0 */
  uint64_t max_ulp;  /* FTV_TOL_ULP */
  double delta;      /* FTV_TOL_REL, e.g. 1e-3 for the paper's 0.1% */
  double abs_floor;  /* FTV_TOL_REL, 0 for none */
} ftv_tol;

/* Per-task result of a vote (device memory, written whole by the library). */
typedef struct ftv_stats {
  uint64_t pair[FTV_MAX_K][FTV_MAX_K]; /* elements where replicas i, j are unequal;
                                          symmetric, zero diagonal, zero beyond k */
  uint64_t disagree[FTV_MAX_K];        /* elements where replica r != consensus */
  uint64_t no_majority;                /* elements without a strict majority */
  uint64_t n;                          /* elements voted */
  int32_t verdict;                     /* FTV_UNANIMOUS .. FTV_UNRESOLVED */
  int32_t winner;                      /* TASK_MAJORITY: lowest replica agreeing with
                                          the most replicas over the whole task;
                                          otherwise the replica with the fewest
                                          disagreements (lowest index on ties) */
} ftv_stats;

/* One vote task: k replicas of n elements of one value type. */
typedef struct ftv_vote_desc {
  const void *replicas[FTV_MAX_K]; /* k device buffers, element-aligned */
  uint32_t k;                      /* 2..FTV_MAX_K */
  int32_t dtype;                   /* FTV_F32 .. FTV_I64 */
  uint64_t n;                      /* elements per replica (0 allowed) */
  ftv_tol tol;
  void *consensus;   /* n elements, or NULL (not written) */
  uint8_t *mask;     /* n bytes, or NULL: bit r = replica r unequal to the
                        consensus, bit 7 = no strict majority */
  ftv_stats *stats;  /* required */
} ftv_vote_desc;

typedef struct ftv_ctx ftv_ctx;

/* Library version string (static). */
const char *ftv_version(void);
/* Description of the last failure on this thread ("" if none). */
const char *ftv_last_error(void);
/* Monotonic clock used for all server timestamps (ns). */
int64_t ftv_now_ns(void);

/* Create a context on HIP device `device`: allocates its workspace (a few MiB).
 * *out receives the handle.  Errors: FTV_E_INVALID, FTV_E_HIP, FTV_E_NOMEM. */
int ftv_ctx_create(int device, ftv_ctx **out);
/* Synchronises the device (work still queued may read the workspace), then
 * frees the context and its workspace. */
int ftv_ctx_destroy(ftv_ctx *ctx);

/* ftv_vote -- the element-wise majority vote of one task (Sec. IV-D).
 *
 * Per element i, with eq() the tolerance test:
 *   support s_r = #{j : eq(x_r, x_j)} (itself included), M = max_r s_r;
 *   the element has a majority iff 2M > k;
 *   the consensus is, among the replicas of support M, the lower median under
 *   IEEE-754 totalOrder of the raw bits (two's-complement order for integers);
 *   mask bit r = !eq(x_r, consensus), bit 7 = no majority.
 * Counts: pair[i][j] = #(!eq(x_i, x_j)), disagree[r] = #(mask bit r),
 * no_majority = #(mask bit 7).  Verdict from those counts (see FTV_* above).
 * Results are bit-exact functions of the inputs: no launch shape, tile size or
 * schedule changes them.
 * No output (consensus, mask, stats) may share a byte with a replica or with
 * another output (FTV_E_INVALID): the general vote of an element may read its
 * replicas again after outputs of the same launch are stored, so the
 * consensus cannot be written over a replica.  Replicas may overlap each
 * other.
 * Errors: FTV_E_INVALID (NULL replica/stats, reserved != 0, bad tolerance,
 * overlapping outputs, n above 2^60),
 * FTV_E_DTYPE, FTV_E_K, FTV_E_ALIGN (pointer not a multiple of the element
 * size; stats not 8-byte aligned), FTV_E_BUSY (a 65th stream on the context),
 * FTV_E_HIP. */
int ftv_vote(ftv_ctx *ctx, const ftv_vote_desc *desc, void *stream);

/* Kernel timing, the measurement of the paper's voter comparison (Sec. V-A
 * times the voter kernels alone, per data size, transfers excluded).  With
 * timing on (on = 1), each ftv_vote records a pair of HIP events on its stream
 * around its vote kernel (the finalize kernel after it is not included), and
 * each ftv_vote_batch launches its three kernels directly instead of from the
 * captured graph, with the events around the persistent vote kernel; the
 * results are unchanged.  At most 1024 launches are recorded between two
 * reads; later ones run untimed.  on = 0 stops recording.  Turning timing on
 * creates the events once (FTV_E_HIP if that fails) and clears the record.
 * Errors: FTV_E_INVALID. */
int ftv_ctx_set_timing(ftv_ctx *ctx, int on);
/* Waits for the recorded launches, writes the kernel time of the first
 * min(cap, count) of them to ms[] (host, milliseconds, in launch order), sets
 * *count to the number recorded, and clears the record.  Errors:
 * FTV_E_INVALID (NULL count, NULL ms with cap > 0), FTV_E_HIP. */
int ftv_ctx_kernel_times(ftv_ctx *ctx, float *ms, uint32_t cap, uint32_t *count);

/* ftv_vote_mem -- ftv_vote over replicas that lie in different memories: a
 * task duplicated onto a CPU and a GPU leaves one result in host memory and
 * one in device memory (Sec. IV-D), and where the results lie decides what a
 * vote costs (Sec. V-A).  memory[r] (HOST array of k) is FTV_MEM_HOST or
 * FTV_MEM_DEVICE and says where replicas[r] lies; consensus, mask and stats
 * are device memory as for ftv_vote.  A host replica in page-locked memory
 * mapped into the device's address space (hipHostMalloc, PyTorch's pinned
 * tensors; the runtime's pointer attributes decide) is read by the vote
 * kernel in place, over the link, with no staging.  Pageable host replicas
 * are streamed in pieces of chunk_bytes per replica (rounded down to 4096
 * elements; in [1 MiB, 4 GiB]) through two device staging sets of the
 * context on a copy stream, each piece voted as soon as it has arrived while
 * the next one is copied; the counts of all pieces form one stats record.
 * Results are identical to ftv_vote on device copies of the same replicas.
 * Host replicas must stay unchanged until the stream has been synchronised.
 * No pageable host replica (or n = 0): one ftv_vote.
 * Errors: those of ftv_vote, FTV_E_INVALID (memory flag, chunk_bytes),
 * FTV_E_NOMEM (staging), FTV_E_HIP. */
int ftv_vote_mem(ftv_ctx *ctx, const ftv_vote_desc *desc, const int32_t *memory, uint64_t chunk_bytes,
                 void *stream);

/* ftv_vote_host -- the same vote on the host's cores.  The paper keeps the
 * voter as kernels for several processing units -- single-threaded, OpenMP
 * and GPU -- because which one is fastest depends on the data size (Sec. V-A,
 * Fig. 3).  Every pointer in `desc` is HOST memory (replicas, consensus,
 * mask, stats).  threads = 1: the calling thread only; 0: one thread per core
 * the process may use; otherwise that many threads (OpenMP); in every case at
 * most one thread per 4096 elements, so a small vote runs on the calling
 * thread without a parallel region.  Results are
 * bit-identical to ftv_vote on the same replicas, under the same overlap
 * rule.  Synchronous: outputs are complete when the call returns.  Needs no GPU.  Errors: FTV_E_INVALID,
 * FTV_E_DTYPE, FTV_E_K, FTV_E_ALIGN (a pointer not a multiple of the element
 * size; stats not 8-byte aligned). */
int ftv_vote_host(const ftv_vote_desc *desc, uint32_t threads);

/* ftv_vote_batch -- ntasks independent votes (any mix of value types, k and
 * tolerances) in ONE persistent kernel launch, replayed from a captured HIP
 * graph (the small-task motivation: Sec. V-A, the voter's best device depends
 * on the data size).  `descs` is a HOST array.  Each task's results are
 * identical to those of ftv_vote on the same task.  Tasks of one call run
 * concurrently: no task may write memory that another
 * task of the call reads or writes (not checked).  Additional requirement:
 * every replica and consensus pointer 16-byte aligned and every mask pointer
 * 4-byte aligned (FTV_E_ALIGN otherwise).  The host arrays may be reused as
 * soon as the call returns.  Errors: those of ftv_vote for the first invalid
 * descriptor (its index in ftv_last_error), FTV_E_INVALID (NULL array, more
 * than 2^32 - 1 tasks or tiles), FTV_E_NOMEM (table growth), FTV_E_HIP. */
int ftv_vote_batch(ftv_ctx *ctx, const ftv_vote_desc *descs, uint64_t ntasks, void *stream);

/* ftv_vote_batch_noalloc -- for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * batched vote of ftv_vote_batch (same descriptors, same rules, identical
 * results) with no context and no allocation of any kind: the task table, tile
 * queue and count accumulators live in a static device array of the library,
 * FTV_NOALLOC_SCRATCH_BYTES on every GPU it runs on, held until the process
 * ends.  Work goes to the CURRENT device on `stream`, with ftv_vote_batch's
 * default schedule (kernels launched directly, no graph).  The host side
 * builds the table in static host arrays under one lock and uploads it from
 * pageable memory (a blocking copy for the host).  Every call on a GPU shares
 * that GPU's array and clears what it needs first; calls on one stream are
 * ordered by it, but calls whose work overlaps on one GPU (other streams,
 * other threads, without an event between them) race and give wrong results:
 * order them.  Errors: those of ftv_vote_batch, and FTV_E_INVALID for more
 * than FTV_NOALLOC_MAX_TASKS tasks (nothing is enqueued) or a device index
 * above 63. */
#define FTV_NOALLOC_MAX_TASKS 4096
#define FTV_NOALLOC_SCRATCH_BYTES (1792u * 1024u)
int ftv_vote_batch_noalloc(const ftv_vote_desc *descs, uint64_t ntasks, void *stream);

/* Schedule of the batched launch, chosen by ftv_tune_batch.  None of these
 * fields can change a result, only the time taken. */
typedef struct ftv_batch_cfg {
  uint32_t tile_vecs;  /* 16-byte vectors per replica per tile (multiple of block) */
  uint32_t block;      /* threads per workgroup: 256 or 512 */
  uint32_t grid_mult;  /* workgroups per compute unit */
  uint32_t order;      /* tiles are handed out task by task in this order:
                          0 = as given, 1 = largest task first (LPT),
                          2 = smallest task first, 3 = grouped by value
                          type, tolerance and k, largest first within a
                          group (co-resident workgroups then run the same
                          code) */
  uint32_t nt_stores;  /* 1 = streaming stores for consensus and mask
                          (non-temporal, agent scope: written through the
                          L2), 0 = ordinary stores */
  uint32_t reserved;
} ftv_batch_cfg;

int ftv_batch_get_config(ftv_ctx *ctx, ftv_batch_cfg *out);
/* FTV_E_INVALID if a field is out of range. */
int ftv_batch_set_config(ftv_ctx *ctx, const ftv_batch_cfg *cfg);
/* Autotuner: coordinate descent from the context's current schedule over tile
 * size, block size, grid multiple, order and store kind, two passes, each
 * candidate timed on this batch (the mean of `iters` back-to-back runs after a
 * warm one, on `stream`, synchronising it); the winner is re-timed against the
 * starting schedule (interleaved, twice) and the faster one is installed in
 * the context and written to
 * *best (may be NULL).  The batch's outputs hold a valid result
 * afterwards.  If the environment variable FTV_TUNE_CACHE names a file, the
 * choice is stored there as JSON keyed by device name, CU count and a coarse
 * signature of the batch, and reused by ftv_tune_batch on a cache hit. */
int ftv_tune_batch(ftv_ctx *ctx, const ftv_vote_desc *descs, uint64_t ntasks, void *stream,
                   uint32_t iters, ftv_batch_cfg *best);

/* ftv_fingerprint -- one 64-bit fingerprint per block of `block_bytes` of a
 * buffer, for validating checkpoints (the paper validates by versioned backup
 * copies, Sec. IV-A/IV-C; the fingerprint makes a copy comparable without
 * moving it).  Definition: the buffer is read as little-endian 64-bit words,
 * zero-padded to whole blocks; a leaf is 64-bit FNV-1a over 8 words (64 B);
 * leaves are combined pairwise, (0,1), (2,3), ..., level by level, a node being
 * FNV-1a over the two words (left, right).
 * block_bytes: a power of two in [4096, 65536].  buf: 16-byte aligned.
 * fp_out: ceil(nbytes / block_bytes) uint64 (device).
 * Errors: FTV_E_INVALID, FTV_E_ALIGN, FTV_E_HIP. */
int ftv_fingerprint(ftv_ctx *ctx, const void *buf, uint64_t nbytes, uint64_t block_bytes,
                    uint64_t *fp_out, void *stream);

/* Result of a block vote (device memory, written whole). */
typedef struct ftv_block_stats {
  uint64_t blocks;              /* ceil(nbytes / block_bytes) */
  uint64_t disagree_blocks;     /* blocks where some fingerprint differs */
  uint64_t fallback_blocks;     /* blocks without a fingerprint majority */
  uint64_t unresolved_elems;    /* elements of fallback blocks without majority */
  uint64_t replica_blocks[FTV_MAX_K]; /* blocks where replica r differs from the source */
  int32_t verdict;              /* UNANIMOUS: no block differs; TASK_MAJORITY:
                                   no fallback and replica `winner` matches the
                                   source everywhere; ELEMENT_MAJORITY: every
                                   element resolved; else UNRESOLVED */
  int32_t winner;
} ftv_block_stats;

/* ftv_vote_blocks -- checkpoint validation plus vote: fingerprints every block
 * of the k replicas, votes the fingerprints by exact equality, and restores the
 * consensus by copying, per block, the block of the lowest-indexed replica that
 * holds a strict-majority fingerprint (recopy from a valid copy, Sec. IV-A).  A
 * block without a fingerprint majority falls back to the element vote of
 * ftv_vote under `fallback_tol` over that block's elements.
 * replicas: HOST array of k device pointers, each 16-byte aligned.
 * nbytes: a multiple of the element size.  block_bytes: power of two in
 * [4096, 65536].  fps: k * nblocks uint64 (replica-major) or NULL (the
 * context then keeps them in a workspace of its own, grown on demand; such
 * calls on different streams are ordered one after the other).
 * blockmap: nblocks bytes: bit r = replica r's fingerprint differs from the
 * source's, bit 7 = no fingerprint majority.  consensus: nbytes, 16-byte
 * aligned.  mask: n bytes (4-byte aligned) or NULL; 0 outside fallback blocks,
 * element-vote mask inside them.  bstats: device, 8-byte aligned.  No output
 * may share a byte with a replica or another output (the restore copies
 * whole blocks while blocks of every replica are still read).
 * Errors: FTV_E_INVALID (NULL argument, block size, nbytes not a multiple of
 * the element size, more than 2^31 - 1 blocks, overlapping outputs), FTV_E_K, FTV_E_DTYPE (also an
 * illegal fallback tolerance), FTV_E_ALIGN, FTV_E_NOMEM (fingerprint
 * workspace), FTV_E_HIP. */
int ftv_vote_blocks(ftv_ctx *ctx, const void *const *replicas, uint32_t k, int32_t dtype,
                    uint64_t nbytes, uint64_t block_bytes, const ftv_tol *fallback_tol,
                    uint64_t *fps, uint8_t *blockmap, void *consensus, uint8_t *mask,
                    ftv_block_stats *bstats, void *stream);

/* ---- serving: continuous batching of vote / fingerprint requests ---------- *
 * The voter as a service that admits requests as tasks finish (Sec. IV-D: the
 * voter is a task the runtime schedules like any other).  A server thread admits
 * queued requests in arrival order while the HBM budget and the slot count
 * allow, and runs iterations: each iteration is one persistent launch over a
 * chunk (<= chunk_bytes per replica) of every admitted request, so requests
 * that arrive while others are on the GPU join the next iteration and their
 * work shares launches.  Results are identical to ftv_vote / ftv_fingerprint of
 * the same request alone. */
typedef struct ftv_server ftv_server;

typedef struct ftv_server_cfg {
  uint64_t hbm_budget_bytes; /* admitted footprint limit: replica inputs held
                                while in flight + outputs until released */
  uint64_t arena_bytes;      /* device memory the server carves outputs from for
                                requests that pass NULL outputs (0 = none) */
  uint64_t chunk_bytes;      /* per-request bytes per replica per iteration */
  uint32_t max_slots;        /* requests admitted at once, 1..4096 */
  uint32_t max_queue;        /* queued (not yet admitted) requests; submit
                                returns FTV_E_BUSY beyond it */
  int32_t device;
  uint32_t reserved;         /* must be 0 */
} ftv_server_cfg;

#define FTV_REQ_VOTE 0
#define FTV_REQ_FINGERPRINT 1

typedef struct ftv_request {
  int32_t kind;        /* FTV_REQ_VOTE or FTV_REQ_FINGERPRINT */
  uint32_t reserved;
  ftv_vote_desc vote;  /* VOTE: replicas/k/dtype/n/tol; consensus and mask may be
                          caller buffers or NULL = allocated by the server from
                          its budget; stats is ignored (the result carries them).
                          Same alignment rules as ftv_vote_batch. */
  const void *fp_buf;  /* FINGERPRINT: 16-byte aligned device buffer */
  uint64_t fp_bytes;
  uint64_t block_bytes;
  int64_t t_arrival_ns; /* ftv_now_ns() clock; 0 = time of submission */
  uint64_t user_tag;
  void *ready;          /* hipEvent_t recorded after the work that produces the
                           request's inputs, or NULL when they are complete at
                           submission; the server's stream waits for it before
                           it first reads them.  It must stay valid and must not
                           be recorded again until ftv_poll reports the request
                           done. */
} ftv_request;

typedef struct ftv_result {
  int32_t status;      /* FTV_OK or the error that ended the request */
  int32_t kind;
  ftv_stats stats;     /* host copy (VOTE) */
  void *consensus;     /* device; server-owned until ftv_release if allocated */
  uint8_t *mask;
  uint64_t *fps;       /* FINGERPRINT: device, server-owned until ftv_release */
  uint64_t nfps;
  int64_t t_arrival_ns, t_submit_ns, t_admit_ns, t_done_ns;
  uint64_t user_tag;
} ftv_result;

typedef struct ftv_server_stats {
  uint64_t submitted, completed, queued, in_flight, rejected;
  uint64_t bytes_in_flight, peak_bytes_in_flight;
  uint64_t iterations, peak_queue_depth;
  uint64_t shared_iterations;          /* iterations that carried work of 2+ requests */
  uint64_t max_requests_per_iteration;
  double mean_queue_depth;   /* time-averaged queued requests */
  double p50_us, p99_us;     /* arrival -> completion, completed requests */
  double mean_us, max_us;
  double replica_gbps;       /* replica bytes voted / busy wall time */
} ftv_server_stats;

/* Start a server on cfg->device (its own stream and thread); *out receives the
 * handle.  Errors: FTV_E_INVALID (NULL argument, a field out of range,
 * reserved != 0), FTV_E_NOMEM (arena or tables), FTV_E_HIP. */
int ftv_server_create(const ftv_server_cfg *cfg, ftv_server **out);
/* Enqueue a request; *ticket identifies it.  A vote request's descriptor
 * follows ftv_vote's rules (FTV_E_INVALID, FTV_E_ALIGN, ... as there);
 * requests in flight together share launches, so no request may write memory
 * that another one in flight reads or writes (not checked).  FTV_E_NOMEM if
 * its footprint alone exceeds the budget, FTV_E_BUSY if the queue is full. */
int ftv_submit(ftv_server *srv, const ftv_request *req, uint64_t *ticket);
/* Wait up to wait_us (0 = do not wait, <0 = forever) for a ticket.
 * FTV_OK with *out filled, FTV_E_NOTREADY, or FTV_E_CLOSED (unknown ticket). */
int ftv_poll(ftv_server *srv, uint64_t ticket, ftv_result *out, int64_t wait_us);
/* Forget a completed ticket and return its server-allocated outputs to the
 * budget.  FTV_E_NOTREADY if it is still in flight, FTV_E_CLOSED if unknown. */
int ftv_release(ftv_server *srv, uint64_t ticket);
/* Counters and latency percentiles so far (host struct).  FTV_E_INVALID on
 * NULL. */
int ftv_server_get_stats(ftv_server *srv, ftv_server_stats *out);
/* Drains in-flight work, then stops the server thread and frees everything. */
int ftv_server_destroy(ftv_server *srv);

/* ---- fault-aware runtime estimation (Sec. IV-B) --------------------------- *
 * A processing unit i with fault-free runtime R_i that produced v_i valid
 * results out of t_i runs has fault probability p_i = 1 - v_i/t_i (the paper
 * prints p_i = v_i/t_i while calling it the fault probability; its worked
 * numbers -- a unit twice as fast is worth keeping below 50%, p = 0.75 gives
 * four times the runtime, a unit three times as fast loses from 66% on --
 * fix this reading) and fault-aware runtime F_i = R_i / (1 - p_i), the
 * expected time until the unit returns a correct result.  F_i is +infinity
 * when p_i = 1; such a unit is only re-tried at check intervals. */
typedef struct ftv_unit {
  double runtime;   /* R_i: fault-free runtime (any unit, > 0) */
  uint64_t valid;   /* v_i */
  uint64_t total;   /* t_i (0 = no history: F_i = R_i) */
  uint64_t skipped; /* decisions that passed the unit over while F_i was
                       +infinity, since it last ran (the check interval's
                       counter; see ftv_run_redundant and the voter database) */
} ftv_unit;

/* F_i of one unit; +infinity when valid == 0 < total; NaN for bad input
 * (runtime <= 0 or valid > total). */
double ftv_fault_aware_runtime(const ftv_unit *unit);
/* Order (host array of n indices) of the units by increasing F_i, ties by
 * lower index; units with F_i = +infinity come last unless `probe` is set, in
 * which case the first of them is moved to the front (the periodic re-check
 * of a unit that looked permanently faulty).  FTV_E_INVALID on bad input. */
int ftv_rank_units(const ftv_unit *units, uint32_t n, int probe, uint32_t *order);
/* Account one voted task: replica r was produced by unit unit_of_replica[r]
 * (host arrays; `stats` is a HOST copy of the task's ftv_stats).  A replica's
 * run is valid when it agrees with the consensus on every element
 * (disagree[r] == 0).  An UNRESOLVED vote decides nothing and changes no
 * counter (the task is re-executed). */
int ftv_record_vote(ftv_unit *units, uint32_t nunits, const uint32_t *unit_of_replica, uint32_t k,
                    const ftv_stats *stats);

/* ---- memory areas with siblings and versions (Sec. IV-A, IV-C) ------------ *
 * The runtime's memory management: a registered area has copies ("siblings")
 * in host memory and in device memory, each tagged with a version that every
 * write raises by one.  A request for the area in some memory
 * returns a sibling there holding the highest version, copying the data into
 * a new (or stale, reused) sibling when that memory has none.  In
 * fault-tolerant mode a request is only served by an existing sibling when
 * another highest-version sibling exists as well; otherwise the request gets a
 * fresh sibling, so the previous one survives as the backup.  A kernel
 * that ran into a fault releases its sibling with ok = 0, which invalidates
 * it; the next request copies from a valid sibling (Fig. 1).  ftv_mm_check
 * compares the highest-version siblings by block fingerprints and invalidates
 * those that differ from a strict majority -- validation of backups without
 * moving them.
 *
 * Readings where the paper is silent: a new sibling reuses the lowest-indexed
 * stale or invalid sibling not in use in that memory before allocating
 * (sibling 0 is the caller's registered host area, so a host request brings
 * the newest data back into it); among candidates the lowest index wins and a
 * copy source in the requested memory is preferred; a sibling handed out for
 * writing is neither a candidate nor a copy source until released, and a
 * write never gets a sibling that has readers; a release with ok = 0
 * invalidates the sibling whatever the access.
 *
 * All calls on one manager are serialised internally (thread-safe).  Copies
 * into device siblings are enqueued on `stream`; a request for host memory
 * synchronises `stream` before it returns. */
typedef struct ftv_mm ftv_mm;

#define FTV_MEM_HOST 0
#define FTV_MEM_DEVICE 1
#define FTV_ACC_READ 1
#define FTV_ACC_WRITE 2
#define FTV_ACC_READWRITE 3
#define FTV_MM_MAX_SIBLINGS 64

typedef struct ftv_sibling_info {
  void *ptr;           /* host or device address of the sibling's bytes */
  int32_t memory;      /* FTV_MEM_HOST or FTV_MEM_DEVICE */
  int32_t valid;       /* 0 after a release with ok = 0 or a failed check */
  uint64_t version;    /* 1 at registration; +1 per successful write */
  uint32_t readers;    /* requests for reading not yet released */
  int32_t writing;     /* handed out for writing, not yet released */
  int32_t caller;      /* 1 for sibling 0, the caller's registered area */
  uint32_t reserved;
} ftv_sibling_info;

typedef struct ftv_mm_check_result {
  uint32_t checked;        /* highest-version siblings compared */
  uint32_t invalidated;    /* of those, marked invalid */
  uint64_t unresolved;     /* blocks without a strict majority fingerprint */
  uint64_t blocks;         /* blocks per sibling */
} ftv_mm_check_result;

/* device >= 0: siblings in that device's memory; device = -1: host memory
 * only (no HIP call is made; device requests and ftv_mm_check fail).
 * fault_tolerant: 0 or 1 (the rules above).  FTV_E_INVALID, FTV_E_HIP,
 * FTV_E_NOMEM. */
int ftv_mm_create(int device, int fault_tolerant, ftv_mm **out);
/* Frees every sibling the manager allocated (never the registered areas). */
int ftv_mm_destroy(ftv_mm *mm);
/* Register the caller's host area (host_ptr, bytes > 0; it stays owned by the
 * caller and must outlive the manager) as sibling 0 at version 1.  *area
 * receives its handle. */
int ftv_mm_register(ftv_mm *mm, void *host_ptr, uint64_t bytes, uint32_t *area);
/* Request the area in `memory` for `access` (FTV_ACC_*): *ptr receives the
 * sibling's address (valid for work on `stream` after this call), *sibling its
 * index for ftv_mm_release.  FTV_E_BUSY when the only highest-version siblings
 * are being written; FTV_E_INVALID when no valid sibling is left (every copy
 * failed: re-register the input) or on bad arguments; FTV_E_NOMEM when a new
 * sibling cannot be allocated or FTV_MM_MAX_SIBLINGS is reached. */
int ftv_mm_request(ftv_mm *mm, uint32_t area, int memory, int access, void *stream, void **ptr,
                   uint32_t *sibling);
/* End the use of a sibling obtained from ftv_mm_request.  ok = 1: a write
 * makes the sibling the newest (version = highest + 1); a read just ends.
 * ok = 0: a fault was detected while the sibling was in use; it becomes
 * invalid.  The caller must have synchronised the work that used it. */
int ftv_mm_release(ftv_mm *mm, uint32_t area, uint32_t sibling, int ok);
/* Copy the sibling table of an area into out[0 .. min(cap, count)) (host);
 * *count receives the number of siblings. */
int ftv_mm_siblings(ftv_mm *mm, uint32_t area, ftv_sibling_info *out, uint32_t cap, uint32_t *count);
/* Fingerprint every valid highest-version sibling not being written (host
 * siblings through a device staging copy) in blocks of block_bytes (a power of
 * two in [4096, 65536], the definition of ftv_fingerprint), vote per block,
 * and invalidate the siblings that differ from a strict majority in some
 * block.  Synchronises `stream`.  Fewer than two such siblings: nothing is
 * compared.  *out (host) receives the counts. */
int ftv_mm_check(ftv_mm *mm, uint32_t area, uint64_t block_bytes, void *stream,
                 ftv_mm_check_result *out);

/* ---- redundant execution with light-weight fault tolerance (Sec. IV-C, IV-D) *
 * A task has several implementations, each a kernel of some processing unit
 * with a profile in `units` (ftv_unit: runtime in SECONDS here, valid runs,
 * runs).  An attempt runs the task on the k implementations with the lowest
 * fault-aware runtime (ties: lower index) not yet failed in this call, each
 * into a replica buffer of the library on a stream of its own.  A run that
 * reports a direct fault (its run function returns non-zero, or a HIP error
 * is pending after it) or, for a unit with a profile (runtime > 0 and
 * valid > 0), does not finish within runtime x timeout_factor seconds is
 * abandoned: not voted, counted as a run that was not valid (total + 1), its
 * implementation excluded for the rest of the call, and its buffer reused only
 * after its work has drained (the call does not wait for it).  At least two
 * surviving runs are voted with ftv_vote into `out`; each voted run counts
 * (total + 1) and is valid (valid + 1) when it agrees with the consensus
 * everywhere, and the runtime of a valid run's unit becomes the running mean
 * of its valid runs' GPU times.  An UNRESOLVED vote changes no profile and
 * starts the next attempt, re-ranked; fewer than two implementations left
 * end the call.  Check intervals (Sec. IV-B: a unit with p = 1 is tried again only
 * at fixed intervals): when cfg->check_interval > 0, each attempt
 * passes over the units with F = +infinity that are not among its k runs,
 * adding 1 to their `skipped`; the first (in rank order) whose count would
 * reach check_interval instead runs as an extra replica of the attempt
 * (k + 1 runs, at most FTV_MAX_K) and is voted and counted like the others,
 * so a unit that has recovered regains a finite F; a unit that runs has its
 * count reset to 0.  Readings: after a fault the paper moves on to the
 * best-ranked remaining pairing of kernel and unit and votes DMR pairs; the exclusion rule, the
 * running mean, counting a failed run as an invalid one and re-trying as an
 * extra replica are this library's. */
typedef int (*ftv_task_fn)(void *user, void *out, void *stream);

typedef struct ftv_impl {
  ftv_task_fn run;   /* enqueue the task's result (n elements) into the device
                        buffer `out` on `stream` (a hipStream_t); must return
                        without waiting for the work */
  void *user;        /* passed to run */
  uint32_t unit;     /* index of its profile in `units` */
  uint32_t reserved;
} ftv_impl;

typedef struct ftv_redundancy_cfg {
  uint32_t k;              /* runs per attempt: 2 (DMR) .. FTV_MAX_K */
  uint32_t max_attempts;   /* >= 1 */
  double timeout_factor;   /* deadline = profiled runtime x factor; 0 = none */
  int32_t dtype;           /* FTV_F32 .. FTV_I64 */
  uint32_t check_interval; /* re-try a unit with F = +infinity every this many
                              attempts that pass it over (0 = never) */
  ftv_tol tol;             /* the vote's tolerance */
} ftv_redundancy_cfg;

typedef struct ftv_redundancy_report {
  uint32_t attempts;       /* attempts started */
  int32_t verdict;         /* of the last vote; FTV_UNRESOLVED if none resolved */
  uint32_t timeouts;       /* runs abandoned at their deadline */
  uint32_t errors;         /* runs that reported a direct fault */
  uint32_t winner_unit;    /* unit of the vote's winner (resolved votes) */
  uint32_t reserved;
  double seconds;          /* wall time of the call */
} ftv_redundancy_report;

/* `impls` (nimpl >= 2) and `units` are HOST arrays; `units` is updated in
 * place.  `out` (device, n elements of cfg->dtype) receives the consensus of
 * the last vote and is complete when the call returns.  The votes use the
 * context's workspace on a stream of the library's own, so work the caller
 * enqueued with this context must have completed before the call.  Returns
 * FTV_OK also when no vote resolved (see rep->verdict); FTV_E_INVALID /
 * FTV_E_K / FTV_E_DTYPE on bad arguments, FTV_E_NOMEM, FTV_E_HIP.  Not
 * thread-safe per context. */
int ftv_run_redundant(ftv_ctx *ctx, const ftv_impl *impls, uint32_t nimpl, ftv_unit *units, uint32_t nunits,
                      const ftv_redundancy_cfg *cfg, uint64_t n, void *out, ftv_redundancy_report *rep);

/* ---- placement of the voter (Sec. IV-B, IV-D, V-A) -------------------------
 * The voter is a task like any other: the runtime keeps past runtimes per
 * problem size and past fault rates for each of its kernels and runs the one
 * with the lowest fault-aware runtime F = R / (1 - p) (see ftv_unit below);
 * the voter may itself be run redundantly, preferably on another device than
 * the one that computed the results.  Voter units: */
#define FTV_VOTER_HOST1 0  /* ftv_vote_host on one thread */
#define FTV_VOTER_HOSTMT 1 /* ftv_vote_host on the database's host threads */
#define FTV_VOTER_GPU 2    /* the MI355X voter (ftv_vote_mem: host replicas streamed in) */
#define FTV_NUM_VOTERS 3
#define FTV_PLACE_REDUNDANT 1u /* run a second voter and require identical results */

/* Performance database of the voter units: one profile (ftv_unit: runtime of
 * valid runs in seconds, valid runs, runs) per unit, size class (floor of
 * log2 of k * n * element size) and data placement (which replicas lie in
 * host memory, where the outputs go), plus pinned host and device staging for
 * the transfers.  check_interval: a unit whose runs for a key have all failed
 * (F = +infinity) is re-tried, as an extra run checked against the returned
 * result, after it has been passed over check_interval - 1 times for that key
 * (0 = never re-tried).  host_threads: threads of FTV_VOTER_HOSTMT (0 = all
 * cores).  Calls on one database are serialised.  Errors: FTV_E_INVALID,
 * FTV_E_NOMEM. */
typedef struct ftv_voter_db ftv_voter_db;
int ftv_voter_db_create(uint32_t check_interval, uint32_t host_threads, ftv_voter_db **out);
int ftv_voter_db_destroy(ftv_voter_db *db);
/* The profile of `unit` for a task of `bytes` replica bytes (k * n * element
 * size) with replicas r in host memory where bit r of host_mask is set and
 * outputs in out_memory; all zero if the unit never ran for that key. */
int ftv_voter_db_profile(ftv_voter_db *db, uint32_t unit, uint64_t bytes, uint32_t host_mask,
                         int32_t out_memory, ftv_unit *out);
/* Fault injection for tests of the fault handling: the next `count` runs of
 * `unit` return a corrupted result (one bit of consensus element 0 flipped, or
 * no_majority + 1 when there is no consensus output).  count = 0 clears it. */
int ftv_voter_db_inject(ftv_voter_db *db, uint32_t unit, uint32_t count);

typedef struct ftv_place_report {
  int32_t unit[3];        /* units that ran, in order; -1 = no run */
  uint32_t runs;          /* number of runs */
  int32_t result_unit;    /* unit whose result is in the caller's outputs */
  int32_t agreed;         /* FTV_PLACE_REDUNDANT: 1 if the first two voters agreed */
  uint32_t probed;        /* 1 if a unit with F = +infinity was re-tried */
  uint32_t reserved;
  double seconds[3];      /* wall time of each run, transfers included */
} ftv_place_report;

/* ftv_vote_placed -- one vote, run by the voter unit of lowest F for its size
 * class and data placement.  memory[r] (HOST array of k) says where
 * replicas[r] lies (FTV_MEM_HOST / FTV_MEM_DEVICE); consensus, mask and stats
 * lie in out_memory.  A unit's time is the wall time of its whole run: copies
 * of device replicas to the host for the host units, streaming of host
 * replicas for the GPU unit (ftv_vote_mem, 64 MiB pieces), and the copies of
 * the outputs to out_memory.  Every unit runs once per key before F decides
 * (a unit never run has no F).  Units in the bit set `avoid` (1 << unit) are
 * used only when no other is left -- e.g. the unit that computed the results.
 * A unit whose run fails directly (an error code) counts as a run that was
 * not valid and the next unit runs.  With FTV_PLACE_REDUNDANT a second unit,
 * on the other device than the first if possible, votes into the database's
 * staging and both results (consensus, mask and stats) must be identical;
 * if not, a third unit votes and the result two of them share is returned
 * (the odd unit's run counts as not valid); three different results return
 * FTV_E_MISMATCH.  Without the flag a run is valid unless it fails directly.
 * Synchronous: `stream` (a hipStream_t) carries the GPU work and the copies
 * and is synchronised before the call returns.  Errors: those of ftv_vote,
 * FTV_E_INVALID (memory flags, out_memory, flags, avoid), FTV_E_MISMATCH,
 * FTV_E_NOMEM, FTV_E_HIP. */
int ftv_vote_placed(ftv_ctx *ctx, ftv_voter_db *db, const ftv_vote_desc *desc, const int32_t *memory,
                    int32_t out_memory, uint32_t avoid, uint32_t flags, void *stream, ftv_place_report *rep);

#ifdef __cplusplus
}
#endif
#endif /* FTV_H */
