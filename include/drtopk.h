/* drtopk -- delegate-centric top-k and k-selection on AMD MI355X (gfx950).
 *
 * Implements the method of "Dr. Top-k: Delegate-Centric Top-k on GPUs"
 * (Gaihre et al., SC'21).  Problem statement (paper, Section 1): top-k returns
 * the k largest elements of an input vector V; k-selection returns the k-th
 * largest.  The method (Sections 4-5): cut V into subranges of 2^alpha
 * elements, keep the top-beta of each as delegates (Rules 1 and 3), take the
 * k-th largest delegate as a lower bound of the answer's k-th element (Rule 2),
 * skip every subrange that cannot reach it, and select among the survivors.
 *
 * Conventions fixed by this library where the paper is silent:
 *   - keys are uint32 (as the paper evaluates), int32, or float32, the latter
 *     ordered by IEEE 754 totalOrder (-NaN < -inf < ... < -0 < +0 < ... < +inf
 *     < +NaN); DRTOPK_SMALLEST asks for the k smallest instead;
 *   - among equal keys the lower position ranks first, so the answer is unique:
 *     out_vals is sorted by key descending, ties by ascending position, and
 *     out_vals[k-1] is the k-th largest counting multiplicity;
 *   - output values are the input's own bit patterns (NaN payloads and -0 kept).
 *
 * Memory: every key / output pointer is DEVICE memory owned by the caller.
 * The library keeps one workspace per (device, stream) that grows on demand
 * (freed by drtopk_release_workspace).  All calls are asynchronous on
 * `stream` (a hipStream_t; NULL means the default stream); outputs are valid
 * once the stream reaches that point.  Calls on different streams may run
 * concurrently.  No C++ exception crosses this interface.
 *
 * Errors are returned synchronously: DRTOPK_EINVAL for bad arguments (null
 * pointer, k == 0, k > n, n >= 2^32, unknown dtype), DRTOPK_ENOMEM when the
 * workspace cannot be allocated (nothing is launched), DRTOPK_EDEVICE when a
 * launch or device query fails.  Faults inside kernels surface at the next
 * synchronisation as HIP errors.  The kernels also run internal consistency
 * checks (a failure means a library defect, never bad input); a failed check
 * is recorded per (device, stream) and reported by drtopk_check, by the
 * calls that synchronise (stats, topk_select_host) and by the server.
 */
#ifndef DRTOPK_H
#define DRTOPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key types.  DRTOPK_SMALLEST may be OR-ed into any dtype argument or field:
 * the call then works on the k smallest keys (the paper's nearest-neighbour
 * and least-score uses, Section 6) -- out_vals ascending, ties by ascending
 * position, the k-th value the k-th smallest.  Everything else is the same.
 * 64-bit keys (DRTOPK_U64, DRTOPK_I64, DRTOPK_F64; float64 by totalOrder) are
 * 8 bytes each: keys and out_vals hold n and k 8-byte elements, out_kth one;
 * key pointers must be 8-byte aligned.  They run one delegate per subrange
 * (beta = 1) or the plain radix select; the per-call functions below take
 * them unless their comment says otherwise. */
typedef enum {
  DRTOPK_U32 = 0,
  DRTOPK_F32 = 1,
  DRTOPK_I32 = 2,
  DRTOPK_U64 = 3,
  DRTOPK_I64 = 4,
  DRTOPK_F64 = 5,
  DRTOPK_SMALLEST = 0x100
} drtopk_dtype_t;

typedef enum {
  DRTOPK_OK = 0,
  DRTOPK_EINVAL = 1,
  DRTOPK_ENOMEM = 2,
  DRTOPK_EDEVICE = 3,
  DRTOPK_EUNSUPPORTED = 4,
  DRTOPK_ESCRATCH = 5 /* topk_select_noalloc: the call needs more than its fixed workspace */
} drtopk_status_t;

/* Top-k (paper, Section 1).
 *   keys     device, n elements of `dtype` (4 bytes each); any alignment
 *            (16-byte aligned input takes the 128-bit load path)
 *   n        1 <= n < 2^32
 *   k        1 <= k <= n
 *   out_vals device, k elements of `dtype`: the k largest, sorted as above
 *   out_idx  device, k uint32 positions into keys (out_vals[r] == keys[out_idx[r]]),
 *            or NULL
 *   stream   hipStream_t or NULL */
int topk_select(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals,
                uint32_t* out_idx, void* stream);

/* topk_select for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, results (bit for bit) and kernels as topk_select, but the
 * workspace is a fixed device array of 128 MiB built into the library, one
 * copy per device, held until the process ends; the call allocates nothing.
 * Its first call on a device (with that device current) looks the array up
 * and synchronises the device once: make that call outside graph capture.
 *   - DRTOPK_ESCRATCH, with nothing enqueued, if the call's workspace exceeds
 *     the array (the workspace is drtopk_footprint(n, k, dtype) minus the
 *     4n + 8k + 4 bytes of input and outputs): at n = 2^30 it fits up to
 *     k = 1024, at n = 2^26 up to k = 16384, and for n <= 2^22 every k fits.
 *   - Every call on a device shares that device's array, which keeps the last
 *     call's contents; each call clears what it needs.  Calls whose work
 *     overlaps on one device (other streams, other host threads) race and
 *     give wrong results: order them on one stream or with events.
 *   - Failed internal checks are recorded on the device and reported by the
 *     next drtopk_check on the device (on any stream, once the calls
 *     concerned have finished; calling it on the calls' stream ensures that).
 * Other errors as topk_select. */
int topk_select_noalloc(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals, uint32_t* out_idx,
                        void* stream);

/* k-selection (paper, Section 1): writes the k-th largest value (1 element of
 * `dtype`, device memory) to out_kth.  Same argument rules as topk_select. */
int kth_select(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_kth, void* stream);

/* One problem of a batch.  All pointers are device memory; out_vals/out_idx
 * hold k elements, out_kth one element; out_idx and out_kth may be NULL. */
typedef struct {
  const void* keys;
  uint64_t n;
  uint32_t k;
  uint32_t dtype;
  void* out_vals;
  uint32_t* out_idx;
  void* out_kth;
} drtopk_problem_t;

/* Many independent top-k problems (the paper's Section 1 problem, applied to
 * each).  `problems` is a HOST array of `count` descriptors, read during the
 * call (the caller may reuse it on return).  Each problem obeys topk_select's
 * rules, except that out_vals may be NULL when out_kth is not (k-selection
 * only).  Results equal topk_select / kth_select on each problem alone, bit
 * for bit.  Problems with n <= 2^22 and k <= 2048 run in one persistent
 * launch, one workgroup per problem at a time, largest first (the delegate
 * method of Sections 4-5 inside the workgroup's LDS); larger ones run one
 * after another through the single-problem path, on the same stream.  Any
 * invalid descriptor, or count >= 2^24, fails the whole call with
 * DRTOPK_EINVAL before any work is enqueued.  Problems of more than 2^16 keys
 * on the delegate route may have their delegate vector built by several
 * workgroups.  Output buffers of different problems must not overlap. */
int topk_select_batched(const drtopk_problem_t* problems, uint32_t count, void* stream);

/* Autotuner table (Rule 4's subrange size and Rule 3's beta, measured rather
 * than modelled).  An entry applies to problems of one form whose
 * floor(log2 n) and floor(log2 k) equal lg_n and lg_k:
 *   form 0 (DRTOPK_FORM_SINGLE): topk_select / kth_select planning, alpha and
 *          beta as in drtopk_options_t (explicit options still win);
 *   form 1 (DRTOPK_FORM_BATCHED): the subrange exponent and delegates per
 *          subrange (beta 2; any other value means 1) of a batched problem
 *          (the planner raises alpha until the delegate vector, S * beta
 *          entries, fits the workgroup's LDS or, for a problem split across
 *          workgroups, its global buffer).
 * Problems with no entry use Rule 4 (const 3).  drtopk_tune_set replaces the
 * whole table (count 0 clears it); entries are validated (alpha 0..24, beta
 * 1/2/4/8) and copied.  The table is process-wide. */
enum { DRTOPK_FORM_SINGLE = 0, DRTOPK_FORM_BATCHED = 1 };
typedef struct {
  int32_t form;
  int32_t lg_n;
  int32_t lg_k;
  int32_t alpha;
  int32_t beta;
} drtopk_tune_t;
int drtopk_tune_set(const drtopk_tune_t* entries, uint32_t count);
/* Copies up to `cap` entries to `out` (host) and the table size to *count. */
int drtopk_tune_get(drtopk_tune_t* out, uint32_t cap, uint32_t* count);

/* How a batched problem of this shape is run (no device work):
 *   *route 0 = single-problem path, 1 = sorted outright in the workgroup,
 *          2 = delegate method in the workgroup with subrange exponent
 *          *alpha and *beta delegates per subrange (1 or 2; beta may be
 *          NULL), 3 = workgroup radix select without delegates.
 * Route 2 falls back to route 3 on the device when the survivors of an
 * input exceed the workgroup's capacity (4096). */
int drtopk_batched_alpha(uint64_t n, uint32_t k, int32_t* route, int32_t* alpha, int32_t* beta);

/* Explicit method parameters (for tests, tuning and ablations).
 *   alpha  subrange = 2^alpha elements (Section 5.1), at most 24; -1 = planner's choice
 *   beta   delegates per subrange (Rule 3): 1, 2, 4 or 8; 0 = planner's choice
 *   mode   0 = planner's choice, 1 = delegate method, 2 = plain radix select
 *          over V with no delegates, 3 = the whole problem in one workgroup
 *          (the batched form's kernel, one launch; n <= 2^22, k <= 2048; the
 *          planner takes it for n <= 2^16; alpha is then the batched form's)
 *   variant  implementation of the steps after the delegate pass, i.e. the
 *          top-k algorithm the delegates assist (Sections 5.1 and 6.1):
 *          0 = one cooperative kernel (default: histogram cut, survivors
 *          bucketed and sorted), 1 = one kernel per step with MSD radix
 *          selects, 2 = bitonic top-k for both selections (k <= 256, else
 *          DRTOPK_EINVAL), 3 = bucket select (equal-width buckets over the
 *          live min..max range) for both selections.  All give bit-identical
 *          results; 32-bit keys only (64-bit keys take 0 or 1, same path). */
typedef struct {
  int32_t alpha;
  int32_t beta;
  int32_t mode;
  int32_t variant;
} drtopk_options_t;

/* Counters of one call (host struct, filled after the call's work finishes;
 * passing non-NULL makes the call synchronise `stream`). */
typedef struct {
  int32_t mode;          /* 1 delegate method, 2 plain radix select, 3 one workgroup
                            (then only alpha, beta, subranges, delegates are set) */
  int32_t alpha, beta;
  uint64_t subranges;    /* S = ceil(n / 2^alpha) */
  uint64_t delegates;    /* |D| = S * beta */
  uint64_t scanned;      /* subranges re-read after the threshold */
  uint64_t candidates;   /* survivors handed to the second select */
  uint32_t t_key_bits;   /* the filter's threshold (Rule 2): the k-th delegate, or a
                            composite ranked at or below it; input bit pattern */
  uint32_t t_idx;        /* its position (a bound, possibly past n, when the
                            threshold is not an element) */
  /* completion time of each step after the delegate pass, in ns since that
   * part started (device clock; 0 = step not run), default variant:
   * [0] refined threshold, [1] Rule 3 over the delegates, [2] re-read,
   * [3] output sorted by one workgroup, [4] output buckets counted,
   * [5] scattered, [6] bucket groups sorted, [7..12] select passes (tie
 * fallback), [13] exact compaction, [14] fallback sort, [15..19] the first
 * five digit passes of the delegate select (massive ties at the threshold;
 * the key digits are skipped when the bin holding t is one key) */
  uint32_t step_ns[20];
  uint32_t err_flags;    /* internal consistency checks that failed (0 = none) */
} drtopk_stats_t;

/* topk_select with explicit options (NULL = defaults) and optional stats. */
int topk_select_ex(const void* keys, uint64_t n, uint32_t k, int dtype, void* out_vals,
                   uint32_t* out_idx, const drtopk_options_t* opt, drtopk_stats_t* stats,
                   void* stream);

/* The delegate vector alone (Rules 1 and 3) for stage-by-stage checks:
 * writes S * beta entries, S = ceil(n / 2^alpha): out_dkeys[s*beta + j] is the
 * j-th delegate's value (input bit pattern) and out_didx[s*beta + j] its
 * position, rows ordered by key descending then position ascending; a
 * subrange with fewer than beta elements pads with position 0xFFFFFFFF.
 * alpha in [0, 24], beta in {1, 2, 4, 8}; device buffers. */
int drtopk_delegates(const void* keys, uint64_t n, int dtype, int alpha, int beta,
                     void* out_dkeys, uint32_t* out_didx, void* stream);

/* The survivors of the filter for given alpha/beta (Rules 1-3): writes their
 * positions (unordered) to out_pos (device, capacity `cap` entries), their
 * count to *count, and the threshold the filter used to t_out (host, 2 words,
 * nullable): its key (input bit pattern) and its position; synchronises
 * `stream`.  Survivors are exactly the elements ranked at or above that
 * threshold (key greater, or key equal and position not greater).  With
 * variant 1 the threshold is the exact k-th delegate t; with variant 0 it is
 * usually a key t' <= t read off the delegate histogram (position 0xFFFFFFFF:
 * every element with key >= t').  DRTOPK_EINVAL if cap is too small. */
int drtopk_candidates(const void* keys, uint64_t n, uint32_t k, int dtype, int alpha, int beta, int variant,
                      uint32_t* out_pos, uint64_t cap, uint64_t* count, uint32_t* t_out, void* stream);

/* The planner's choice for a problem (no device work). */
int drtopk_plan(uint64_t n, uint32_t k, int dtype, drtopk_options_t* out);

/* Phase timing with HIP events, for measurement runs.  While enabled, every
 * top-k call records events on its own stream around the delegate pass (the
 * one pass that streams all of V) and around everything after it.
 * drtopk_timing_read synchronises on those events, returns the summed
 * milliseconds of each phase and the number of calls since the last read,
 * and resets the counters.  Enabling costs two event pairs per call. */
int drtopk_timing_enable(int on);
int drtopk_timing_read(double* delegate_ms, double* tail_ms, uint64_t* calls);

/* HBM bytes a problem occupies while it is in flight: its input (4n), its
 * outputs (8k + 4) and the workspace of the route it takes.  The serving loop
 * admits requests by this figure.  DRTOPK_EINVAL for arguments topk_select
 * would reject. */
int drtopk_footprint(uint64_t n, uint32_t k, int dtype, uint64_t* bytes);

/* Serving loop: continuous batching of requests over device-resident arrays
 * (each request is a drtopk_problem_t: device pointers, the caller keeps them
 * alive until the request completes).  A server owns `streams` launch streams
 * and one dispatcher thread.  Whenever a stream is free, the dispatcher looks
 * at the oldest queued request: one that a workgroup cannot own (n > 2^22 or
 * k > 2048) is launched alone through the single-problem path; otherwise the
 * queued small requests are admitted in arrival order while the summed
 * footprint of admitted, unfinished requests stays within hbm_budget (a
 * request larger than the budget is admitted alone), at most max_batch per
 * launch, and launched together with topk_select_batched on that stream (a
 * launch of one request calls topk_select directly).  Requests arriving while
 * launches run join the next launch, so their work overlaps on the device.
 * Results are bit-identical to topk_select / kth_select on each request
 * alone.  plain = 1 turns the server into the per-request baseline: one
 * topk_select (or kth_select) call per request, in arrival order.
 * A launch whose kernels raise an internal check flag (see drtopk_check)
 * completes all of its requests with DRTOPK_EDEVICE.
 * The device is the caller's current device at creation.  A server keeps a
 * record (about 100 bytes) of every request until a drain reports it. */
typedef struct drtopk_server drtopk_server_t;
typedef struct {
  uint64_t hbm_budget; /* bytes; 0 = 8 GiB */
  uint32_t max_batch;  /* >= 1 */
  uint32_t streams;    /* 1..16, default priority */
  uint32_t plain;      /* 0 batched server, 1 per-request baseline */
  uint32_t reserved;   /* 0 */
} drtopk_server_config_t;
typedef struct {
  uint64_t completed;          /* latencies recorded since the last reset */
  uint64_t launches;           /* launches since the last reset */
  uint64_t launched_items;     /* requests in those launches */
  uint64_t max_inflight_bytes; /* peak admitted footprint */
  double mean_us, p50_us, p99_us, max_us; /* arrival -> completion seen by the host */
} drtopk_server_stats_t;
int drtopk_server_create(const drtopk_server_config_t* cfg, drtopk_server_t** out);
/* Queues one request (arrival = now); *ticket identifies it. */
int drtopk_server_submit(drtopk_server_t* server, const drtopk_problem_t* req, uint64_t* ticket);
/* Blocks until the request completes; returns its status and, if non-NULL,
 * its latency in microseconds.  DRTOPK_EINVAL for a ticket never issued or
 * already reported by a drain. */
int drtopk_server_wait(drtopk_server_t* server, uint64_t ticket, double* latency_us);
/* Blocks until every submitted request has completed; returns a failure
 * status among the requests completed since the previous drain, else OK, and
 * drops their records (their tickets are no longer valid for wait). */
int drtopk_server_drain(drtopk_server_t* server);
/* Latency percentiles (nearest rank) over requests completed since the last
 * reset; reset != 0 starts a new window. */
int drtopk_server_stats(drtopk_server_t* server, drtopk_server_stats_t* out, int reset);
/* Open-loop load: submits reqs[i] at arrival_us[i] (non-decreasing, from the
 * call's start) from the calling thread, waits for all, and writes each
 * request's latency (from its scheduled arrival) to latency_us[i] and the
 * wall time of the whole replay to *elapsed_us (either may be NULL). */
int drtopk_server_replay(drtopk_server_t* server, const drtopk_problem_t* reqs, const double* arrival_us,
                         uint32_t count, double* latency_us, double* elapsed_us);
/* Finishes queued work, stops the dispatcher and frees the server.  No other
 * call on this server may run concurrently with or after it.  If the
 * dispatcher runs out of host memory, every unfinished request completes with
 * DRTOPK_ENOMEM and later submits return DRTOPK_ENOMEM. */
int drtopk_server_destroy(drtopk_server_t* server);

/* Top-k of keys that carry a payload (key-value pairs; the paper's own
 * selections run on (key, value) pairs, Section 5.1): as topk_select, plus
 * out_payload[r] = payload[out_idx[r]] for every output slot r.
 *   payload      device, n elements of payload_bytes (4 or 8) each
 *   out_payload  device, k elements of payload_bytes
 *   out_idx      may be NULL (the positions are then kept in the stream's
 *                workspace; no per-call allocation)
 * Errors as topk_select; DRTOPK_EINVAL for another payload_bytes or a null
 * payload / out_payload. */
int topk_select_payload(const void* keys, uint64_t n, uint32_t k, int dtype, const void* payload,
                        int payload_bytes, void* out_vals, uint32_t* out_idx, void* out_payload, void* stream);

/* Top-k over keys in HOST memory, streamed through the device in chunks: for
 * inputs larger than the device memory (the paper's reload of sub-vectors
 * that do not fit one GPU, Section 5.4).  Each chunk's top-k (positions
 * offset to the whole input) is merged with the running top-k by a top-k over
 * the two lists (running list first: it holds the lower positions, so the tie
 * rule carries over); copies of the next chunk overlap the current chunk's
 * selection (two device buffers, a copy stream of default priority).
 *   host_keys  host memory (pageable or pinned), n keys of `dtype`
 *   n, k, dtype as for topk_select (DRTOPK_SMALLEST allowed)
 *   chunk      keys per transfer; 0 = min(n, 2^26); at most n
 *   out_vals / out_idx  device memory, as for topk_select (out_idx may be NULL)
 * Allocates device buffers for two chunks and the candidate lists, and
 * returns once the result is complete (it synchronises `stream`), so the
 * host buffer may be reused on return.  DRTOPK_EINVAL on bad arguments,
 * DRTOPK_ENOMEM if the buffers cannot be allocated, DRTOPK_EDEVICE if a copy
 * or launch fails or the stream's check record holds flags at the end (they
 * stay recorded for drtopk_check). */
int topk_select_host(const void* host_keys, uint64_t n, uint32_t k, int dtype, uint64_t chunk, void* out_vals,
                     uint32_t* out_idx, void* stream);

/* Measurement helper: reads keys[0 .. n - n mod 2^20) once with the delegate
 * pass's access pattern and launch geometry (4 MiB per workgroup, 16-byte
 * non-temporal loads, eight in flight per lane) and writes their maximum to
 * *out_max (device).  Timing it gives the read bandwidth that pattern reaches
 * on the device, the practical ceiling of the delegate pass.  keys 16-byte
 * aligned, 2^20 <= n < 2^32; else DRTOPK_EINVAL. */
int drtopk_read_probe(const void* keys, uint64_t n, uint32_t* out_max, void* stream);

/* Frees the calling thread's current device's workspaces (synchronises it). */
int drtopk_release_workspace(void);

/* Internal check flags (bits of *flags):
 *   1   a radix-select bucket search found no bucket holding the sought rank
 *   2   fewer survivors than k reached the output step
 *   16  a bounded buffer was full and writes past its end were dropped
 *   64  a phase wait inside a kernel gave up after about one second
 *   128 an output sort group exceeded one workgroup
 * Any of them means the outputs of the calls concerned are not to be trusted. */
enum {
  DRTOPK_CHECK_SELECT = 1,
  DRTOPK_CHECK_FEW = 2,
  DRTOPK_CHECK_CAPACITY = 16,
  DRTOPK_CHECK_WAIT = 64,
  DRTOPK_CHECK_GROUP = 128
};

/* Synchronises `stream`, then reports and clears the check flags recorded by
 * the kernels of every call enqueued on it (on the current device) since the
 * previous drtopk_check of that stream, together with those recorded by
 * topk_select_noalloc calls on the device: DRTOPK_OK and *flags = 0 if none,
 * DRTOPK_EDEVICE with the OR of the flags otherwise (flags may be NULL).
 * DRTOPK_EDEVICE with *flags = 0 if the synchronisation itself fails. */
int drtopk_check(void* stream, uint32_t* flags);

/* Testing hook for the error path: caps the survivor buffers of the delegate
 * method (topk_select, kth_select, and the single-problem part of the other
 * entry points) at `cap` entries for calls planned after it; 0 restores the
 * planner's bound.  With a cap below what an input needs, kernels drop the
 * writes past it, raise flag 16 (and usually 2) and exit normally.
 * Process-wide; not for production use. */
int drtopk_set_survivor_cap(uint64_t cap);

/* Human-readable name of a status code (static string). */
const char* drtopk_status_string(int status);

/* Library version string. */
const char* drtopk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DRTOPK_H */
