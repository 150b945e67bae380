/*
 * wrs.h -- C ABI of an MI355X (gfx950) implementation of the data-parallel hot
 * path of weighted random sampling from Huebschle-Schneider & Sanders,
 * "Parallel Weighted Random Sampling" (arXiv 1903.00227).
 *
 * Problems (Section 1): items 0..n-1 with weights w_i >= 0, W = sum of w_i.
 *   - alias table construction (Section 2.2 defines the table; Section 4.2 and
 *     Algorithm 3 split the sweep of Section 4.1 into independent pieces;
 *     Section 4.2.1 takes greedy blocks first; Section 4.4 builds 2-level
 *     tables);
 *   - sampling with replacement (problem WRS-R): k independent alias queries,
 *     or output-sensitively (Section 5): the distinct items drawn with their
 *     multiplicities;
 *   - sampling without replacement (problem WRS-N) with exponential clocks
 *     (Section 2.3): the k items with the smallest -ln(u_i)/w_i;
 *   - weighted random permutation (problem WRP, Section 7): all items in the
 *     order of those keys.
 *
 * Conventions for every call:
 *   - Pointers named d_* are device pointers (HIP global memory of the current
 *     device); h_* are host pointers.  The caller owns all of them; the library
 *     never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous and ordered on that stream unless stated otherwise.
 *   - Host-detectable errors are returned immediately and nothing is launched.
 *     Errors found on the device (a weight that is negative, NaN or infinite, a
 *     zero total) are written to a status word inside the caller's workspace and
 *     read with wrs_status(); outputs are unspecified then.
 *   - Items are 0-based; n is limited to 2^31 - 1 (indices are int32).
 *   - Random bits come from Philox-4x32-10 (Salmon et al., SC'11), keyed by
 *     `seed`; a draw is a pure function of (seed, stream_id, counter), so results
 *     do not depend on launch shapes, batching or the order of calls.
 */
#ifndef WRS_H
#define WRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One bucket of an alias table, 8 bytes, array-of-structs (the paper's
 * experiments store tables this way, Section 10.1).  Bucket r returns item r
 * with probability t and item `alias` otherwise (Section 2.2). */
typedef struct {
    float t;
    int32_t alias;
} wrs_entry;

enum {
    WRS_OK = 0,
    WRS_EINVAL = -1,    /* null pointer, n < 1, n > 2^31-1, k < 0, workspace too small */
    WRS_EDOMAIN = -2,   /* weight < 0, NaN or Inf; W == 0; WOR with k > #positive weights */
    WRS_ENOMEM = -3,    /* an allocation inside the library failed (server only) */
    WRS_EDEVICE = -4,   /* a HIP call failed; wrs_last_error() has the text */
    WRS_EBUSY = -5,     /* server: request not finished / table in use */
    WRS_ENOTFOUND = -6  /* server: unknown table or request id */
};

enum { WRS_OP_BUILD = 1, WRS_OP_WOR = 2, WRS_OP_BUILD_PLUS = 3, WRS_OP_PERM = 4, WRS_OP_TWOLEVEL = 5,
       WRS_OP_OS = 6 };

/* Items per block (meta-item) of the 2-level tables (part of their layout). */
#define WRS_TWOLEVEL_BLOCK 2048

/* Items per greedy block of wrs_alias_build_plus (part of its result). */
#define WRS_PSAPLUS_BLOCK 2048

/* Bytes of device workspace needed by wrs_alias_build (op = WRS_OP_BUILD, k
 * ignored), wrs_alias_build_plus (op = WRS_OP_BUILD_PLUS, k ignored),
 * wrs_sample_wor (op = WRS_OP_WOR), wrs_permutation (op = WRS_OP_PERM, k
 * ignored), wrs_twolevel_build (op = WRS_OP_TWOLEVEL, k ignored) or
 * wrs_os_build and wrs_os_sample (op = WRS_OP_OS; k = the largest sample the
 * workspace serves, 0 for a build only).  Depends on n (and k) only.
 * Returns 0 for invalid arguments. */
size_t wrs_workspace_bytes(int op, int64_t n, int64_t k);

/* Build an alias table (Section 2.2) for d_w[0..n) into d_table[0..n).
 * Method: the sweeping construction of Section 4.1 split into independent
 * pieces as in Section 4.2 (Algorithm 3) with block-wise prefix sums
 * (Section 4.2.2); all sums are exact integers on a grid derived from W, so
 * the table equals the sequential sweep's table whenever every weight is at
 * least 2^-40 of the mean weight (always for the paper's input families).
 * d_w: n FP32 weights (device, any alignment).  d_table: n entries (device,
 * 8-byte aligned).  d_ws: wrs_workspace_bytes(WRS_OP_BUILD, n, 0) bytes
 * (device, 256-byte aligned).  The workspace afterwards holds the status word
 * and the total weight (wrs_total_weight). */
int wrs_alias_build(const float* d_w, int64_t n, wrs_entry* d_table,
                    void* d_ws, size_t ws_bytes, void* stream);

/* ---- building without allocation ------------------------------------------ */

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): wrs_alias_build with its
 * workspace in a fixed device array of WRS_NOALLOC_SCRATCH_BYTES bytes that
 * the library holds on every GPU it runs on, until the process ends, instead
 * of caller memory.  Same table as wrs_alias_build.  n must satisfy
 * wrs_workspace_bytes(WRS_OP_BUILD, n, 0) <= WRS_NOALLOC_SCRATCH_BYTES (about
 * 2.2e7 items), else WRS_EINVAL and nothing is launched.  d_status (optional,
 * device, 4-byte aligned): receives the build's status word (WRS_OK or
 * WRS_EDOMAIN) on the stream.  The call allocates nothing and does not
 * synchronise.  Every call on one GPU uses that GPU's array and leaves its
 * contents there: calls that overlap on one GPU (streams not ordered against
 * each other, or other threads) race. */
#define WRS_NOALLOC_SCRATCH_BYTES (128u << 20)
int wrs_alias_build_noalloc(const float* d_w, int64_t n, wrs_entry* d_table, int32_t* d_status, void* stream);

/* Build an alias table with greedy blocks first (Section 4.2.1, PSA+).  The
 * items are cut into consecutive blocks of WRS_PSAPLUS_BLOCK items; inside
 * each block the sweep of Section 4.1 runs on the block's own items until the
 * block runs out of light or of heavy items, and what it packed is final.
 * The items left (the heavy each block stopped at, with the part of its size
 * not yet placed, and the untouched items) then go through the splitting
 * construction of wrs_alias_build, in index order.  The table differs from
 * wrs_alias_build's; it is the sequential definition of this two-stage
 * construction in the same exact grid arithmetic.
 * Arguments as for wrs_alias_build, with d_ws of
 * wrs_workspace_bytes(WRS_OP_BUILD_PLUS, n, 0) bytes.  The call blocks the
 * calling thread until the greedy stage has run on the stream (it sizes the
 * second stage from the number of items left), so it cannot be captured in a
 * graph; the second stage is queued on the stream when the call returns.
 * Device-side errors (weight domain) are reported through wrs_status. */
int wrs_alias_build_plus(const float* d_w, int64_t n, wrs_entry* d_table,
                         void* d_ws, size_t ws_bytes, void* stream);

/* Weighted random permutation (problem WRP, Sections 1 and 7): d_out[0..n)
 * receives every item once, in the order of the sequential process of
 * sampling without replacement run to k = n.  Exponential clocks (Section
 * 2.3): item i has key -ln(u_i)/w_i with u_i from the same Philox counters as
 * wrs_sample_wor (so d_out[0..k) as a set is wrs_sample_wor's sample of size
 * k), keys ascending, ties by the smaller index; zero-weight items come last,
 * in index order.  d_w: n FP32 weights >= 0 (device).  d_out: n int32
 * (device, 4-byte aligned).  d_ws: wrs_workspace_bytes(WRS_OP_PERM, n, 0)
 * bytes (device, 256-byte aligned; about 25 bytes per item).  A negative, NaN
 * or infinite weight sets the workspace status to WRS_EDOMAIN (wrs_status);
 * d_out is then unspecified. */
int wrs_permutation(const float* d_w, int64_t n, uint64_t seed, uint32_t stream_id, int32_t* d_out,
                    void* d_ws, size_t ws_bytes, void* stream);

/* Output-sensitive sampling with replacement (Section 5): a sample of k draws
 * returned as the s distinct items drawn with their multiplicities, in
 * expected work O(s + log n) after a build.
 * Structure: the items with w > 0 are grouped by binary exponent (weights
 * within a factor of two; groups heaviest first, items of a group by index);
 * a divide-and-conquer tree over the groups and one over each group's items
 * split a node asked for m draws by a binomial variate (always in the top
 * tree, at m >= 2 inside a group), and a group node asked for one draw takes
 * it from the group's bucket table by rejection.  A node over [lo, hi) splits
 * at floor((lo + hi)/2).  The draws of node h are the Philox-4x32-10 counter
 * blocks (h mod 2^32, h >> 32, tag, attempt) under key `seed`, tag = the group's
 * position or 0xFFFFFFFF in the top tree; binomial variates by inversion below
 * mean 10, else by transformed rejection (BTRS), both in IEEE basic operations,
 * so results are a pure function of (weights, k, seed).
 * Bytes of the structure for n items (about 12 per item); 0 if n is out of
 * range. */
size_t wrs_os_bytes(int64_t n);

/* Build the structure for d_w[0..n) (FP32 weights, device) into d_os
 * (wrs_os_bytes(n) bytes, device, 256-byte aligned; it holds no pointer, so it
 * may be copied or moved).  d_ws: wrs_workspace_bytes(WRS_OP_OS, n, 0) bytes
 * or more (device, 256-byte aligned), free again when the build has run.  The
 * call blocks the calling thread until its first pass over the weights has run
 * on the stream: it reads back one flag to sort by one 8-bit digit of the
 * group key, or by two when a weight is zero or below 2^-128.  So it cannot be
 * captured in a graph.  A negative, NaN or infinite weight, or no positive
 * weight, sets the structure's status (wrs_status(d_os)) to WRS_EDOMAIN. */
int wrs_os_build(const float* d_w, int64_t n, void* d_os, size_t os_bytes, void* d_ws, size_t ws_bytes,
                 void* stream);

/* Draw k (0 <= k <= 2^31 - 1) items with replacement from a built structure
 * of n items, seed `seed`.  Writes the s distinct items drawn to d_items and
 * their multiplicities (>= 1, summing to k) to d_counts, in no particular
 * order, and s to *d_s (device int64).  d_items, d_counts: min(k, n) int32
 * each (device, 4-byte aligned).  d_ws: wrs_workspace_bytes(WRS_OP_OS, n, k)
 * bytes (device, 256-byte aligned); its status word (wrs_status(d_ws)) is
 * the structure's build status, WRS_EINVAL if the structure was built for
 * another n, or WRS_EDEVICE if a bound that the method never reaches was
 * reached; *d_s is 0 unless the status is WRS_OK. */
int wrs_os_sample(const void* d_os, int64_t n, int64_t k, uint64_t seed, int32_t* d_items, int32_t* d_counts,
                  int64_t* d_s, void* d_ws, size_t ws_bytes, void* stream);

/* Build a 2-level alias table (Section 4.4, replicated top level).  The items
 * are cut into blocks of WRS_TWOLEVEL_BLOCK consecutive items; block g is a
 * meta-item whose weight is the sum of its items' weights.  d_table[0..n)
 * receives every block's own alias table (the sweep of Section 4.1 with the
 * block as the instance; aliases are global item indices), and
 * d_top[0..G), G = ceil(n / WRS_TWOLEVEL_BLOCK), the alias table over the
 * meta-items (the splitting construction of wrs_alias_build).  A block of
 * total weight 0 keeps t = 1, alias = self and is never drawn.  A block far
 * lighter than the total (its sum below 2^40 units of the items' grid) builds
 * its table on a grid of its own and gives its meta-item a light threshold
 * from its size as a double, so every positive weight keeps its probability
 * within 1e-6 relative.  d_w: n FP32
 * weights (device).  d_table, d_top: device, 8-byte aligned.  d_ws:
 * wrs_workspace_bytes(WRS_OP_TWOLEVEL, n, 0) bytes (device, 256-byte aligned,
 * about 0.1 byte per item plus a fixed part).  Stream-ordered, no host wait
 * (graph-capturable).  Domain errors go to the workspace status word. */
int wrs_twolevel_build(const float* d_w, int64_t n, wrs_entry* d_table, wrs_entry* d_top,
                       void* d_ws, size_t ws_bytes, void* stream);

/* k draws from a 2-level table: draw s (counter c = first_counter + s) picks
 * block g by the query of wrs_alias_sample over the G top-level buckets with
 * Philox counter (c lo, c hi, stream_id, 0), then the item by the same query
 * over the block's m items with Philox counter (c lo, c hi, stream_id, 2).
 * Each draw reads the top table (small: L2-resident) and one block entry. */
int wrs_twolevel_sample(const wrs_entry* d_top, const wrs_entry* d_table, int64_t n, uint64_t seed,
                        uint32_t stream_id, uint64_t first_counter, int64_t k, int32_t* d_out, void* stream);

/* After wrs_alias_build_plus on this workspace: the number of items its
 * greedy blocks left to the splitting stage (0 if the weights were rejected).
 * Synchronizes the stream, then reads one device word. */
int wrs_plus_leftovers(const void* d_ws, void* stream, int64_t* nleft);

/* Draw k samples with replacement from a table: d_out[s] = query at counter
 * c = first_counter + s, for s in [0, k).  One Philox block per draw with
 * key = seed and counter = (c low 32 bits, c high 32 bits, stream_id, 0):
 * bucket r = floor((x1 2^32 + x0) n / 2^64), coin u = (x2 >> 8) 2^-24, result
 * r if u < t_r else alias_r (Section 2.2 query; branch-free select as in
 * Section 10).  d_table: n entries with t in [0,1] and alias in [0,n) (the
 * kernel trusts the table).  d_out: k int32 (device). */
int wrs_alias_sample(const wrs_entry* d_table, int64_t n, uint64_t seed, uint32_t stream_id,
                     uint64_t first_counter, int64_t k, int32_t* d_out, void* stream);

/* Sample k distinct items without replacement (problem WRS-N, Section 1) by
 * exponential clocks (Section 2.3): u_i = (x_j + 1) 2^-32 from word j = i mod 4
 * of the Philox block with counter (g low, g high, stream_id, 1), g = floor(i / 4),
 * key_i = -ln(u_i) / w_i (FP64), and the
 * k smallest keys, ties broken by the smaller index, win.  d_out receives the
 * k indices in ascending order.  Requires 0 <= k and, on the device, k <= the
 * number of positive weights (else status WRS_EDOMAIN).  d_ws:
 * wrs_workspace_bytes(WRS_OP_WOR, n, k) bytes. */
int wrs_sample_wor(const float* d_w, int64_t n, int64_t k, uint64_t seed, uint32_t stream_id,
                   int32_t* d_out, void* d_ws, size_t ws_bytes, void* stream);

/* Synchronise `stream` and read the device status word of a workspace used by
 * wrs_alias_build, wrs_alias_build_plus, wrs_sample_wor or wrs_permutation.
 * *status_out is WRS_OK or an error code. */
int wrs_status(const void* d_ws, void* stream, int* status_out);

/* Synchronise `stream` and read the total weight W found by the last
 * wrs_alias_build on this workspace, as an unevaluated pair hi + lo. */
int wrs_total_weight(const void* d_ws, void* stream, double* hi, double* lo);

/* ---- batched operation -------------------------------------------------- */

/* One independent table: build from d_w[0..n) into d_table, then draw k
 * samples into d_out exactly as wrs_alias_sample(d_table, n, seed, stream_id,
 * 0, k, d_out) would.  k may be 0 (build only). */
typedef struct {
    const float* d_w;
    int64_t n;
    wrs_entry* d_table;
    int64_t k;
    uint64_t seed;
    uint32_t stream_id;
    int32_t* d_out;
} wrs_job;

/* Workspace for a batch (device bytes); depends on the jobs' n only. */
size_t wrs_batch_workspace_bytes(const wrs_job* h_jobs, int32_t njobs);

/* Build and sample all jobs with one launch per phase for the whole batch
 * (all tables share each launch).  Every job's table and samples are
 * bit-identical to a single wrs_alias_build + wrs_alias_sample of that job.
 * The descriptors are copied to the workspace, so h_jobs may be reused when
 * the call returns.  The first call for a given batch shape records the
 * launches into a hipGraph that later calls with identical descriptors replay
 * (see wrs_batch_graph_mode). */
int wrs_batch_build_sample(const wrs_job* h_jobs, int32_t njobs, void* d_ws, size_t ws_bytes,
                           void* stream);

/* Per-job status after a batch: synchronises `stream`, copies njobs status
 * words into h_status. */
int wrs_batch_status(const void* d_ws, int32_t njobs, void* stream, int* h_status);

/* 1 (default): wrs_batch_build_sample records its launches once into a
 * hipGraph per distinct batch (same descriptors and workspace) and replays it;
 * 0: plain stream launches every call. */
int wrs_batch_graph_mode(int enable);

/* Small tables in one persistent launch: with max_n > 0, every job of a batch
 * with n <= max_n is built and sampled by one workgroup, in one launch for all
 * such jobs beside the phase launches of the others; the workgroup runs the
 * construction's phases one after another and draws the samples from the
 * finished table copied into LDS (WRS_FUSE_MAX_N items at most).  Tables and
 * samples are the same bits as without it.  0 (default) gives every job to the
 * phase launches, which measure faster on the batches this library is timed
 * on.  WRS_EINVAL for max_n outside [0, WRS_FUSE_MAX_N].  Per process. */
#define WRS_FUSE_MAX_N 8192
int wrs_batch_fuse_small(int32_t max_n);

/* ---- launch-parameter tuning -------------------------------------------- */

/* Two launch parameters are free and never change a result: the tile events
 * each block of the merge handles (op WRS_TUNE_BUILD: 4, 8, 16 or 32) and the
 * draws per sampler thread (op WRS_TUNE_SAMPLE: 1, 2, 4 or 8).  Tables and
 * samples are bit-identical for every value; only speed differs.  A value is
 * kept per device kind (architecture name and CU count) and size class:
 * ceil(log2 n) for the build, ceil(log2 k) for the sampler.  A class without
 * an entry uses a default derived from the size and the CU count.  At first
 * use the library reads the JSON file named by the environment variable
 * WRS_TUNE_FILE, if set.  The tables are per process and thread-safe. */
enum { WRS_TUNE_BUILD = 1, WRS_TUNE_SAMPLE = 2 };

/* Value in effect on the current device for `size` (n or k >= 1). */
int wrs_tune_get(int op, int64_t size, int32_t* value);

/* Set the value for the size class of `size` on the current device; 0 removes
 * the entry (back to the default).  WRS_EINVAL for a value not listed above. */
int wrs_tune_set(int op, int64_t size, int32_t value);

/* Time every candidate on the current device and keep the fastest for the
 * size class: WRS_TUNE_BUILD builds a table of n synthetic uniform weights,
 * WRS_TUNE_SAMPLE draws k samples from such a table of n items.  Allocates
 * and frees device memory (about 17 n + 4 k bytes) and synchronises `stream`;
 * not for use inside stream capture.  *best (optional) receives the winner. */
int wrs_autotune(int op, int64_t n, int64_t k, void* stream, int32_t* best);

/* Write every entry to a JSON file, or merge the entries of such a file
 * (entries for other devices are kept but not used on this one). */
int wrs_tune_save(const char* path);
int wrs_tune_load(const char* path);

/* ---- serving -------------------------------------------------------------- */

/* A request loop on one device: build requests create resident tables, sample
 * requests draw from them.  Admission is limited by an HBM budget; admitted
 * requests are packed into batched launches while earlier batches are still
 * running (continuous batching), or issued one launch per request in arrival
 * order when `one_at_a_time` is set (the baseline).
 * wrs_serve_create reserves the whole budget as one device allocation and,
 * per concurrent batch, descriptor buffers for max_batch requests (device
 * memory from the budget and pinned host memory), plus a pinned staging arena
 * of host_stage_bytes for builds from host weights; requests allocate nothing
 * outside these.  Idle tables are evicted, least recently used first, to
 * admit a build.  A build that cannot be admitted while nothing runs and no
 * table is idle (the budget is held by tables that requests queued behind it
 * still need) fails with WRS_ENOMEM rather than wait for ever; so do draws
 * from its table.  A batch whose launch fails fails all its requests with
 * WRS_EDEVICE.  Every address a served request's kernels write is fixed by its
 * sizes (table entry i < n, draw s < k), never by the weights' values.
 *
 * Ordering with the caller: each submit takes the caller's stream, a
 * hipStream_t of the server's device; NULL is the legacy default stream (the
 * stream of frameworks that have not set one) and is ordered like any other.
 * The server records an event on that stream during the call, and the
 * request's batch waits for that event on the device before it reads the
 * request's weights or writes its outputs: everything the caller queued on
 * that stream before the submit (producing the weights, a previous reader of
 * the output buffer, a deallocation and reuse of the buffer's memory by a
 * caching allocator) runs first.  WRS_SERVE_UNORDERED instead of a stream
 * skips the event: the caller must have completed that work already (for
 * instance with a device synchronisation).  Completion is reported on the host
 * (wrs_serve_poll, wrs_serve_wait); a result may be read on any stream after
 * that. */
#define WRS_SERVE_UNORDERED ((void*)(intptr_t)-1)
#define WRS_SERVE_MAX_BATCH 4096
#define WRS_SERVE_MAX_INFLIGHT 16
typedef struct {
    size_t hbm_budget_bytes;   /* tables + per-request workspace + descriptors, bytes (>= 1 MiB) */
    int32_t max_batch;         /* requests per batched launch, 1..WRS_SERVE_MAX_BATCH */
    int32_t one_at_a_time;     /* 0: continuous batching, 1: one launch per request, FIFO */
    int32_t inflight;          /* batches that may run concurrently, 1..WRS_SERVE_MAX_INFLIGHT */
    int32_t pad;
    size_t host_stage_bytes;   /* pinned staging for host weights (0: device weights only) */
} wrs_serve_config;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t builds, samples;
    uint64_t items_built, samples_drawn;
    uint64_t launches;              /* batched launches issued */
    double p50_us, p99_us, max_us;  /* completion - submission latency */
    double busy_s;                  /* first submission to last completion */
    size_t bytes_in_use, bytes_peak;
    uint64_t tables_resident;
} wrs_serve_stats_t;

int wrs_serve_create(const wrs_serve_config* cfg, void** srv);
/* Build request over n weights (problem statement of Section 1; the table is
 * wrs_alias_build's).  w_on_host = 0: w is a device pointer that must stay
 * valid until the request completes.  w_on_host = 1: w is host memory; the
 * call copies the n weights into the staging arena (waiting, if the arena is
 * full, for running requests to retire; WRS_ENOMEM if 4 n bytes exceed the
 * arena) and w is free again when it returns; the server copies them to the
 * device on the batch's stream.  stream: see "Ordering with the caller".
 * *table_id names the resident table. */
int wrs_serve_submit_build(void* srv, const float* w, int64_t n, int32_t w_on_host, void* stream,
                           uint64_t* table_id, uint64_t* req);
/* Sample request: k draws from a resident table (seed, stream_id 0, counters
 * 0..k-1) into the device buffer d_out (k int32).  The table may still be
 * under construction; the request then runs after it.  stream: see
 * "Ordering with the caller". */
int wrs_serve_submit_sample(void* srv, uint64_t table_id, int64_t k, uint64_t seed, int32_t* d_out,
                            void* stream, uint64_t* req);
int wrs_serve_poll(void* srv, uint64_t req, int* done, int* status);
int wrs_serve_wait(void* srv, uint64_t req, int* status);
/* Submission and completion times of a finished request, in seconds of the
 * host's steady clock (the clock of wrs_serve_stats' latencies); WRS_EBUSY
 * while it runs.  For latency statistics over a chosen part of a request
 * stream (for instance after a warm-up). */
int wrs_serve_request_times(void* srv, uint64_t req, double* submit_s, double* done_s);
/* Drop a table once no pending request uses it (WRS_EBUSY otherwise). */
int wrs_serve_release_table(void* srv, uint64_t table_id);
/* Read a table back into host memory (n entries), e.g. to compare results. */
int wrs_serve_read_table(void* srv, uint64_t table_id, wrs_entry* h_table, int64_t n);
int wrs_serve_stats(void* srv, wrs_serve_stats_t* out);
int wrs_serve_destroy(void* srv);

/* Text of the last error on this thread ("" if none).  The request server's
 * worker runs on a thread of its own: its failures reach the caller as
 * request statuses (wrs_serve_wait, wrs_serve_poll), not through this text. */
const char* wrs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WRS_H */
