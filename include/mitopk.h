/* mitopk — key-only Top-K selection on MI355X (gfx950).
 *
 * The ordering primitive of "GPU-Augmented OLAP Execution Engine: GPU
 * Offloading" (arXiv 2601.19911): sec. III-A defines LIMIT-based Top-K as
 * key-only transfer, partial or radix-based selection on the GPU, and a return
 * of the Top-K pointers; sec. II-C states the key-only contract (only (Key,
 * Pointer(RowID)) pairs cross to the device, the device returns only sorted
 * pointers, the host late-materializes the few returned rows); sec. V-B gives
 * the query template ORDER BY value DESC LIMIT 100.
 *
 * Result definition (every entry point computes exactly this):
 *   pair a comes before pair b
 *     TK_DESC: key_a > key_b, or key_a == key_b and rowid_a < rowid_b
 *     TK_ASC:  key_a < key_b, or key_a == key_b and rowid_a < rowid_b
 *   with numeric order for int32/int64 keys and IEEE 754-2019 totalOrder
 *   (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN) for float32 and
 *   float64 keys (float64 is the key type of the paper's workload, sec. V-A).
 *   The output is the first K_eff = min(k, n) pairs in that order, best
 *   first: out_keys[j] holds the original key bits, out_rowids[j] its row-id.
 *
 * Conventions for all calls:
 *   - Keys and row-ids are separate arrays (structure of arrays).  rowids may
 *     be NULL: row-id i is then the index i (for rid type u32, n <= 2^32).
 *   - Device pointers are plain HIP device (or host-mapped) addresses; the
 *     caller owns every buffer: inputs, outputs and workspace.  The library
 *     owns only its opaque objects (tk_plan, tk_server).
 *   - Stream-ordered and asynchronous: tk_topk enqueues work on `stream`
 *     (a hipStream_t, NULL = the default stream) and returns without waiting.
 *     Outputs are valid once the stream has reached that point.
 *   - Errors: argument errors are returned at once (negative tk_status_t) and
 *     nothing is enqueued.  Failures found on the device afterwards (which
 *     correct use never produces) are kept in the workspace and reported by
 *     tk_query_info after the stream is synchronized.
 *   - Reentrant when calls use distinct workspaces.
 */
#ifndef MITOPK_H
#define MITOPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { TK_KEY_I32 = 0, TK_KEY_I64 = 1, TK_KEY_F32 = 2, TK_KEY_F64 = 3 } tk_key_t;
typedef enum { TK_RID_U32 = 0, TK_RID_U64 = 1 } tk_rid_t;
typedef enum { TK_DESC = 0, TK_ASC = 1 } tk_order_t;

typedef enum {
  TK_OK = 0,
  TK_EINVAL = -1,        /* bad argument: null pointer with n > 0, bad enum, small workspace */
  TK_ENOMEM = -2,        /* host allocation failed */
  TK_EHIP = -3,          /* a HIP runtime call failed */
  TK_EUNSUPPORTED = -4,  /* no usable gfx950 device, or a size beyond the limits */
  TK_EDEVICE = -5,       /* the device reported a failure (see tk_query_info) */
  TK_EAGAIN = 1          /* not finished yet (serving poll) */
} tk_status_t;

/* Bytes of device workspace tk_topk needs for a query of n keys and limit k
 * (any k; it is capped at n).  Depends only on (n, min(k, n), key type,
 * row-id type) and the current tuning.  Never 0.  For a query with no usable
 * sample from 2^16 keys (path 9) it includes the full sort's scratch, about
 * 2 n (key + row-id) bytes. */
size_t tk_workspace_size(uint64_t n, uint64_t k, int key_type, int rid_type);
/* The least workspace tk_topk accepts for the same query: tk_workspace_size
 * without the full sort's scratch.  With less than tk_workspace_size (and at
 * least this), a query with no usable sample takes path 5 instead of 9; the
 * result is the same.  Never 0. */
size_t tk_workspace_min_size(uint64_t n, uint64_t k, int key_type, int rid_type);

/* One Top-K query (paper sec. III-A): selects the best min(k, n) (key,
 * row-id) pairs and writes them best first.
 *   keys        device array of n keys (int32, int64, float32 or float64 bits)
 *   rowids      device array of n row-ids of rid_type, or NULL (row-id = index)
 *   out_keys    device array of >= min(k, n) keys, or NULL (row-ids only)
 *   out_rowids  device array of >= min(k, n) row-ids of rid_type, or NULL
 *   out_count   host pointer, set to min(k, n) before return (may be NULL)
 *   workspace   device buffer of >= tk_workspace_size(...) bytes, 256-byte
 *               aligned, scratch until the stream passes the call.  Needs no
 *               initialization: every query sets up the state it reads
 *   stream      hipStream_t (NULL: default stream)
 * k = 0 or n = 0 is valid and enqueues nothing.  Returns TK_OK or an error. */
int tk_topk(const void* keys, const void* rowids, uint64_t n, uint64_t k, int key_type,
            int rid_type, int order, void* out_keys, void* out_rowids, uint64_t* out_count,
            void* workspace, size_t workspace_bytes, void* stream);

/* Allocation-free tk_topk, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and asynchrony as tk_topk, without the
 * workspace: the query's workspace is a library-owned device array of
 * TK_NOALLOC_SCRATCH_BYTES, one per device, held from the library's load until
 * the process ends.  The call allocates nothing.  A query that does not fit
 * the array (K of a few hundred thousand and up; every K <= 100000 fits at any
 * N <= 2^30) returns TK_EUNSUPPORTED and enqueues nothing; a query with no
 * usable sample whose full-sort scratch does not fit takes path 5 instead of
 * path 9.  Every call on one device shares that device's array: two calls
 * whose work may overlap on one device (different streams without ordering
 * between them, different host threads) race and may return wrong results;
 * order them on one stream.  The array's contents are left from the last
 * call; each query sets up every word it reads. */
#define TK_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int tk_topk_noalloc(const void* keys, const void* rowids, uint64_t n, uint64_t k, int key_type,
                    int rid_type, int order, void* out_keys, void* out_rowids, uint64_t* out_count,
                    void* stream);

/* What the device did for the last tk_topk that used `workspace`.  Copies a
 * few words from the device synchronously; call after the stream has passed
 * the query. */
typedef struct {
  uint32_t path;        /* 2 sampled: streaming filter, then one workgroup's select +
                           sort of the survivors; 3 sampled: streaming filter, then the
                           survivors ranked across workgroups; 6 sampled, large K:
                           survivors grouped by bucket, each hot bucket sorted in LDS;
                           7 a small query (N within one LDS tile) ranked across
                           workgroups over the whole input;
                           4 sampled, but the sample misjudged: exact select
                           over the input (by the whole device from 2^29 keys,
                           see tk_tuning.recover_min_log2; by one workgroup
                           below); queries with no usable sample (N below 2^15,
                           K above N / 2, or K above N / 16 with N above 2^20):
                           8 exact radix select over the input by one workgroup,
                           below 2^16 keys; 9 from 2^16 keys, the full radix
                           sort of the input (as tk_sort) writing its first K
                           pairs; 5 exact radix select over the input by a
                           cooperative grid, where the workspace has no room for
                           the sort's scratch (or with tk_tuning.force_exact);
                           0 after a one-workgroup query (N within one LDS tile,
                           K > 2048) */
  uint32_t status;      /* 0, or device failure bits (1: a grid barrier timed out,
                           2: a wait between engine items timed out) */
  uint64_t survivors;   /* keys that passed the sampled threshold (paths 2-4, 6) */
  uint64_t threshold_key;  /* sampled threshold, order-preserving key image */
} tk_info;
int tk_query_info(const void* workspace, tk_info* info);

/* Process-wide tuning and test knobs; values <= 0 leave a field unchanged.
 * Not thread-safe against concurrent tk_topk calls. */
typedef struct {
  double sample_sigma;       /* margin of the sampled threshold (std devs), default 4: the
                                sample misjudges (fewer than K keys pass) with probability
                                below 2e-5 for any K at N = 2^28 on random keys */
  double cap_sigma;          /* survivor capacity margin (std devs), default 6 */
  int32_t max_sample_log2;   /* largest sample, default 20 */
  int32_t filter_grid;       /* workgroups of the streaming pass (< 0: back to the default,
                                3 per CU) */
  int64_t force_cap;         /* > 0: fixed survivor capacity (forces the fallback) */
  int32_t force_exact;       /* 1: always the exact radix select, 2: back to default */
  int32_t tail_mode;         /* 1: the survivors are ranked across workgroups when they fit
                                (default), 2: one workgroup selects and sorts them */
  int32_t filter_unroll;     /* 16-byte loads in flight per thread in the streaming pass:
                                4 or 8 (others leave it unchanged) */
  int32_t recover_min_log2;  /* sampled queries of at least 2^this keys (default 29) enqueue a
                                cooperative exact select over the device, which returns at
                                once unless the sample misjudged (the launch itself costs
                                about 21 us per query); smaller ones (or all, when < 0) fall
                                back to one workgroup's select over the input */
  int32_t join_bloom;        /* 1: join tables are built with the bloom prefilter (default),
                                2: without (tables built before keep theirs) */
} tk_tuning;
int tk_set_tuning(const tk_tuning* t);

/* ---- Batched form ----------------------------------------------------------------------------
 * Q independent Top-K queries over one packed device key buffer: query i
 * covers keys[offsets[i] .. offsets[i+1]) with its own k[i] and order[i]
 * (0 descending, 1 ascending).  Row-ids are the local index inside the query
 * when rowids is NULL at launch, else rowids[offsets[i] + j].  Results are
 * packed: query i's min(k[i], n_i) results start at element out_offsets[i]
 * (exclusive prefix sum, see tk_plan_output_offsets).  The plan classifies
 * every query: the sampled path (sample, streaming filter, tail over the
 * survivors), or, for queries too small for a sample or whose K is a large
 * share of N, one workgroup's radix select over the query.  A launch is four
 * kernels over all queries (sample workgroups, one threshold workgroup per
 * sampled query, filter workgroups, one tail workgroup per query); from the
 * second launch with the same pointers and stream they are replayed from a
 * captured hipGraph.  A one-thread kernel before them stamps the launch's
 * start and every tail workgroup its query's end (tk_plan_query_times).
 * Results equal tk_topk on each query alone. */
typedef struct tk_plan tk_plan;
typedef struct {
  uint32_t tile_keys;        /* keys each filter workgroup streams; 0: 32768 (>= 4096) */
  uint32_t filter_grid;      /* filter workgroups, each looping over the slices (the next
                                slice's record prefetched); 0: three per CU; 0xFFFFFFFF (any
                                count >= the slices): one per slice */
  uint32_t min_sample_log2;  /* smallest sample; queries under 16x it take the exact select; 0: 12 */
  uint32_t max_sample_log2;  /* largest sample; 0: 14 */
  double sample_sigma;       /* margin of the sampled threshold; 0: the process default (4) */
  int32_t use_graph;         /* >= 0: capture launches on a created stream in a hipGraph and
                                replay it (the default stream is never captured: launches
                                there are direct); < 0: always launch directly */
  double cap_sigma;          /* survivor capacity margin (std devs); 0: the process tuning's
                                (default 6) */
} tk_plan_params;

/* Workspace bytes for a plan (0 on invalid arguments).  Host arrays:
 * offsets[q+1] (non-decreasing), ks[q], orders[q].  params may be NULL. */
size_t tk_plan_workspace_size(const uint64_t* offsets, const uint32_t* ks, const uint8_t* orders,
                              uint32_t q, int key_type, int rid_type, const tk_plan_params* params);
/* Creates a plan bound to `workspace` (device, 256-byte aligned, at least
 * tk_plan_workspace_size bytes, needing no initialization, owned by the
 * caller and reserved for the plan until tk_plan_destroy).  *plan receives an
 * object owned by the library, which also holds a pinned host staging buffer
 * of the plan's argument records.  Enqueues nothing. */
int tk_plan_create(const uint64_t* offsets, const uint32_t* ks, const uint8_t* orders, uint32_t q,
                   int key_type, int rid_type, const tk_plan_params* params, void* workspace,
                   size_t workspace_bytes, tk_plan** plan);
/* out_offsets[q+1]: where each query's results start in the packed outputs. */
int tk_plan_output_offsets(const tk_plan* plan, uint64_t* out_offsets);
/* Queries on the sampled route, queries on the whole-input route, and the
 * workgroups of one launch (sample + filter + tail). */
int tk_plan_info(const tk_plan* plan, uint32_t* n_sampled, uint32_t* n_exact, uint32_t* n_items);
/* Runs every query of the plan on `stream` (asynchronous).  keys: the packed
 * device key buffer; rowids: packed row-ids or NULL; out_keys/out_rowids:
 * packed outputs (out_keys may be NULL).  When the pointer set differs from
 * the previous launch, the per-query argument records are uploaded first, by
 * an asynchronous copy on `stream` from the plan's pinned staging (the host
 * waits only if the previous upload's copy has not yet run).  Calls on one
 * plan must not overlap. */
int tk_plan_launch(tk_plan* plan, const void* keys, const void* rowids, void* out_keys,
                   void* out_rowids, void* stream);
/* Per-query completion times of the last launch: seconds[i] is the time from
 * the launch's start (a stamp its first kernel writes) to the end of query i's
 * tail workgroup, both read from the device's constant-rate clock (0 for a
 * query with min(k, n) = 0).  Every query's tail writes its stamp in every
 * launch, replays included.  Synchronous copy of q + 1 words; call after the
 * launch's stream has been synchronized.  TK_EINVAL before the first launch. */
int tk_plan_query_times(const tk_plan* plan, double* seconds);
/* After a launch has finished: sampled queries whose sample misjudged (the
 * tail selected over the whole input instead), and sampled queries with no
 * recorded path (must be 0).  Synchronous copy of the 64-byte query states. */
int tk_plan_stats(const tk_plan* plan, uint32_t* fallbacks, uint32_t* unfinished);
void tk_plan_destroy(tk_plan* plan);

/* The per-query baseline of the batched form: every query of a plan's
 * description run as its own tk_topk, enqueued from C in query order,
 * round robin over `nstreams` streams; results packed as by a plan
 * (tk_plan_output_offsets).  workspace: nstreams x
 * tk_topk_each_workspace_size bytes (256-byte aligned), stream s using slice
 * s.  With `seconds` (q entries) the call also records an event after every
 * query and a start event that every stream waits for, waits for them all,
 * and returns each query's completion time from that start; without it the
 * call is asynchronous.  TK_EINVAL on a bad argument. */
size_t tk_topk_each_workspace_size(const uint64_t* offsets, const uint32_t* ks, uint32_t q,
                                   int key_type, int rid_type);
int tk_topk_each(const void* keys, const void* rowids, const uint64_t* offsets, const uint32_t* ks,
                 const uint8_t* orders, uint32_t q, int key_type, int rid_type, void* out_keys,
                 void* out_rowids, void* workspace, size_t workspace_bytes, void* const* streams,
                 uint32_t nstreams, double* seconds);

/* ---- Served form -----------------------------------------------------------------------------
 * Continuous batching of Top-K requests over key columns with the cost gate
 * of the paper (sec. II-B): a request is offloaded only when the estimated
 * CPU cost exceeds the estimated GPU cost (transfer + kernel + result return)
 * by more than a margin; otherwise it runs on the host CPU path over the
 * column's host copy.  The gate's signals are the paper's: N (rows), K (the
 * limit, capped at N), the bytes B a GPU route must move over the host link
 * (N x key bytes for a host-resident column, 0 for a device-resident one) and
 * the estimated CPU cost.  A batcher thread forms micro-batches of one key
 * type whenever one of `slots` stream slots is free, admitting requests while
 * the slot's arena, staging and result buffers have room; batches on
 * different slots overlap on the device.  Row-ids are the global row index
 * in the column (uint64).  Every result equals tk_topk on the same keys,
 * whichever route and batch it took. */
typedef struct tk_server tk_server;
/* Cost model of one key type, seconds, K = min(k, N):
 *   C_cpu = cpu_a*N + cpu_b*K*log2(K+1) + cpu_c
 *   C_gpu = gpu_a*N + gpu_b*K + gpu_c  (+ B / h2d_bytes_per_s for a host-resident column) */
typedef struct {
  double cpu_a, cpu_b, cpu_c, gpu_a, gpu_b, gpu_c;
} tk_cost_model;
typedef struct {
  uint32_t max_batch;   /* requests per micro-batch; 0: 256 */
  uint32_t slots;       /* micro-batches in flight; 0: 2 */
  double window_us;     /* wait this long for a batch to fill; 0: no wait */
  int32_t gate;         /* 0 always GPU, 1 cost gate, 2 always CPU */
  double margin_ms;     /* gate margin */
  int32_t cpu_threads;  /* CPU-route workers; 0: 4 */
  /* per key type, indexed by tk_key_t; an all-zero entry takes the library's
   * default for that type (a fit measured on MI355X, device-resident keys,
   * against the CPU route on 16 host threads) */
  tk_cost_model cost[4];
  double h2d_bytes_per_s;  /* host-to-device rate for host-resident columns; 0: 5.0e10 */
} tk_server_cfg;
typedef struct {
  uint64_t t_submit_ns, t_start_ns, t_done_ns;  /* host steady clock */
  int32_t route;   /* 0 GPU, 1 CPU */
  int32_t status;  /* TK_OK, or the request's error (TK_ENOMEM: larger than a slot
                      and no host copy to run it on the CPU) */
  uint64_t count;  /* results written */
} tk_req_info;
typedef struct {
  uint64_t submitted, completed, routed_gpu, routed_cpu, batches, batched_requests;
  uint64_t live;          /* requests the server still holds: queued, running, or
                             finished and not yet taken by tk_server_result */
  uint64_t failed;        /* requests finished with an error status */
} tk_server_counters;

/* arena: caller-owned device buffer (256-byte aligned) split among the
 * slots; it bounds how much one micro-batch may hold. */
int tk_server_create(const tk_server_cfg* cfg, void* arena, size_t arena_bytes, tk_server** server);
/* A column of n keys.  d_keys: device copy (NULL: host-resident only, the GPU
 * route then copies each request's rows into the slot's arena, and the gate
 * counts those bytes); h_keys: host copy for the CPU route (NULL: GPU only;
 * pinned memory from hipHostMalloc keeps a host-resident column's copies
 * asynchronous).  At least one of the two is required.  The caller keeps both
 * alive until tk_server_destroy. */
int tk_server_add_column(tk_server* server, const void* d_keys, const void* h_keys, uint64_t n,
                         int key_type, uint32_t* col_id);
/* Top-K of rows [offset, offset + n) of a column; returns at once. */
int tk_server_submit(tk_server* server, uint32_t col, uint64_t offset, uint64_t n, uint32_t k,
                     int order, uint64_t* req_id);
/* Copies a finished request's keys and row-ids to host memory and releases
 * the request (its id is then unknown: TK_EINVAL); TK_EAGAIN while it runs.
 * Returns the request's own status. */
int tk_server_result(tk_server* server, uint64_t req_id, void* h_keys, uint64_t* h_rowids,
                     tk_req_info* info);
/* Submits `count` requests at t_arrival_s[i] seconds after the call (an
 * open-loop arrival trace, e.g. Poisson) from the calling thread. */
int tk_server_replay(tk_server* server, uint64_t count, const double* t_arrival_s,
                     const uint32_t* cols, const uint64_t* offsets, const uint64_t* ns,
                     const uint32_t* ks, const uint8_t* orders, uint64_t* req_ids);
/* Waits until every submitted request has finished. */
int tk_server_drain(tk_server* server);
int tk_server_stats(tk_server* server, tk_server_counters* stats);
void tk_server_destroy(tk_server* server);

/* Multithreaded CPU Top-K over host arrays: the CPU route of the cost gate
 * (paper sec. II-B) with the same result definition.  nthreads <= 0 uses
 * every core in the process affinity mask.  Synchronous. */
int tk_cpu_topk(const void* keys, const void* rowids, uint64_t n, uint64_t k, int key_type,
                int rid_type, int order, void* out_keys, void* out_rowids, uint64_t* out_count,
                int nthreads);

/* Late materialization (paper sec. II-C): the caller fetches payload rows at
 * the returned row-ids.  `cols` is a row-major [ncols][n] array of float64
 * payload columns, `rowids` k row-ids (uint32 or uint64 per rid_type), `out`
 * a [ncols][k] array: out[c][j] = cols[c][rowids[j]].
 *   tk_gather_f64_host    host arrays, synchronous, nthreads host threads;
 *                         a row-id >= n returns TK_EINVAL before any write.
 *   tk_gather_f64_device  device arrays, stream-ordered and asynchronous (the
 *                         full-row comparison, whose payload already sits in
 *                         HBM); a row-id >= n yields 0.0 in its output slots.
 * k = 0 or ncols = 0 is a no-op returning TK_OK. */
int tk_gather_f64_host(const double* cols, uint32_t ncols, uint64_t n, const void* rowids,
                       int rid_type, uint64_t k, double* out, int nthreads);
int tk_gather_f64_device(const double* cols, uint32_t ncols, uint64_t n, const void* rowids,
                         int rid_type, uint64_t k, double* out, void* stream);

/* Kernel timing for roofline reports.  Between tk_profile_begin and
 * tk_profile_end, every streaming pass over the keys (the dominant kernel:
 * the filter of tk_topk, the persistent kernel of tk_plan_launch) is
 * bracketed by a HIP event pair recorded on the caller's stream, for at most
 * max_launches launches.  tk_profile_end waits for the recorded events and
 * returns the summed kernel time in milliseconds and the number of launches
 * timed.  Process-wide; for measurement, not for concurrent use. */
int tk_profile_begin(uint32_t max_launches);
int tk_profile_end(double* total_ms, uint64_t* launches);

/* Read-ceiling probe: the bandwidth the streaming pass (the HBM-bound step of
 * the selection, sec. III-A) is compared against.  Enqueues one read-only pass
 * over `buf` with 16-byte nontemporal loads and one compare per 4-byte word,
 * on wg_per_cu workgroups of 256 threads per CU striding over 16 KiB tiles;
 * each workgroup adds its count of words above 0xFFFFFFFF (always 0) to the
 * device word `sink`, so no other byte is written.  Reads the whole tiles of
 * `bytes` (rounded down to 16 KiB).  buf: device memory, 16-byte aligned;
 * sink: device uint32; 1 <= wg_per_cu <= 32.  Stream-ordered and
 * asynchronous; time it with events on `stream`.  TK_EINVAL on a bad argument. */
int tk_read_probe(const void* buf, uint64_t bytes, uint32_t wg_per_cu, void* sink, void* stream);

/* ---- Chunk-pipelined key-only streaming ------------------------------------------------------
 * Top-K over a key column left in host memory (paper sec. II-C: only keys and
 * row-ids cross the host link; sec. IV-A: the link bounds the end-to-end
 * time).  The column is copied in chunks of `chunk` keys into two device
 * staging buffers on `copy_stream` while the previous chunk's Top-K runs on
 * `stream`; each chunk's best min(k, chunk) pairs, with their column row-ids,
 * are merged into the running result by one more Top-K over the two lists.
 * The result equals tk_topk over the whole column: the best K of the column
 * are among the union of the chunks' best K, and every step breaks ties by
 * row-id.  The device holds two chunks and a few K-sized lists, so n may
 * exceed the device memory.
 *   h_keys      host array of n keys; pinned (hipHostMalloc) for the copies to
 *               overlap the queries, pageable works but copies synchronously
 *   h_rowids    host array of n row-ids of rid_type, or NULL (row-id = column
 *               position, also across chunks)
 *   chunk       keys per chunk (0: 2^24)
 *   out_keys, out_rowids, out_count   as for tk_topk (device outputs)
 *   workspace   device buffer of >= tk_stream_workspace_size bytes, 256-byte
 *               aligned, needing no initialization
 *   stream      compute stream; copy_stream: the stream of the copies (NULL:
 *               the compute stream, no overlap).  The copies wait for the work
 *               enqueued on `stream` before the call; the outputs are valid
 *               once `stream` passes the call, and the host arrays must stay
 *               unchanged until then.
 * Stream-ordered and asynchronous.  TK_EINVAL on a bad argument (nothing
 * enqueued); TK_EHIP if a runtime call fails part-way (the outputs are then
 * undefined). */
size_t tk_stream_workspace_size(uint64_t n, uint64_t k, uint64_t chunk, int key_type, int rid_type,
                                int with_rowids);
int tk_topk_stream(const void* h_keys, const void* h_rowids, uint64_t n, uint64_t k, int key_type,
                   int rid_type, int order, uint64_t chunk, void* out_keys, void* out_rowids,
                   uint64_t* out_count, void* workspace, size_t workspace_bytes, void* stream,
                   void* copy_stream);

/* ---- Full sort: ORDER BY key without LIMIT ---------------------------------------------------
 * The query template of sec. V-B with K = N: every pair, in the order every
 * Top-K call uses (key descending or ascending, equal keys by ascending
 * row-id), written as out_keys[0..n) / out_rowids[0..n).  The result equals
 * tk_topk with k = n.  Least-significant-digit radix sort on 8-bit digits of the
 * order-preserving key image: 4 passes for 32-bit keys, 8 for 64-bit, plus one
 * per row-id byte when explicit row-ids are given (their order then decides
 * ties; with rowids == NULL the input order is the row-id order).  Each pass
 * reads and writes every pair once more; nothing waits across workgroups. */
/* Device workspace bytes for n pairs (0 on a bad type): two ping-pong copies of
 * the keys and row-ids, and 1 KiB of digit counts per 4096 pairs. */
size_t tk_sort_workspace_size(uint64_t n, int key_type, int rid_type);
/* keys: n device keys; rowids: n device row-ids of rid_type or NULL (row-id =
 * position); out_keys: n keys or NULL; out_rowids: n row-ids of rid_type
 * (required); workspace: >= tk_sort_workspace_size bytes, 256-byte aligned,
 * scratch until the stream passes the call.  Inputs and outputs must not
 * overlap the workspace.  Stream-ordered and asynchronous; n = 0 enqueues
 * nothing.  TK_EINVAL on a bad argument, TK_EUNSUPPORTED for n >= 2^32 (the
 * digit counts are 32-bit); nothing enqueued on an error. */
int tk_sort(const void* keys, const void* rowids, uint64_t n, int key_type, int rid_type,
            int order, void* out_keys, void* out_rowids, void* workspace, size_t workspace_bytes,
            void* stream);

/* ---- Matching primitive: key-only hash-join probe (paper sec. III-B) ---------------------
 * The probe phase of an inner equi-join done key-only, as sec. III-B states it:
 * the build side's (key, row-id) pairs go into a device hash table, the probe
 * keys are looked up in parallel, and only matched pointers come back (sec.
 * II-C, "Processing"); the host late-materializes the rows.  The result is the
 * multiset of pairs (probe row-id, build row-id) with probe_key == build_key,
 * one per equal (probe row, build row), returned in no particular order.  Keys
 * are int32 or int64 and compare by numeric equality (float keys:
 * TK_EUNSUPPORTED).  Row-ids may be NULL on either side (row-id = position).
 *
 * The table lives in a caller-owned device buffer; tk_join_table describes it
 * (a plain struct the caller keeps; the library allocates nothing).  One build
 * serves any number of probes, concurrent ones included, while the buffer
 * stays untouched. */
typedef struct {
  void* table;           /* the device buffer given to tk_join_build */
  uint64_t table_bytes;  /* its size */
  uint64_t n_build;      /* build pairs */
  uint64_t slots;        /* hash slots: a power of two >= 2 * n_build (load <= 1/2) */
  int32_t key_type;      /* TK_KEY_I32 or TK_KEY_I64 */
  int32_t rid_type;      /* build row-id type, also the type of out_build_rowids */
  uint64_t bloom_words;  /* 64-bit words of the bloom prefilter (slots / 16), or 0 when the
                            table was built without it (tk_tuning.join_bloom); probes read
                            a key's word first and skip the slots when it rules the key out */
} tk_join_table;

/* Device bytes of the table for n_build pairs (0 on a bad type or n_build > 2^31):
 * a 256-byte header, the slots (8 bytes each for int32 keys with uint32 row-ids,
 * 16 bytes otherwise), room for n_build row-ids, the bloom prefilter's
 * slots / 2 bytes (reserved whether or not the build fills it) and an 8 KiB
 * filter of the build keys that occur more than once. */
size_t tk_join_table_size(uint64_t n_build, int key_type, int rid_type);
/* Builds the table from n_build build pairs (stream-ordered, asynchronous).
 *   keys     device array of n_build int32/int64 keys
 *   rowids   device array of n_build row-ids of rid_type, or NULL (row-id = position)
 *   table    device buffer of >= tk_join_table_size bytes, 256-byte aligned, needing
 *            no initialization (the build clears it); reserved until the last probe
 *            that reads it has run
 *   out      host descriptor, filled before return
 * TK_EUNSUPPORTED for float keys or n_build > 2^31; TK_EINVAL for other bad
 * arguments (nothing is enqueued then). */
int tk_join_build(const void* keys, const void* rowids, uint64_t n_build, int key_type,
                  int rid_type, void* table, size_t table_bytes, tk_join_table* out, void* stream);
/* Probes the table with n_probe keys (of the table's key type); stream-ordered,
 * asynchronous.
 *   rowids            device array of n_probe probe row-ids of rid_type, or NULL
 *   out_probe_rowids  device array of `capacity` rid_type row-ids
 *   out_build_rowids  device array of `capacity` row-ids of the table's rid_type
 *   capacity          pairs the outputs hold (0: count only; the outputs may be NULL)
 *   d_count           device uint64, set to the number of matched pairs M once the
 *                     stream passes the call (the library zeroes it first)
 * min(M, capacity) pairs are written; when M > capacity the written ones are
 * an arbitrary subset and the caller probes again with capacity >= M.  Returns
 * TK_OK or TK_EINVAL (nothing enqueued). */
int tk_join_probe(const tk_join_table* table, const void* keys, const void* rowids,
                  uint64_t n_probe, int rid_type, void* out_probe_rowids, void* out_build_rowids,
                  uint64_t capacity, uint64_t* d_count, void* stream);

/* Human-readable name of a tk_status_t value. */
const char* tk_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* MITOPK_H */
